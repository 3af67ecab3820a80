"""Complex Laplace-domain frequencies on a circle in the right half plane.

The paper's gCQ contour (App. A) is only partly legible, so the workloads use circles
s_l = c0 * (1 + rho * exp(2 pi i (l + 1/2) / L)), l = 0..L-1.  The circle is symmetric
about the real axis, so s_{L-1-l} is the complex conjugate of s_l; the generator
computes the upper half and writes the mirror as an exact conjugate (App. A notes that
only half of a real-symmetric contour needs computing).
"""
from __future__ import annotations

import numpy as np


def circle_frequencies(L: int, c0: float, rho: float) -> np.ndarray:
    if L < 1:
        raise ValueError("L must be >= 1")
    s = np.empty(L, dtype=np.complex128)
    half = (L + 1) // 2
    for l in range(half):
        theta = 2.0 * np.pi * (l + 0.5) / L
        s[l] = c0 * (1.0 + rho * np.cos(theta)) + 1j * (c0 * rho * np.sin(theta))
    for l in range(half, L):
        s[l] = np.conj(s[L - 1 - l])
    if L % 2 == 1:
        # the middle point sits on the real axis
        m = L // 2
        s[m] = complex(s[m].real, 0.0)
    return s
