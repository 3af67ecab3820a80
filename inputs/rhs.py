"""Seeded random complex right-hand sides X[l][i][b] = N(0,1) + i N(0,1)."""
from __future__ import annotations

import numpy as np


def random_rhs(L: int, M: int, nrhs: int, seed: int = 0, dtype=np.complex128) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((L, M, nrhs))
    im = rng.standard_normal((L, M, nrhs))
    return (re + 1j * im).astype(dtype)
