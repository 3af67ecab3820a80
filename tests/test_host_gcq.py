"""The library's gCQ integration points and weights (host code, App. A) against the oracle's
independent computation (scipy's elliptic functions), and its error paths."""
import numpy as np
import pytest

import paper_2312_11219_amd as gaca
from paper_2312_11219_amd._binding import GacaError
from oracle.gcq import IMPLICIT_EULER, RADAU_IIA_2, contour

RADAU_IIA_3 = np.array([[(88 - 7 * np.sqrt(6)) / 360, (296 - 169 * np.sqrt(6)) / 1800, (-2 + 3 * np.sqrt(6)) / 225],
                        [(296 + 169 * np.sqrt(6)) / 1800, (88 + 7 * np.sqrt(6)) / 360, (-2 - 3 * np.sqrt(6)) / 225],
                        [(16 - np.sqrt(6)) / 36, (16 + np.sqrt(6)) / 36, 1.0 / 9.0]])


@pytest.mark.parametrize("A", [IMPLICIT_EULER[0], RADAU_IIA_2[0], RADAU_IIA_3],
                         ids=["euler", "radau2", "radau3"])
@pytest.mark.parametrize("nq,dts", [(16, (0.05, 0.1)), (64, (0.001, 0.1)), (33, (0.02, 0.021))])
def test_contour_matches_oracle(A, nq, dts):
    s, w = gaca.gcq_contour(A, dts[0], dts[1], nq)
    so, wo = contour(dts[0], dts[1], A, nq)
    assert np.abs(s - so).max() <= 1e-12 * np.abs(so).max()
    assert np.abs(w - wo).max() <= 1e-12 * np.abs(wo).max()
    assert np.array_equal(s[::-1], np.conj(s)) and np.array_equal(w[::-1], np.conj(w))


def test_contour_rejects_equal_steps():
    with pytest.raises(GacaError) as e:
        gaca.gcq_contour(IMPLICIT_EULER[0], 0.1, 0.1, 8)
    assert e.value.code == -1
    with pytest.raises(GacaError):
        gaca.gcq_contour(np.zeros((2, 2)), 0.1, 0.2, 8)
