"""Host-side tests of libgaca (no GPU): the library loads and exports every symbol the
header declares, the host tree/partition equals the oracle's, the library's own
quadrature tables are exact, and invalid meshes are rejected."""
import ctypes
import os
import re

import numpy as np
import pytest

from inputs import cube_mesh, icosphere_mesh, lshape_mesh
import paper_2312_11219_amd as gaca
from paper_2312_11219_amd._binding import GacaError, quadrature_rule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "gaca.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gaca_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    lib = gaca.load_library()
    syms = _header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    ver = int(re.search(r"#define GACA_ABI_VERSION (\d+)", open(os.path.join(ROOT, "include", "gaca.h")).read()).group(1))
    assert lib.gaca_abi_version() == ver


def test_no_gpu_context_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(GacaError) as e:
        gaca.Context(0)
    assert e.value.code == -4   # GACA_ERR_STATE


def test_options_default():
    o = gaca.options_default()
    assert o.leaf_size == 32 and o.eta == 1.0 and o.n_duffy == 16
    assert o.tie == 1e-9 and o.delta_zero == 1e-13
    o2 = gaca.options_default(leaf_size=16, precision="mixed")
    assert o2.leaf_size == 16 and o2.precision == 1


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 10, 16, 40])
def test_library_gauss_legendre(n):
    x, w = quadrature_rule("gauss", n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, 0.5 * (xr + 1), atol=2e-15, rtol=0)
    assert np.allclose(w, 0.5 * wr, atol=2e-15, rtol=0)
    for d in range(2 * n):
        assert abs(np.sum(w * x ** d) - 1.0 / (d + 1)) < 1e-14


def test_library_triangle6():
    from math import factorial
    b, w = quadrature_rule("triangle6", 6)
    assert abs(w.sum() - 1) < 1e-15
    for deg in range(5):
        for a in range(deg + 1):
            c = deg - a
            approx = 0.5 * np.sum(w * b[:, 1] ** a * b[:, 2] ** c)
            exact = factorial(a) * factorial(c) / factorial(a + c + 2)
            assert abs(approx - exact) < 1e-15
    assert abs(w[0] - 0.223381589678011) < 1e-14
    assert abs(b[1, 0] - 0.445948490915965) < 1e-14


MESHES = [("cube4", cube_mesh(4), 16, 1.0), ("cube4-l4", cube_mesh(4), 4, 1.0),
          ("cube8", cube_mesh(8), 16, 1.0), ("cube16", cube_mesh(16), 32, 1.0),
          ("lshape8", lshape_mesh(8), 32, 1.0), ("ico4", icosphere_mesh(4), 32, 1.0),
          ("cube8-eta2", cube_mesh(8), 16, 2.0)]


@pytest.mark.parametrize("name,mesh,leaf,eta", MESHES, ids=[m[0] for m in MESHES])
def test_partition_equals_oracle(name, mesh, leaf, eta):
    from oracle import tree as T
    xyz, tri = mesh
    perm, far, near = gaca.partition_host(xyz, tri, leaf, eta)
    operm, root = T.build_tree(xyz, tri, leaf)
    ofar, onear = T.build_partition(root, eta)
    assert np.array_equal(perm, operm)
    assert np.array_equal(far, np.array(ofar, dtype=np.int64).reshape(-1, 4))
    assert np.array_equal(near, np.array(onear, dtype=np.int64).reshape(-1, 4))


def test_invalid_meshes_rejected():
    xyz, tri = cube_mesh(2)
    bad = tri.copy()
    bad[0, 1] = bad[0, 0]          # degenerate triangle
    with pytest.raises(GacaError) as e:
        gaca.partition_host(xyz, bad, 8, 1.0)
    assert e.value.code == -1
    bad = tri.copy()
    bad[3, 2] = xyz.shape[0]       # vertex id out of range
    with pytest.raises(GacaError):
        gaca.partition_host(xyz, bad, 8, 1.0)
    x2 = xyz.copy()
    x2[5, 1] = np.nan
    with pytest.raises(GacaError):
        gaca.partition_host(x2, tri, 8, 1.0)
    with pytest.raises(GacaError):
        gaca.partition_host(xyz, tri, 0, 1.0)


@pytest.mark.parametrize("mesh,leaf", [("cube8", 16), ("sphere3", 16), ("lshape2", 8)])
def test_p1_partition_matches_oracle(mesh, leaf):
    """Vertex tree and partition of the P1 double layer: identical to the oracle's."""
    from inputs import cube_mesh, icosphere_mesh, lshape_mesh
    from oracle.tree import build_partition, build_tree_p1
    import paper_2312_11219_amd as gaca
    xyz, tri = {"cube8": lambda: cube_mesh(8), "sphere3": lambda: icosphere_mesh(3),
                "lshape2": lambda: lshape_mesh(2)}[mesh]()
    perm, far, near = gaca.partition_host(xyz, tri, leaf, 1.0, scheme="p1")
    operm, root = build_tree_p1(xyz, tri, leaf)
    ofar, onear = build_partition(root, 1.0)
    assert np.array_equal(perm, operm)
    assert np.array_equal(far, np.array(ofar, dtype=np.int64).reshape(-1, 4))
    assert np.array_equal(near, np.array(onear, dtype=np.int64).reshape(-1, 4))
