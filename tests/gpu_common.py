"""Shared fixtures for GPU tests: workloads, oracle references, helpers."""
import functools
import sys

import numpy as np

from inputs import circle_frequencies, cube_mesh, get_config, mesh_for_config


def log(*args):
    print(*args, flush=True)
    sys.stdout.flush()


# Small far-field workload the oracle finishes in seconds: 768-triangle cube, leaf 16.
SMALL = dict(name="cube768", mesh=("cube", 8), L=16, c0=10.0, rho=0.9, leaf=16, eta=1.0,
             eps=1e-4, scheme="collocation")
SMALL_GAL = dict(name="lshape768", mesh=("lshape", 4), L=16, c0=10.0, rho=0.9, leaf=16,
                 eta=1.0, eps=1e-4, scheme="galerkin")
# small P1 double layer workload: the same cube, its 386 vertices as degrees of freedom
SMALL_P1 = dict(name="p1cube386", mesh=("cube", 8), L=16, c0=10.0, rho=0.9, leaf=16,
                eta=1.0, eps=1e-4, scheme="p1")
# small Galerkin P1 workload (hypersingular operator, adjoint double layer): the same cube,
# 8 frequencies, touching pairs with 6 points per variable of the regularising maps
SMALL_GP1 = dict(name="gp1cube386", mesh=("cube", 8), L=8, c0=10.0, rho=0.9, leaf=16,
                 eta=1.0, eps=1e-4, scheme="galerkin_p1", n_touch=6)


def workload(name):
    if name == "cube768":
        cfg = dict(SMALL)
        xyz, tri = cube_mesh(8)
    elif name == "p1cube386":
        cfg = dict(SMALL_P1)
        xyz, tri = cube_mesh(8)
    elif name == "gp1cube386":
        cfg = dict(SMALL_GP1)
        xyz, tri = cube_mesh(8)
    elif name == "lshape768":
        # small Galerkin workload: reentrant-corner cube, 1/8 grid (768 triangles)
        cfg = dict(SMALL_GAL)
        from inputs import lshape_mesh
        xyz, tri = lshape_mesh(4)
    else:
        cfg = get_config(name)
        xyz, tri = mesh_for_config(name)
    cfg.setdefault("eps_aca", cfg["eps"] / 100.0)
    s = circle_frequencies(cfg["L"], cfg["c0"], cfg["rho"])
    return cfg, xyz, tri, s


@functools.lru_cache(maxsize=None)
def context():
    import paper_2312_11219_amd as gaca
    return gaca.Context(0)


def gpu_problem(name, **kw):
    import paper_2312_11219_amd as gaca
    cfg, xyz, tri, s = workload(name)
    opts = dict(leaf_size=cfg["leaf"], eta=cfg["eta"], eps3d=cfg["eps"], eps_aca=cfg["eps_aca"])
    if "n_touch" in cfg:
        opts["n_touch"] = cfg["n_touch"]
    opts.update(kw)
    scheme = cfg.get("scheme", "collocation")
    return cfg, gaca.Problem(context(), xyz, tri, s, scheme=scheme, **opts), (xyz, tri, s)


def oracle_problem(name):
    from oracle.hmatrix import Problem
    cfg, xyz, tri, s = workload(name)
    return cfg, Problem(xyz, tri, s, cfg["leaf"], cfg["eta"], scheme=cfg.get("scheme", "collocation"),
                        n_touch=cfg.get("n_touch"))


def rel_fro(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def reconstruct(h, idx):
    """Dense m x n x L tensor of far block idx from its exported factors: the sum over the
    block's crosses of (U_l W_l^T) outer f_l (Sec. 4, eq. (outerProd)), in FP64 on the CPU."""
    b = h.export_block(idx)
    out = np.zeros((b["m"], b["n"], h.L), dtype=complex)
    for c in b["crosses"]:
        out += (c["U"] @ c["W"].T)[:, :, None] * c["f"][None, None, :]
    return out
