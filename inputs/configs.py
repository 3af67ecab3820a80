"""The five named workloads: meshes, frequency circles and tolerances.

C1  cube 4x4 squares per face (192 triangles), collocation, single layer, L=16,
    s_l = 10 (1 + 0.9 e^{i theta_l}), leaf 16, eta 1, eps 1e-4, FP64.
C2  cube 16x16 per face (3072), collocation, single + double layer, L=64,
    s_l = 20 (1 + 0.95 e^{i theta_l}), leaf 32, eta 1, eps 1e-6, FP64.
C3  icosphere level 5 (20480), collocation, single layer, L=128,
    s_l = 40 (1 + 0.95 e^{i theta_l}), leaf 32, eps 1e-5, mixed precision.
C4  reentrant-corner cube, grid 1/32 (12288), Galerkin, single layer, L=96,
    s_l = 20 (1 + 0.95 e^{i theta_l}), leaf 32, eps 1e-5.
C5  icosphere level 6 (81920), collocation, single layer, L=256,
    s_l = 40 (1 + 0.95 e^{i theta_l}), leaf 32, eps 1e-6, apply with 256 right-hand sides.
P1  icosphere level 5 (20480 triangles, 10242 vertices), the double layer with linear
    continuous trial functions collocated at the vertices, L=128, s_l = 40 (1 + 0.95
    e^{i theta_l}), leaf 32, eps 1e-5, FP64.

The face tolerance is eps_aca = eps / 100 (the paper's choice eps = 100 eps_aca).
"""
from __future__ import annotations

CONFIGS = {
    "C1": dict(mesh=("cube", 4), M=192, L=16, c0=10.0, rho=0.9, leaf=16, eta=1.0, eps=1e-4,
               scheme="collocation", kernels=("slp",), precision="fp64", nrhs=2),
    "C2": dict(mesh=("cube", 16), M=3072, L=64, c0=20.0, rho=0.95, leaf=32, eta=1.0, eps=1e-6,
               scheme="collocation", kernels=("slp", "dlp"), precision="fp64", nrhs=2),
    "C3": dict(mesh=("icosphere", 5), M=20480, L=128, c0=40.0, rho=0.95, leaf=32, eta=1.0,
               eps=1e-5, scheme="collocation", kernels=("slp",), precision="mixed", nrhs=2),
    "C4": dict(mesh=("lshape", 16), M=12288, L=96, c0=20.0, rho=0.95, leaf=32, eta=1.0,
               eps=1e-5, scheme="galerkin", kernels=("slp",), precision="fp64", nrhs=2),
    "C5": dict(mesh=("icosphere", 6), M=81920, L=256, c0=40.0, rho=0.95, leaf=32, eta=1.0,
               eps=1e-6, scheme="collocation", kernels=("slp",), precision="mixed", nrhs=256),
    "P1": dict(mesh=("icosphere", 5), M=10242, L=128, c0=40.0, rho=0.95, leaf=32, eta=1.0,
               eps=1e-5, scheme="p1", kernels=("dlp",), precision="fp64", nrhs=2),
}


def get_config(name: str) -> dict:
    cfg = dict(CONFIGS[name])
    cfg["name"] = name
    cfg["eps_aca"] = cfg["eps"] / 100.0
    return cfg
