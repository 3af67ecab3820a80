"""Seeded synthetic workload generators shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only builds surface meshes,
the complex frequency lists and random right-hand sides that both the independent CPU
oracle and the GPU library consume as inputs.
"""
from .meshes import cube_mesh, lshape_mesh, icosphere_mesh, voxel_surface_mesh, mesh_for_config
from .frequencies import circle_frequencies
from .rhs import random_rhs
from .configs import CONFIGS, get_config

__all__ = [
    "cube_mesh", "lshape_mesh", "icosphere_mesh", "voxel_surface_mesh", "mesh_for_config",
    "circle_frequencies", "random_rhs", "CONFIGS", "get_config",
]
