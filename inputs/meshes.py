"""Procedural triangle surface meshes: cube, reentrant-corner cube (L-shape) and icosphere.

The paper's examples (Sec. 5: unit cube, cube with a reentrant corner, unit ball) come
with mesh tables but no mesh files, so these generators build synthetic meshes of the
same kind.  Every mesh is closed, conforming and oriented so that each triangle's
vertices run counter-clockwise seen from outside (outward normal by the right-hand
rule), which is the orientation the double layer sign convention assumes.

Returns ``(xyz, tri)``: ``xyz`` float64 ``(nv, 3)``, ``tri`` int32 ``(M, 3)``.
"""
from __future__ import annotations

import numpy as np

# Outward unit normal, and in-face axes (u, v) with u x v = normal, for the six faces of
# an axis-aligned box.  (axis, side) with side = 0 for the low face, 1 for the high face.
_FACES = []
for _axis in range(3):
    for _side in (0, 1):
        _n = np.zeros(3, dtype=np.int64)
        _n[_axis] = 1 if _side == 1 else -1
        _a, _b = (_axis + 1) % 3, (_axis + 2) % 3
        _u = np.zeros(3, dtype=np.int64)
        _v = np.zeros(3, dtype=np.int64)
        _u[_a] = 1
        _v[_b] = 1
        if np.any(np.cross(_u, _v) != _n):
            _u, _v = _v, _u
        assert np.all(np.cross(_u, _v) == _n)
        _FACES.append((_axis, _side, _n, _u, _v))


def voxel_surface_mesh(cells, cell_size: float, sub: int, origin=(0.0, 0.0, 0.0)):
    """Boundary of a union of axis-aligned cubic cells, each exposed cell face split
    into ``sub x sub`` squares and every square cut along its local (0,0)-(1,1) diagonal.

    ``cells`` is an iterable of integer (i, j, k) cell indices.  Vertices lie on an
    integer lattice of spacing ``cell_size / sub`` and are shared between faces, so the
    mesh is conforming.
    """
    cells = {tuple(int(c) for c in cell) for cell in cells}
    lattice = {}
    verts = []
    tris = []

    def vid(p):
        key = (int(p[0]), int(p[1]), int(p[2]))
        idx = lattice.get(key)
        if idx is None:
            idx = len(verts)
            lattice[key] = idx
            verts.append(key)
        return idx

    for cell in sorted(cells):
        c = np.array(cell, dtype=np.int64)
        for axis, side, n, u, v in _FACES:
            nb = tuple(c + n)
            if nb in cells:
                continue  # interior face
            # face corner (lattice units): low corner of the cell, shifted to the high side
            base = c * sub
            base = base + (n > 0) * sub
            # the face spans u and v directions from the cell's low corner on that plane
            for a in range(sub):
                for b in range(sub):
                    p00 = base + u * a + v * b
                    p10 = p00 + u
                    p11 = p00 + u + v
                    p01 = p00 + v
                    i00, i10, i11, i01 = vid(p00), vid(p10), vid(p11), vid(p01)
                    tris.append((i00, i10, i11))
                    tris.append((i00, i11, i01))
    h = cell_size / sub
    xyz = np.asarray(verts, dtype=np.float64) * h + np.asarray(origin, dtype=np.float64)
    tri = np.asarray(tris, dtype=np.int32)
    return xyz, tri


def cube_mesh(n: int):
    """Centred cube [-0.5, 0.5]^3 (Sec. 5.1), each face n x n squares, 12 n^2 triangles."""
    return voxel_surface_mesh([(0, 0, 0)], 1.0, n, origin=(-0.5, -0.5, -0.5))


def lshape_mesh(n_half: int):
    """Unit cube [0,1]^3 with the octant [0.5,1]^3 removed (reentrant corner, Sec. 5.2).

    Each exposed half-size cell face gets ``n_half x n_half`` squares, so the grid
    spacing is 1 / (2 n_half); ``n_half = 16`` gives 12288 triangles.
    """
    cells = [(i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1) if (i, j, k) != (1, 1, 1)]
    return voxel_surface_mesh(cells, 0.5, n_half)


def icosphere_mesh(level: int):
    """Unit sphere: icosahedron, each triangle split into four ``level`` times with the
    edge midpoints projected onto the sphere.  20 * 4**level triangles."""
    t = (1.0 + np.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    xyz = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = xyz[a] + xyz[b]
                xyz.append(p / np.linalg.norm(p))
                idx = len(xyz) - 1
                cache[key] = idx
            return idx

        new = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(faces, dtype=np.int32)
    # orient counter-clockwise seen from outside (centroid direction = outward)
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return xyz, tri


def mesh_for_config(name: str):
    """Mesh of a named workload (see ``inputs.configs``)."""
    from .configs import get_config
    cfg = get_config(name)
    kind, arg = cfg["mesh"]
    if kind == "cube":
        return cube_mesh(arg)
    if kind == "lshape":
        return lshape_mesh(arg)
    if kind == "icosphere":
        return icosphere_mesh(arg)
    raise ValueError(kind)
