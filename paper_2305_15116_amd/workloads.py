"""Seeded synthetic macro meshes shared by the tests, the benchmark and the oracle harness.

This module only produces inputs: vertex coordinates and cell vertex lists of
macro meshes, plus the seeded random affine maps that shape them.  It holds
none of the finite-element arithmetic of the method (no stiffness, no
stencils, no refinement), so that both the HIP path and the oracle can take
their inputs from here without sharing any of the computation under test.

The workloads follow the paper's setting: unstructured triangles (or tets)
that are each uniformly refined (Intro, "Hybrid Tetrahedral Grids"); the
benchmarked case of the paper is a single macro triangle (Performance
Modeling, experiment description).
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "unit_triangle", "unit_tet", "two_triangle_square", "kuhn_cube",
    "strip_2d", "strip_3d", "random_affine", "apply_affine", "shuffle_cell_orders",
    "affine_triangle",
]


def unit_triangle():
    """Reference triangle (0,0),(1,0),(0,1); vertex 0 is the right angle."""
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    cells = np.array([[0, 1, 2]], dtype=np.int64)
    return coords, cells


def unit_tet():
    coords = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, 1]])
    cells = np.array([[0, 1, 2, 3]], dtype=np.int64)
    return coords, cells


def two_triangle_square():
    """Unit square split along the (1,0)-(0,1) diagonal.

    Cells (0,0),(1,0),(0,1) and (1,1),(0,1),(1,0): with these vertex orders the
    refined grid is the axis-aligned lattice with the anti-diagonal in every
    square, in both cells.
    """
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    cells = np.array([[0, 1, 2], [3, 2, 1]], dtype=np.int64)
    return coords, cells


_SJT_PERMS = [(0, 1, 2), (0, 2, 1), (2, 0, 1), (2, 1, 0), (1, 2, 0), (1, 0, 2)]


def _cube_vertex(offset, bits):
    return offset + np.array(bits, dtype=np.float64)


def kuhn_cube(order: str = "canonical", seed: int | None = None, n_cubes: int = 1):
    """Unit cube(s) split into 6 Kuhn tetrahedra each.

    For a permutation s of the three axes the tet is
    (0, (1,1,1), e_s1 + e_s2, e_s2) where s = (s0, s1, s2): its index-space
    lattice maps e1 - e2, e2 - e3 and e3 onto the three axes, so every macro's
    refinement is the global Kuhn grid of the cube.  ``order='random'``
    permutes the vertices of every tet with ``numpy.random.default_rng(seed)``
    (still conforming, but the refined grids are no longer the global Kuhn grid).
    Cubes are placed in a row along x; consecutive tets of one cube share a face.
    """
    corners = {}
    coords = []

    def vid(p):
        key = tuple(int(round(c)) for c in p)
        if key not in corners:
            corners[key] = len(coords)
            coords.append([float(c) for c in key])
        return corners[key]

    cells = []
    for c in range(n_cubes):
        off = np.array([float(c), 0.0, 0.0])
        for s in _SJT_PERMS:
            e = np.eye(3)
            v0 = off
            v1 = off + np.ones(3)
            v2 = off + e[s[1]] + e[s[2]]
            v3 = off + e[s[2]]
            cells.append([vid(v0), vid(v1), vid(v2), vid(v3)])
    coords = np.array(coords, dtype=np.float64)
    cells = np.array(cells, dtype=np.int64)
    if order == "random":
        cells = shuffle_cell_orders(cells, seed if seed is not None else 5)
    elif order != "canonical":
        raise ValueError(order)
    return coords, cells


def strip_2d(k: int):
    """ceil(k/2) unit squares in a row along x, each split along its (1,0)-(0,1)
    diagonal; the first k triangles."""
    if k < 1:
        raise ValueError("k >= 1")
    nsq = (k + 1) // 2
    coords = []
    for i in range(nsq + 1):
        coords.append([float(i), 0.0])
        coords.append([float(i), 1.0])
    cells = []
    for i in range(nsq):
        a, b = 2 * i, 2 * i + 1          # (i,0), (i,1)
        c, d = 2 * i + 2, 2 * i + 3      # (i+1,0), (i+1,1)
        cells.append([a, c, b])
        cells.append([d, b, c])
    cells = np.array(cells[:k], dtype=np.int64)
    used = np.unique(cells)
    remap = -np.ones(len(coords), dtype=np.int64)
    remap[used] = np.arange(len(used))
    return np.array(coords)[used], remap[cells]


def strip_3d(k: int):
    """ceil(k/6) unit cubes in a row along x, 6 Kuhn tets each; the first k."""
    if k < 1:
        raise ValueError("k >= 1")
    coords, cells = kuhn_cube(n_cubes=(k + 5) // 6)
    cells = cells[:k]
    used = np.unique(cells)
    remap = -np.ones(len(coords), dtype=np.int64)
    remap[used] = np.arange(len(used))
    return coords[used], remap[cells]


def _rotation(dim, rng):
    if dim == 2:
        t = rng.uniform(0.0, 2.0 * np.pi)
        return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_affine(dim: int, seed: int):
    """Seeded affine map x -> J x + t with J = R1 diag(sigma) R2, det J > 0,
    smallest singular value 1 and largest ~ U[1, 10] (so cond(J) <= 10), and
    t ~ U[-1, 1]^dim."""
    rng = np.random.default_rng(seed)
    smax = rng.uniform(1.0, 10.0)
    if dim == 2:
        sig = np.array([1.0, smax])
    else:
        sig = np.array([1.0, rng.uniform(1.0, smax), smax])
    J = _rotation(dim, rng) @ np.diag(sig) @ _rotation(dim, rng)
    t = rng.uniform(-1.0, 1.0, dim)
    return J, t


def apply_affine(coords, J, t):
    return coords @ np.asarray(J).T + np.asarray(t)


def affine_triangle(seed: int):
    """The reference triangle under ``random_affine(2, seed)``."""
    coords, cells = unit_triangle()
    J, t = random_affine(2, seed)
    return apply_affine(coords, J, t), cells


def shuffle_cell_orders(cells, seed: int):
    """Seeded random permutation of the vertex order of every cell."""
    rng = np.random.default_rng(seed)
    out = np.array(cells, copy=True)
    for i in range(out.shape[0]):
        out[i] = out[i][rng.permutation(out.shape[1])]
    return out


def all_permutations(n):
    return list(itertools.permutations(range(n)))
