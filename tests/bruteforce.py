"""Dense brute-force P1 assembly by geometric refinement (tiny levels only).

A second, independent construction used to pin the oracle: each macro cell is
refined recursively in physical space (2D: red refinement at edge midpoints;
3D: Bey's rule, children [x0,x01,x02,x03], [x01,x1,x12,x13],
[x02,x12,x2,x23], [x03,x13,x23,x3] and the four tets around the x02-x13
diagonal), vertices are merged by rounded coordinates, and the dense
stiffness matrix is summed from P1 element matrices whose gradients come from
numpy.linalg.solve.  Nothing here looks at index spaces, keys or stencils.
"""
from __future__ import annotations

import numpy as np


def _mid(a, b):
    return 0.5 * (a + b)


def refine(verts, dim):
    """Children of one simplex given as a (dim+1, dim) array of vertices."""
    if dim == 2:
        a, b, c = verts
        ab, ac, bc = _mid(a, b), _mid(a, c), _mid(b, c)
        return [np.array(t) for t in ([a, ab, ac], [ab, b, bc], [ac, bc, c], [ab, bc, ac])]
    x0, x1, x2, x3 = verts
    x01, x02, x03 = _mid(x0, x1), _mid(x0, x2), _mid(x0, x3)
    x12, x13, x23 = _mid(x1, x2), _mid(x1, x3), _mid(x2, x3)
    kids = [[x0, x01, x02, x03], [x01, x1, x12, x13], [x02, x12, x2, x23], [x03, x13, x23, x3],
            [x01, x02, x03, x13], [x01, x02, x12, x13], [x02, x03, x13, x23], [x02, x12, x13, x23]]
    return [np.array(t) for t in kids]


def refined_elements(coords, cells, level):
    """List of micro-simplices (arrays of physical vertices) after `level` refinements."""
    dim = coords.shape[1]
    elems = [coords[c] for c in cells]
    for _ in range(level):
        nxt = []
        for e in elems:
            nxt.extend(refine(e, dim))
        elems = nxt
    return elems


def assemble_dense(coords, cells, level, decimals=10):
    """Returns (points, A, boundary) with A the dense pre-boundary-condition
    stiffness matrix and boundary the flags of points on boundary facets
    (micro-facets that belong to exactly one micro-element)."""
    coords = np.asarray(coords, dtype=np.float64)
    dim = coords.shape[1]
    elems = refined_elements(coords, np.asarray(cells), level)
    index = {}
    pts = []

    def pid(p):
        k = tuple(np.round(p, decimals) + 0.0)
        if k not in index:
            index[k] = len(pts)
            pts.append(p)
        return index[k]

    conn = [[pid(p) for p in e] for e in elems]
    n = len(pts)
    A = np.zeros((n, n))
    facets = {}
    for e, ids in zip(elems, conn):
        E = (e[1:] - e[0]).T
        # grad lambda_k (k>=1) are the rows of E^{-1}
        Ginv = np.linalg.solve(E, np.eye(dim))
        G = np.vstack([-Ginv.sum(axis=0), Ginv])
        vol = abs(np.linalg.det(E)) / (2.0 if dim == 2 else 6.0)
        K = vol * G @ G.T
        for i in range(dim + 1):
            for j in range(dim + 1):
                A[ids[i], ids[j]] += K[i, j]
        for skip in range(dim + 1):
            f = tuple(sorted(ids[k] for k in range(dim + 1) if k != skip))
            facets[f] = facets.get(f, 0) + 1
    bnd = np.zeros(n, dtype=bool)
    for f, c in facets.items():
        if c == 1:
            bnd[list(f)] = True
    return np.array(pts), A, bnd
