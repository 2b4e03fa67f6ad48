"""The blended-macro oracle pinned to things other than itself (CPU only).

Blended macros map their lattice by F_c(xi) = affine(xi) + xi0 xi1 xi2 d_c;
the micro mesh has straight triangles on the mapped points.  Pins: the test
maps every DoF itself (from its exact key and the macro map), then checks
that u^T A u equals the discrete energy summed from those coordinates (which
fixes every entry of a symmetric matrix), that linear functions of the
mapped coordinates give zero interior rows (the micro triangles are
straight, so the interpolant is exact), that d = 0 gives the affine matrix,
and constants in the kernel, symmetry and identity Dirichlet rows.
"""
import numpy as np
import pytest

from oracle.oracle import OracleMesh
from paper_2305_15116_amd import workloads as W

MESHES = {
    "tri": lambda: W.affine_triangle(2),
    "square": W.two_triangle_square,
    "strip5_shuffled": lambda: (W.strip_2d(5)[0], W.shuffle_cell_orders(W.strip_2d(5)[1], 3)),
}


def _bubbles(nc, seed):
    return np.random.default_rng(seed).uniform(-0.8, 0.8, (nc, 2))


def _mapped_xyz(om, co, ce, d):
    """Mapped coordinates of every unique DoF, from its key: points inside a
    macro use that macro's bubble; points on macro edges have none."""
    vid, wt = om.keys()
    N = om.N
    out = np.zeros((om.n, 2))
    cells = [set(int(v) for v in c) for c in ce]
    for i in range(om.n):
        sup = [(int(v), int(w)) for v, w in zip(vid[i], wt[i]) if v >= 0 and w > 0]
        out[i] = sum(w * co[v] for v, w in sup) / N
        if len(sup) == 3:
            c = next(k for k, cs in enumerate(cells) if cs == {v for v, _ in sup})
            lam = {v: w / N for v, w in sup}
            out[i] += lam[ce[c][0]] * lam[ce[c][1]] * lam[ce[c][2]] * d[c]
    return out


def _energy(om, X, u):
    el = om.elements()
    P = X[el]
    E = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))
    du = u[el[:, 1:]] - u[el[:, :1]]
    g = np.linalg.solve(np.transpose(E, (0, 2, 1)), du[..., None])[..., 0]
    area = np.abs(np.linalg.det(E)) / 2.0
    return float(np.sum(area * np.sum(g * g, axis=1)))


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("L", [1, 2, 4])
def test_energy_and_linear_functions(name, L):
    co, ce = MESHES[name]()
    om = OracleMesh(co, ce, L)
    d = _bubbles(len(ce), L)
    A = om.csr_blended(d, dirichlet=False)
    scale = abs(A).max()
    assert abs(A - A.T).max() <= 1e-13 * scale
    assert np.abs(A @ np.ones(om.n)).max() <= 1e-12 * scale
    X = _mapped_xyz(om, co, ce, d)
    rng = np.random.default_rng(L)
    for _ in range(2):
        u = rng.standard_normal(om.n)
        e = _energy(om, X, u)
        assert abs(u @ (A @ u) - e) <= 1e-11 * max(1.0, e)
    inner = ~om.boundary()
    lin = 0.7 - 1.3 * X[:, 0] + 2.1 * X[:, 1]
    if inner.any():
        assert np.abs((A @ lin)[inner]).max() <= 1e-11 * scale


@pytest.mark.parametrize("name", ["tri", "strip5_shuffled"])
def test_zero_bubble_is_affine_and_dirichlet_rows(name):
    co, ce = MESHES[name]()
    om = OracleMesh(co, ce, 3)
    A0 = om.csr_blended(np.zeros((len(ce), 2)), dirichlet=False).toarray()
    A1 = om.csr(dirichlet=False).toarray()
    np.testing.assert_allclose(A0, A1, rtol=0, atol=1e-13 * np.abs(A1).max())
    d = _bubbles(len(ce), 9)
    Ad = om.csr_blended(d, dirichlet=True).toarray()
    An = om.csr_blended(d, dirichlet=False).toarray()
    bnd = om.boundary()
    np.testing.assert_array_equal(Ad[bnd], np.eye(om.n)[bnd])
    np.testing.assert_array_equal(Ad[~bnd], An[~bnd])
    # a real bubble changes the interior rows
    assert np.abs(An - A1).max() > 1e-3 * np.abs(A1).max()
