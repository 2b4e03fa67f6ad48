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


def _exact_row(co, ce, c, d, N, p, xval):
    """Row p of the blended operator in exact rational arithmetic: the six
    micro-triangles of macro c around the interior lattice point p, each with
    the textbook P1 matrix K_ij = (E_i . E_j) / (4 |T|), E_i the edge opposite
    vertex i, on exactly mapped points F(i, j) = P0 + (P1 - P0) i/N +
    (P2 - P0) j/N + (N - i - j) i j / N^3 d."""
    from fractions import Fraction as Fr
    P = [[Fr(float(v)) for v in co[k]] for k in ce[c]]
    dd = [Fr(float(v)) for v in d[c]]

    def F(q):
        i, j = q
        bub = Fr((N - i - j) * i * j, N ** 3)
        return [P[0][r] + (P[1][r] - P[0][r]) * Fr(i, N) + (P[2][r] - P[0][r]) * Fr(j, N) + bub * dd[r]
                for r in range(2)]

    i, j = p
    tris = [((i, j), (i + 1, j), (i, j + 1)), ((i - 1, j), (i, j), (i - 1, j + 1)), ((i, j - 1), (i + 1, j - 1), (i, j)),
            ((i, j), (i, j + 1), (i - 1, j + 1)), ((i, j - 1), (i, j), (i - 1, j)), ((i + 1, j - 1), (i + 1, j), (i, j))]
    acc = Fr(0)
    for t in tris:
        X = [F(q) for q in t]
        E = [[X[2][r] - X[1][r] for r in range(2)], [X[0][r] - X[2][r] for r in range(2)],
             [X[1][r] - X[0][r] for r in range(2)]]
        area2 = abs(E[2][0] * (-E[1][1]) - E[2][1] * (-E[1][0]))  # |det [X1-X0, X2-X0]|
        me = t.index(p)
        for k in range(3):
            acc += (E[me][0] * E[k][0] + E[me][1] * E[k][1]) / (2 * area2) * xval[t[k]]
    return acc


def test_sampled_rows_match_exact_rational_rows_at_level_14():
    """At level 14 the mapped points are O(1) apart from the origin but 1/N
    apart from each other; the oracle's rows must still agree with rows
    computed in exact rational arithmetic to about the rounding of the
    element matrices (1e-13 of the row's absolute sum)."""
    from fractions import Fraction as Fr

    from oracle.oracle import keyed_points, sample_rows_blended
    co, ce = W.affine_triangle(2)
    L = 14
    N = 1 << L
    d = np.array([[0.45, -0.3]])
    rng = np.random.default_rng(5)
    pts = []
    while len(pts) < 12:
        i, j = int(rng.integers(1, N)), int(rng.integers(1, N))
        if i + j <= N - 1:
            pts.append((i, j))
    pts += [(1, 1), (N - 2, 1), (1, N - 2), (N // 3, N // 3)]
    y, bnd = sample_rows_blended(co, ce, L, 11, d, np.zeros(len(pts), np.int64), np.array(pts))
    assert not bnd.any()
    for p, yo in zip(pts, y):
        nb = [(p[0] + a, p[1] + b) for a, b in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1))]
        xv = keyed_points(ce, 2, L, 11, np.zeros(len(nb), np.int64), np.array(nb))
        xval = {q: Fr(float(v)) for q, v in zip(nb, xv)}
        ex = _exact_row(co, ce, 0, d, N, p, xval)
        scale = float(sum(abs(v) for v in xval.values()))
        assert abs(yo - float(ex)) <= 1e-13 * scale, (p, yo, float(ex))


@pytest.mark.parametrize("name", sorted(MESHES))
def test_row_evaluator_matches_assembled_rows(name):
    """The sampled-row evaluator (no global build) against the assembled CSR
    of the same blended operator, every point of a small level."""
    import harness
    from oracle.oracle import sample_rows_blended
    co, ce = MESHES[name]()
    L = 3
    d = _bubbles(len(ce), 4)
    om = OracleMesh(co, ce, L)
    yo = om.csr_blended(d) @ om.keyed_random(9)
    N = om.N
    pts = np.array([(c, i, j) for c in range(len(ce)) for j in range(N + 1) for i in range(N + 1 - j)], np.int64)
    ys, _ = sample_rows_blended(co, ce, L, 9, d, pts[:, 0], pts[:, 1:])
    # map (cell, lattice point) to unique DoFs through the exact keys
    vid, wt = om.keys()
    key_of = {tuple(sorted((int(v), int(w)) for v, w in zip(vv, ww) if v >= 0 and w > 0)): u
              for u, (vv, ww) in enumerate(zip(vid, wt))}
    for (c, i, j), val in zip(pts, ys):
        cv = ce[c]
        k = tuple(sorted((int(v), int(w)) for v, w in zip(cv, (N - i - j, i, j)) if w > 0))
        assert abs(val - yo[key_of[k]]) <= 1e-13 * max(1.0, np.abs(yo).max())
