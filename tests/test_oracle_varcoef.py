"""The variable-coefficient oracle pinned to things other than itself (CPU only).

For a symmetric matrix the quadratic form fixes every entry, and for
-div(k grad u) with k the P1 interpolant of nodal values the form is the
discrete energy: u^T A u = sum over micro-elements T of |T| mean_T(k)
|grad u_h|^2, where grad u_h is the gradient of the linear interpolant on T.
The test computes that sum from vertex coordinates alone (no element
matrices), so a wrong coefficient average, a missing element or a wrong sign
in the assembly fails it.  Also: k = 1 gives the constant-coefficient matrix,
linearity in k, constants in the kernel, identity Dirichlet rows.
"""
import numpy as np
import pytest

from oracle.oracle import OracleMesh
from paper_2305_15116_amd import workloads as W

MESHES = {
    "tri": (lambda: W.affine_triangle(2), 2),
    "strip4_shuffled": (lambda: (W.strip_2d(4)[0], W.shuffle_cell_orders(W.strip_2d(4)[1], 3)), 2),
    "cube_random": (lambda: W.kuhn_cube("random", 5), 3),
}


def _mesh(name, L):
    mk, dim = MESHES[name]
    co, ce = mk()
    J, t = W.random_affine(dim, 13)
    return OracleMesh(W.apply_affine(co, J, t), ce, L)


def _energy(om, k, u):
    """sum_T |T| mean_T(k) |grad u_h|^2 from the element vertex coordinates."""
    el = om.elements()
    xyz = om.xyz()
    d = xyz.shape[1]
    P = xyz[el]                              # ne x (d+1) x d
    E = np.transpose(P[:, 1:, :] - P[:, :1, :], (0, 2, 1))  # columns X_k - X_0
    du = u[el[:, 1:]] - u[el[:, :1]]          # ne x d
    g = np.linalg.solve(np.transpose(E, (0, 2, 1)), du[..., None])[..., 0]  # E^T g = du
    vol = np.abs(np.linalg.det(E)) / (2.0 if d == 2 else 6.0)
    kt = k[el].mean(axis=1)
    return float(np.sum(vol * kt * np.sum(g * g, axis=1)))


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("L", [1, 2, 3])
def test_energy_identity(name, L):
    om = _mesh(name, L)
    rng = np.random.default_rng(L)
    k = 0.5 + rng.random(om.n) * 2.0
    A = om.csr_varcoef(k, dirichlet=False)
    scale = abs(A).max()
    assert abs(A - A.T).max() <= 1e-13 * scale
    for _ in range(3):
        u = rng.standard_normal(om.n)
        e_ref = _energy(om, k, u)
        assert abs(u @ (A @ u) - e_ref) <= 1e-12 * max(1.0, abs(e_ref))
    u, v = rng.standard_normal(om.n), rng.standard_normal(om.n)
    pol = 0.5 * (_energy(om, k, u + v) - _energy(om, k, u) - _energy(om, k, v))
    assert abs(u @ (A @ v) - pol) <= 1e-11 * max(1.0, abs(pol))


@pytest.mark.parametrize("name", ["tri", "strip4_shuffled"])
def test_constant_and_linear_in_k(name):
    om = _mesh(name, 3)
    A1 = om.csr(dirichlet=False)
    ones = np.ones(om.n)
    np.testing.assert_allclose(om.csr_varcoef(ones, dirichlet=False).toarray(), A1.toarray(), rtol=0,
                               atol=1e-15 * abs(A1).max())
    np.testing.assert_allclose(om.csr_varcoef(2.5 * ones, dirichlet=False).toarray(), 2.5 * A1.toarray(), rtol=0,
                               atol=1e-14 * abs(A1).max())
    rng = np.random.default_rng(4)
    k1, k2 = rng.random(om.n), rng.random(om.n)
    S = om.csr_varcoef(k1 + k2, dirichlet=False).toarray()
    T = om.csr_varcoef(k1, dirichlet=False).toarray() + om.csr_varcoef(k2, dirichlet=False).toarray()
    np.testing.assert_allclose(S, T, rtol=0, atol=1e-13 * abs(S).max())
    Ak = om.csr_varcoef(0.5 + k1, dirichlet=False)
    assert np.abs(Ak @ ones).max() <= 1e-13 * abs(Ak).max()
    Ad = om.csr_varcoef(0.5 + k1, dirichlet=True).toarray()
    bnd = om.boundary()
    np.testing.assert_array_equal(Ad[bnd], np.eye(om.n)[bnd])
    np.testing.assert_array_equal(Ad[~bnd], Ak.toarray()[~bnd])


@pytest.mark.parametrize("dim", [2, 3])
def test_row_evaluator_matches_assembled_varcoef_rows(dim):
    """The sampled-row evaluator (no global build) against the assembled
    variable-coefficient CSR, every point of a small level."""
    from oracle.oracle import sample_rows_varcoef
    if dim == 2:
        co, ce = W.strip_2d(3)
    else:
        co, ce = W.kuhn_cube("random", 5)
    J, t = W.random_affine(dim, 6)
    co = W.apply_affine(co, J, t)
    L = 2
    om = OracleMesh(co, ce, L)
    k = om.keyed_random(8) + 1.5
    yo = om.csr_varcoef(k) @ om.keyed_random(9)
    N = om.N
    if dim == 2:
        lat = [(i, j) for j in range(N + 1) for i in range(N + 1 - j)]
    else:
        lat = [(i, j, z) for z in range(N + 1) for j in range(N + 1 - z) for i in range(N + 1 - j - z)]
    pts = np.array([(c, *p) for c in range(len(ce)) for p in lat], np.int64)
    ys, _ = sample_rows_varcoef(co, ce, L, 9, 8, 1.5, pts[:, 0], pts[:, 1:])
    vid, wt = om.keys()
    key_of = {tuple(sorted((int(v), int(w)) for v, w in zip(vv, ww) if v >= 0 and w > 0)): u
              for u, (vv, ww) in enumerate(zip(vid, wt))}
    for row, val in zip(pts, ys):
        c, p = row[0], row[1:]
        bary = (N - int(sum(p)), *[int(q) for q in p])
        key = tuple(sorted((int(v), w) for v, w in zip(ce[c], bary) if w > 0))
        assert abs(val - yo[key_of[key]]) <= 1e-13 * max(1.0, np.abs(yo).max())
