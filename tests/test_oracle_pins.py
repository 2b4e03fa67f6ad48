"""The oracle pinned to things other than itself (CPU only).

Each test checks the oracle against a fact the paper or the mathematics fixes:
counts printed in the paper, closed forms of the P1 stencil, invariants of
the stiffness matrix, the Galerkin identity of nested P1 spaces, a discrete
manufactured solution, a published generator test vector, and an independent
dense brute-force assembly by geometric refinement (tests/bruteforce.py).
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import bruteforce
from oracle.oracle import OracleMesh, keyed_points, prolongation, sample_rows, solve, splitmix64
from paper_2305_15116_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _match(a, b):
    d, i = cKDTree(b).query(a)
    assert d.max() < 1e-8
    return i


def _find(xyz, p):
    d = np.abs(xyz - p).sum(1)
    j = int(np.argmin(d))
    assert d[j] < 1e-9
    return j


MESHES_2D = {
    "tri": lambda: W.affine_triangle(2),
    "square": W.two_triangle_square,
    "strip5": lambda: W.strip_2d(5),
    "strip4_shuffled": lambda: (W.strip_2d(4)[0], W.shuffle_cell_orders(W.strip_2d(4)[1], 3)),
}
MESHES_3D = {
    "tet": W.unit_tet,
    "cube": W.kuhn_cube,
    "cube_random": lambda: W.kuhn_cube("random", 5),
    "strip9": lambda: W.strip_3d(9),
}


def _mapped(mk, dim, seed=11):
    co, ce = mk()
    J, t = W.random_affine(dim, seed)
    return W.apply_affine(co, J, t), ce


# ---------------------------------------------------------------- counts
def test_vertex_dof_count_matches_paper():
    """One triangle has (2^l+1)(2^l+2)/2 vertex DoFs; the paper prints 525825 at level 10."""
    g = json.load(open(os.path.join(GOLDEN, "paper_level10.json")))
    for L in range(0, 7):
        N = 1 << L
        assert OracleMesh(*W.unit_triangle(), L).n == (N + 1) * (N + 2) // 2
    assert OracleMesh(*W.unit_triangle(), g["level"]).n == g["vertex_dofs"]
    # the paper's total P2 count and byte figures follow from the same counts
    N = 1 << g["level"]
    edge = N * (N + 1) // 2
    assert edge == g["edge_dofs_per_orientation"]
    assert g["vertex_dofs"] + 3 * edge == g["total_p2_dofs"]
    assert 8 * g["total_p2_dofs"] == g["dof_mem_bytes"]
    assert 8 * g["vertex_stencil_entries_p2"] * g["vertex_dofs"] == g["vertex_stencil_bytes"]
    assert 8 * g["edge_stencil_entries_p2"] * 3 * edge == g["edge_stencil_bytes"]


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4])
def test_3d_unique_counts(L):
    N = 1 << L
    assert OracleMesh(*W.unit_tet(), L).n == (N + 1) * (N + 2) * (N + 3) // 6
    assert OracleMesh(*W.kuhn_cube(), L).n == (N + 1) ** 3
    assert OracleMesh(*W.kuhn_cube("random", 5), L).n == (N + 1) ** 3


def test_two_square_counts():
    for L in range(4):
        N = 1 << L
        assert OracleMesh(*W.two_triangle_square(), L).n == (N + 1) ** 2


# ---------------------------------------------------------------- pin 1: 2D closed form
@pytest.mark.parametrize("seed", [2, 7, 19])
def test_2d_stencil_closed_form(seed):
    """For an affine triangle with J = [P1-P0 | P2-P0], M = (J^T J)^-1 = [[a,b],[b,c]]
    and D = |det J|, every interior row is C = 2D(a+b+c), E = W = -D(a+b),
    N = S = -D(b+c), NW = SE = D b, independent of the level."""
    co, ce = W.affine_triangle(seed)
    J = np.column_stack([co[1] - co[0], co[2] - co[0]])
    M = np.linalg.inv(J.T @ J)
    a, b, c = M[0, 0], M[0, 1], M[1, 1]
    D = abs(np.linalg.det(J))
    expect = {(0, 0): 2 * D * (a + b + c), (1, 0): -D * (a + b), (-1, 0): -D * (a + b),
              (0, 1): -D * (b + c), (0, -1): -D * (b + c), (-1, 1): D * b, (1, -1): D * b}
    for L in (2, 4):
        m = OracleMesh(co, ce, L)
        A = m.csr(dirichlet=False)
        xyz = m.xyz()
        N = m.N
        P0, e1, e2 = co[0], (co[1] - co[0]) / N, (co[2] - co[0]) / N
        rng = np.random.default_rng(seed + L)
        for _ in range(10):
            y = int(rng.integers(1, N - 1))
            x = int(rng.integers(1, N - y))
            u = _find(xyz, P0 + x * e1 + y * e2)
            row = A.getrow(u)
            assert row.nnz == 7
            for (dx, dy), val in expect.items():
                j = _find(xyz, P0 + (x + dx) * e1 + (y + dy) * e2)
                assert abs(A[u, j] - val) <= 1e-13 * max(1.0, abs(expect[(0, 0)]))


@pytest.mark.parametrize("L", [10, 14])
def test_sampled_rows_at_full_level_match_closed_form(L):
    """At the benchmark level the oracle's row evaluator still reproduces the
    closed-form stencil of an affine triangle to rounding (its micro-element
    edge vectors carry full precision)."""
    co, ce = W.affine_triangle(2)
    J = np.column_stack([co[1] - co[0], co[2] - co[0]])
    M = np.linalg.inv(J.T @ J)
    a, b, c = M[0, 0], M[0, 1], M[1, 1]
    D = abs(np.linalg.det(J))
    offs = [((0, -1), -D * (b + c)), ((1, -1), D * b), ((-1, 0), -D * (a + b)), ((0, 0), 2 * D * (a + b + c)),
            ((1, 0), -D * (a + b)), ((-1, 1), D * b), ((0, 1), -D * (b + c))]
    N = 1 << L
    rng = np.random.default_rng(L)
    ys = rng.integers(1, N - 1, 200)
    xs = np.array([rng.integers(1, N - y) for y in ys])
    pts = np.stack([xs, ys], 1)
    got, bnd = sample_rows(co, ce, L, 5, np.zeros(len(pts), np.int64), pts)
    assert not bnd.any()
    exp = np.zeros(len(pts))
    for (dx, dy), w in offs:
        exp += w * keyed_points(ce, 2, L, 5, np.zeros(len(pts), np.int64), pts + np.array([dx, dy]))
    wsum = sum(abs(w) for _, w in offs)
    assert np.abs(got - exp).max() <= 1e-14 * wsum


def test_reference_triangle_is_five_point():
    """The reference triangle gives 4, -1, -1 and exactly zero diagonal weights."""
    m = OracleMesh(*W.unit_triangle(), 3)
    A = m.csr(dirichlet=False)
    xyz = m.xyz()
    h = 1.0 / m.N
    u = _find(xyz, np.array([3 * h, 2 * h]))
    assert A[u, u] == pytest.approx(4.0, abs=1e-14)
    for d in ([h, 0], [-h, 0], [0, h], [0, -h]):
        assert A[u, _find(xyz, xyz[u] + d)] == pytest.approx(-1.0, abs=1e-14)
    for d in ([-h, h], [h, -h]):
        assert abs(A[u, _find(xyz, xyz[u] + d)]) <= 1e-15


# ---------------------------------------------------------------- pin 2: Kuhn cube
@pytest.mark.parametrize("L", [1, 2, 3])
def test_kuhn_cube_is_seven_point_fd(L):
    """With the canonical vertex order every non-boundary row of the 6-tet cube,
    including DoFs on the shared macro faces, edges and diagonal, is
    6h x_c - h * (sum of the 6 axis neighbours), all other entries zero."""
    m = OracleMesh(*W.kuhn_cube(), L)
    A = m.csr(dirichlet=True)
    bnd = m.boundary()
    xyz = m.xyz()
    h = 1.0 / m.N
    for u in np.where(~bnd)[0]:
        expect = {u: 6 * h}
        for ax in range(3):
            for s in (-1, 1):
                p = xyz[u].copy()
                p[ax] += s * h
                expect[_find(xyz, p)] = -h
        row = A.getrow(u)
        for j, v in zip(row.indices, row.data):
            assert abs(v - expect.get(j, 0.0)) <= 1e-14
        for j, v in expect.items():
            assert abs(A[u, j] - v) <= 1e-14
    # boundary rows are identity rows
    for u in np.where(bnd)[0]:
        row = A.getrow(u)
        assert list(row.indices) == [u] and row.data[0] == 1.0


# ---------------------------------------------------------------- pin 3: invariants
@pytest.mark.parametrize("name", list(MESHES_2D) + list(MESHES_3D))
def test_matrix_invariants(name):
    """A 1 = 0 and A (affine) = 0 on non-boundary rows; symmetric before boundary
    conditions; every row strictly inside a macro has 7 (2D) / 15 (3D) entries
    and a positive diagonal."""
    mk = MESHES_2D.get(name) or MESHES_3D[name]
    dim = 2 if name in MESHES_2D else 3
    co, ce = _mapped(mk, dim)
    m = OracleMesh(co, ce, 3 if dim == 2 else 2)
    A0 = m.csr(dirichlet=False)
    A = m.csr(dirichlet=True)
    bnd = m.boundary()
    xyz = m.xyz()
    scale = abs(A0).max()
    assert abs(A0 - A0.T).max() <= 1e-14 * scale
    rng = np.random.default_rng(1)
    affine = 0.3 + xyz @ rng.uniform(-1, 1, dim)
    for vec in (np.ones(m.n), affine):
        r = (A @ vec)[~bnd]
        assert np.abs(r).max() <= 1e-13 * scale * max(1.0, np.abs(vec).max())
    v, _ = m.keys()
    strictly_inside = (v >= 0).sum(1) == dim + 1
    nnz = np.diff(A.indptr)
    assert (nnz[strictly_inside & ~bnd] == (7 if dim == 2 else 15)).all()
    assert (A.diagonal()[~bnd] > 0).all()


# ---------------------------------------------------------------- pin 4: mesh
@pytest.mark.parametrize("name", ["tri", "strip5", "tet", "cube_random", "strip9"])
def test_micro_mesh(name):
    """N^d micro-elements per macro; volumes sum to the macro volume; every
    internal micro-facet has two elements; a lone tet has 4 N^2 boundary faces."""
    mk = MESHES_2D.get(name) or MESHES_3D[name]
    dim = 2 if name in MESHES_2D else 3
    co, ce = _mapped(mk, dim)
    for L in (1, 2, 3):
        m = OracleMesh(co, ce, L)
        el = m.elements()
        assert el.shape[0] == ce.shape[0] * m.N ** dim
        xyz = m.xyz()
        E = xyz[el[:, 1:]] - xyz[el[:, :1]]
        vol = np.abs(np.linalg.det(E)) / (2 if dim == 2 else 6)
        macro = np.abs(np.linalg.det(co[ce[:, 1:]] - co[ce[:, :1]])) / (2 if dim == 2 else 6)
        assert vol.sum() == pytest.approx(macro.sum(), rel=1e-12)
        assert vol.min() > 0
        faces = {}
        for e in el:
            for skip in range(dim + 1):
                f = tuple(sorted(np.delete(e, skip)))
                faces[f] = faces.get(f, 0) + 1
        assert max(faces.values()) == 2
        if name == "tet":
            assert sum(1 for c in faces.values() if c == 1) == 4 * m.N ** 2


# ---------------------------------------------------------------- pin 5: Galerkin
@pytest.mark.parametrize("name", ["strip4_shuffled", "tri", "cube_random", "strip9", "tet"])
def test_galerkin_identity(name):
    """P^T A_l P = A_{l-1} for the P1 prolongation of nested spaces, and P maps
    a coarse affine function onto the fine one."""
    mk = MESHES_2D.get(name) or MESHES_3D[name]
    dim = 2 if name in MESHES_2D else 3
    co, ce = _mapped(mk, dim, seed=3)
    for L in (1, 2, 3):
        f, c = OracleMesh(co, ce, L), OracleMesh(co, ce, L - 1)
        P = prolongation(f, c)
        Af, Ac = f.csr(dirichlet=False), c.csr(dirichlet=False)
        assert abs(P.T @ Af @ P - Ac).max() <= 1e-13 * abs(Ac).max()
        g = np.array([0.7, -1.3, 0.4][:dim])
        assert np.abs(P @ (c.xyz() @ g + 2.0) - (f.xyz() @ g + 2.0)).max() <= 1e-13


# ---------------------------------------------------------------- pin 6: manufactured solution
@pytest.mark.parametrize("mesh,L", [("square", 2), ("square", 4), ("cube", 2), ("cube", 3)])
def test_discrete_manufactured_solution(mesh, L):
    """On the two-triangle square and the Kuhn cube, (A u)_i = h^(d-2)(2d u_i -
    sum of axis neighbours) and the lumped mass is h^d, so for
    u* = prod sin(pi x_k) and f = d pi^2 u* the exact discrete solution of
    A u = M_lumped f is u* (pi^2 h^2 / 4) / sin^2(pi h / 2)."""
    co, ce = W.two_triangle_square() if mesh == "square" else W.kuhn_cube()
    dim = co.shape[1]
    m = OracleMesh(co, ce, L)
    h = 1.0 / m.N
    xyz = m.xyz()
    us = np.prod(np.sin(np.pi * xyz), axis=1)
    b = m.lumped_mass() * dim * np.pi ** 2 * us
    bnd = m.boundary()
    b[bnd] = 0.0
    uh = us * (np.pi ** 2 * h ** 2 / 4) / np.sin(np.pi * h / 2) ** 2
    uh[bnd] = 0.0
    r = m.spmv(uh) - b
    assert np.abs(r).max() <= 1e-13 * np.abs(b).max()
    # and the oracle's solve reproduces it
    u = solve(m, b, tol=1e-14)
    assert np.abs(u - uh).max() <= 1e-10


# ---------------------------------------------------------------- pin 7: brute force
@pytest.mark.parametrize("name", list(MESHES_2D) + list(MESHES_3D))
def test_bruteforce_dense_assembly(name):
    mk = MESHES_2D.get(name) or MESHES_3D[name]
    dim = 2 if name in MESHES_2D else 3
    co, ce = _mapped(mk, dim, seed=23)
    for L in range(0, 4 if dim == 2 else 3):
        m = OracleMesh(co, ce, L)
        pts, A, bnd = bruteforce.assemble_dense(co, ce, L)
        assert len(pts) == m.n
        i = _match(m.xyz(), pts)
        Ab = A[np.ix_(i, i)]
        assert np.abs(m.csr(dirichlet=False).toarray() - Ab).max() <= 1e-12 * np.abs(Ab).max()
        assert (m.boundary() == bnd[i]).all()


def test_bruteforce_level3_3d():
    co, ce = _mapped(MESHES_3D["cube_random"], 3, seed=29)
    m = OracleMesh(co, ce, 3)
    pts, A, bnd = bruteforce.assemble_dense(co, ce, 3)
    i = _match(m.xyz(), pts)
    Ab = A[np.ix_(i, i)]
    assert np.abs(m.csr(dirichlet=False).toarray() - Ab).max() <= 1e-12 * np.abs(Ab).max()


# ---------------------------------------------------------------- internal agreement
@pytest.mark.parametrize("name", ["strip5", "cube_random", "strip9"])
def test_elementwise_and_sampled_rows_match_csr(name):
    """The element-by-element apply and the sampled-row evaluator give the CSR rows."""
    mk = MESHES_2D.get(name) or MESHES_3D[name]
    dim = 2 if name in MESHES_2D else 3
    co, ce = _mapped(mk, dim, seed=31)
    L = 4 if dim == 2 else 3
    m = OracleMesh(co, ce, L)
    x = m.keyed_random(77)
    y = m.spmv(x)
    assert np.abs(m.apply_elementwise(x) - y).max() <= 1e-13 * np.abs(y).max()
    # sample every lattice point of every cell and compare by key
    N = m.N
    sc, sl = [], []
    for c in range(ce.shape[0]):
        if dim == 2:
            pts = [(px, py) for py in range(N + 1) for px in range(N + 1 - py)]
        else:
            pts = [(px, py, pz) for pz in range(N + 1) for py in range(N + 1 - pz) for px in range(N + 1 - py - pz)]
        sc += [c] * len(pts)
        sl += pts
    ys, _ = sample_rows(co, ce, L, 77, np.array(sc), np.array(sl))
    # map each sample to its unique DoF by physical coordinates
    P = co[ce[np.array(sc)]]
    lat = np.array(sl, dtype=float) / N
    X = P[:, 0] + np.einsum("sk,skd->sd", lat, P[:, 1:] - P[:, :1])
    idx = _match(X, m.xyz())
    assert np.abs(ys - y[idx]).max() <= 1e-13 * np.abs(y).max()


def test_splitmix64_published_sequence():
    """SplitMix64 from state 0 emits e220a8397b1dcdaf, 6e789e6aa1b965f4, 06c45d188009454f."""
    g = 0x9E3779B97F4A7C15
    M = (1 << 64) - 1
    out = [splitmix64((k * g) & M) for k in range(3)]
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_keyed_random_is_uniform_and_copy_consistent():
    m = OracleMesh(*W.strip_2d(6), 5)
    x = m.keyed_random(3)
    assert x.min() >= -1 and x.max() < 1
    assert abs(x.mean()) < 0.05 and abs(x.var() - 1 / 3) < 0.03
    assert not np.array_equal(x, m.keyed_random(4))


def test_nonconforming_mesh_rejected():
    co = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [-1, 1.0]])
    ce = np.array([[0, 1, 2], [1, 3, 2], [0, 2, 1]])  # duplicate cell
    with pytest.raises(ValueError):
        OracleMesh(co, ce, 1)
