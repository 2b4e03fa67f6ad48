"""GPU parity of the fused 2D P2 operator (apply_p2, through the C ABI).

FP64 results must match the oracle's assembled P2 matrix within 1e-12
relative in the max norm; FP32 results within 32 u32 (|A| |x|)_i per row
(at most 19 products, the paired additions and the rounded weights).  At the
full size of the benchmark (P2 level 13, 134,242,305 DoFs) the oracle cannot
be assembled, so the whole output is checked against what the P2 space fixes
exactly: for the interpolant of a quadratic q, Dirichlet rows give q, interior
vertex rows 0 and interior edge rows -Laplace(q) times the basis integral.
"""
import numpy as np
import pytest

import harness
import paper_2305_15116_amd as P
from oracle.oracle import OracleMesh
from paper_2305_15116_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _mesh(name):
    table = {
        "tri_ref": (W.unit_triangle, False),
        "tri_affine": (lambda: W.affine_triangle(2), False),
        "square": (W.two_triangle_square, True),
        "strip2d": (lambda: W.strip_2d(5), True),
        "strip2d_shuf": (lambda: (W.strip_2d(6)[0], W.shuffle_cell_orders(W.strip_2d(6)[1], 4)), True),
    }
    mk, affine = table[name]
    co, ce = mk()
    if affine:
        J, t = W.random_affine(2, 17)
        co = W.apply_affine(co, J, t)
    return co, ce


def _setup(name, level, flags=P.MF_FLAG_DIRICHLET):
    co, ce = _mesh(name)
    m = P.create_macro_mesh(co, ce, level + 1, flags)
    om = OracleMesh(co, ce, level + 1)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, level + 1), om.keys())
    return m, om, s2u


CASES = [("tri_ref", 2), ("tri_affine", 0), ("tri_affine", 1), ("tri_affine", 4), ("tri_affine", 7),
         ("square", 5), ("strip2d", 4), ("strip2d_shuf", 3), ("strip2d_shuf", 6)]


@pytest.mark.parametrize("dirichlet", [True, False])
@pytest.mark.parametrize("name,level", CASES)
def test_p2_apply_fp64_matches_oracle(name, level, dirichlet):
    m, om, s2u = _setup(name, level, P.MF_FLAG_DIRICHLET if dirichlet else 0)
    s, _ = P.mesh_num_dofs(m, level + 1)
    x = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, level + 1, 300 + level, x)
    y = torch.full_like(x, float("nan"))
    P.apply_p2(m, level, x, y)
    torch.cuda.synchronize()
    xo = om.keyed_random(300 + level)
    assert np.array_equal(x.cpu().numpy(), xo[s2u]), "keyed generators disagree"
    yo = om.spmv_p2(xo, dirichlet=dirichlet)
    ys = y.cpu().numpy()
    assert np.isfinite(ys).all()
    assert harness.copies_consistent(ys, s2u)
    assert harness.rel_err_max(ys, yo[s2u]) <= 1e-12


@pytest.mark.parametrize("name,level", [("tri_affine", 6), ("strip2d_shuf", 5)])
def test_p2_apply_fp32_within_rounding_bound(name, level):
    m, om, s2u = _setup(name, level)
    s, _ = P.mesh_num_dofs(m, level + 1)
    x = torch.empty(s, dtype=torch.float32, device="cuda")
    P.mesh_fill_random(m, level + 1, 9, x)
    y = torch.empty_like(x)
    P.apply_p2(m, level, x, y)
    torch.cuda.synchronize()
    xo = om.keyed_random(9).astype(np.float32).astype(np.float64)
    A = om.csr_p2(dirichlet=True)
    yo = A @ xo
    bound = 32 * U32 * (abs(A) @ np.abs(xo))
    ys = y.cpu().numpy().astype(np.float64)
    assert harness.copies_consistent(y.cpu().numpy(), s2u)
    assert (np.abs(ys - yo[s2u]) <= bound[s2u] + 1e-30).all()


def test_p2_rejects_bad_calls():
    m3 = P.create_macro_mesh(*W.unit_tet(), 2)
    x = torch.zeros(P.mesh_num_dofs(m3, 2)[0], dtype=torch.float64, device="cuda")
    with pytest.raises(P.MFError, match=r"\[-4\]"):
        P.apply_p2(m3, 1, x, torch.empty_like(x))
    m2 = P.create_macro_mesh(*W.unit_triangle(), 3)
    x = torch.zeros(P.mesh_num_dofs(m2, 3)[0], dtype=torch.float64, device="cuda")
    with pytest.raises(P.MFError, match=r"\[-1\]"):
        P.apply_p2(m2, 3, x, torch.empty_like(x))  # would need level 4
    with pytest.raises(P.MFError, match=r"\[-1\]"):
        P.apply_p2(m2, 2, x, x)
    torch.cuda.synchronize()


def _lattice(M):
    """Fine-lattice coordinates (X, Y) of every storage point of one macro."""
    rows = torch.arange(M + 1, device="cuda", dtype=torch.int64)
    lengths = M + 1 - rows
    Y = torch.repeat_interleave(rows, lengths)
    start = torch.cumsum(lengths, 0) - lengths
    X = torch.arange(int(lengths.sum()), device="cuda", dtype=torch.int64) - start[Y]
    return X, Y


@pytest.mark.parametrize("level", [6, 13, 14])
def test_p2_full_size_quadratic_rows(level):
    """Benchmark size (level 13) and the largest level (14, on the level-15
    lattice): the whole output checked against the closed form."""
    co, ce = W.affine_triangle(2)
    m = P.create_macro_mesh(co, ce, level + 1)
    M = 1 << (level + 1)
    X, Y = _lattice(M)
    assert X.numel() == P.mesh_num_dofs(m, level + 1)[0]
    P0, P1, P2 = (torch.tensor(co[i], device="cuda") for i in ce[0])
    u, v = X.double() / M, Y.double() / M
    px = P0[0] + u * (P1[0] - P0[0]) + v * (P2[0] - P0[0])
    py = P0[1] + u * (P1[1] - P0[1]) + v * (P2[1] - P0[1])
    del u, v
    x = px * px + 3.0 * px * py - 2.0 * py * py + px  # Laplace = -2
    del px, py
    y = torch.full_like(x, float("nan"))
    P.apply_p2(m, level, x, y)
    torch.cuda.synchronize()
    N = M // 2
    area = 0.5 * abs(np.linalg.det(np.array([co[ce[0][1]] - co[ce[0][0]], co[ce[0][2]] - co[ce[0][0]]])))
    edge_row = 2.0 * 2.0 * (area / N ** 2) / 3.0  # -Laplace(q) * (|T1| + |T2|) / 3
    inner = (X >= 1) & (Y >= 1) & (X + Y <= M - 1)
    vert = (X % 2 == 0) & (Y % 2 == 0)
    expect = torch.where(inner, torch.where(vert, torch.zeros_like(x), torch.full_like(x, edge_row)), x)
    assert torch.isfinite(y).all()
    err = (y - expect).abs().max().item()
    assert err <= 1e-12, err
    assert (y[~inner] == x[~inner]).all()


def test_p2_fp32_full_size_quadratic_rows():
    """Benchmark size in FP32 (P2 level 13): the quadratic's interpolant gives
    interior vertex rows 0 and interior edge rows -Laplace(q) times the basis
    integral, to FP32 rounding of rows whose terms are O(1); Dirichlet rows
    copy x exactly."""
    level = 13
    co, ce = W.affine_triangle(2)
    m = P.create_macro_mesh(co, ce, level + 1)
    M = 1 << (level + 1)
    X, Y = _lattice(M)
    P0, P1, P2 = (torch.tensor(co[i], device="cuda") for i in ce[0])
    u, v = X.double() / M, Y.double() / M
    px = P0[0] + u * (P1[0] - P0[0]) + v * (P2[0] - P0[0])
    py = P0[1] + u * (P1[1] - P0[1]) + v * (P2[1] - P0[1])
    del u, v
    x = (px * px + 3.0 * px * py - 2.0 * py * py + px).float()
    del px, py
    y = torch.full_like(x, float("nan"))
    P.apply_p2(m, level, x, y)
    torch.cuda.synchronize()
    N = M // 2
    area = 0.5 * abs(np.linalg.det(np.array([co[ce[0][1]] - co[ce[0][0]], co[ce[0][2]] - co[ce[0][0]]])))
    edge_row = 2.0 * 2.0 * (area / N ** 2) / 3.0
    inner = (X >= 1) & (Y >= 1) & (X + Y <= M - 1)
    vert = (X % 2 == 0) & (Y % 2 == 0)
    expect = torch.where(vert, torch.zeros_like(y, dtype=torch.float64), torch.full_like(y, edge_row, dtype=torch.float64))
    assert bool(torch.isfinite(y).all())
    assert bool((y[~inner] == x[~inner]).all())
    # rows add up to 19 terms of size about |w| |x| with |x| <= 6 and |w| <= 8/3:
    # FP32 rounding of the inputs and the sums bounds the error by about 1e-4
    err = (y[inner].double() - expect[inner]).abs().max().item()
    assert err <= 2e-4, err
