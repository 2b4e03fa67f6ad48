"""Full-size checks in the benchmark's launch configuration.

At the benchmark sizes (one affine triangle at level 14, 134,242,305 DoFs;
the 6-tet unit cube at level 8, 17,173,254 storage DoFs) the oracle cannot
assemble the whole matrix, so sampled rows are recomputed one by one by the
oracle's row evaluator (same keyed input), and properties that hold at any
size are checked on every row.
"""
import numpy as np
import pytest

import paper_2305_15116_amd as P
from oracle.oracle import sample_rows
from paper_2305_15116_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    yield
    torch.cuda.synchronize()


def _samples_2d(N, rng, n=3000):
    pts = []
    for _ in range(n):
        y = int(rng.integers(0, N + 1))
        pts.append((int(rng.integers(0, N + 1 - y)), y))
    for k in range(0, N + 1, 62):      # tile column edges
        for y in (1, 2, 63, 64, 65, 128):
            for x in (k - 1, k, k + 1, k + 2):
                if 0 <= x and x + y <= N:
                    pts.append((x, y))
    for y in range(0, N + 1, max(1, N // 64)):  # hypotenuse band and the legs
        for x in (N - y, N - y - 1, N - y - 2, 0, 1):
            if 0 <= x and x + y <= N:
                pts.append((x, y))
    pts += [(0, 0), (N, 0), (0, N), (1, 1), (N - 2, 1), (1, N - 2)]
    return np.array(pts, dtype=np.int64)


def _samples_3d(N, nc, rng, n=3000):
    pts = []
    for _ in range(n):
        c = int(rng.integers(0, nc))
        z = int(rng.integers(0, N + 1))
        y = int(rng.integers(0, N + 1 - z))
        x = int(rng.integers(0, N + 1 - z - y))
        pts.append((c, x, y, z))
    for c in range(nc):
        for z in (0, 1, 2, N // 2, N - 3, N - 2, N - 1, N):
            M = N - z
            for y in (0, 1, 16, 17, M // 2, M - 1, M):
                for x in (0, 1, 61, 62, 63, M - y - 1, M - y):
                    if 0 <= y <= M and 0 <= x and x + y <= M:
                        pts.append((c, x, y, z))
    return np.array(pts, dtype=np.int64)


def _check_sampled(co, ce, m, L, y, seed, pts_ml, tol):
    idx = P.mesh_dof_index(m, L, pts_ml)
    got = y[torch.as_tensor(idx, device="cuda")].double().cpu().numpy()
    dim = co.shape[1]
    yo, bnd = sample_rows(co, ce, L, seed, pts_ml[:, 0], pts_ml[:, 1:1 + dim])
    scale = np.abs(yo).max()
    return np.abs(got - yo), scale, bnd


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_2d_level14_affine_triangle(dtype):
    co, ce = W.affine_triangle(2)
    L = 14
    N = 1 << L
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    assert s == u == (N + 1) * (N + 2) // 2 == 134242305
    x = torch.empty(s, dtype=dtype, device="cuda")
    P.mesh_fill_random(m, L, 3, x)
    y = torch.empty_like(x)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(42)
    pts = _samples_2d(N, rng)
    ml = np.hstack([np.zeros((len(pts), 1), np.int64), pts])
    err, scale, _ = _check_sampled(co, ce, m, L, y, 3, ml, None)
    if dtype == torch.float64:
        assert err.max() <= 1e-12 * scale
    else:
        w = np.abs(P.mesh_stencil(m, L, 0)).sum()
        assert err.max() <= 16 * U32 * w
    # A 1 = 0 on interior rows and 1 on the boundary, checked on every row
    x.fill_(1.0)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    wsum = np.abs(P.mesh_stencil(m, L, 0)).sum()
    yb = y.double()
    bidx = torch.as_tensor(P.mesh_dof_index(m, L, np.array(
        [[0, xx, 0] for xx in range(N + 1)] + [[0, 0, yy] for yy in range(1, N + 1)] +
        [[0, N - yy, yy] for yy in range(1, N)])), device="cuda")
    assert torch.all(yb[bidx] == 1.0)
    yb[bidx] = 0.0
    tol = 1e-12 if dtype == torch.float64 else 16 * U32
    assert float(yb.abs().max()) <= tol * wsum


@pytest.mark.parametrize("order", ["canonical", "random"])
def test_3d_level8_cube(order):
    co, ce = W.kuhn_cube(order, 5)
    L = 8
    N = 1 << L
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    assert s == 17173254 and u == 16974593
    x = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 4, x)
    y = torch.empty_like(x)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(43)
    ml = _samples_3d(N, 6, rng)
    err, scale, bnd = _check_sampled(co, ce, m, L, y, 4, ml, None)
    assert err.max() <= 1e-12 * scale
    if order == "canonical":
        # every non-boundary row is h (6 x_c - sum of axis neighbours): A 1 = 0 there, and
        # A applied to x = 1 gives exactly 1 on the Dirichlet rows
        x.fill_(1.0)
        P.apply_stencil(m, L, x, y)
        torch.cuda.synchronize()
        h = 1.0 / N
        assert float((y - torch.where(y == 1.0, y, torch.zeros_like(y))).abs().max()) <= 1e-12 * 12 * h


def test_2d_level15_largest_supported_level():
    """Level 15 (537,001,985 DoFs, 4.3 GB per FP64 vector) is the largest 2D
    level: row offsets inside a macro reach 2^29, near the 32-bit index limit.
    Sampled rows against the oracle's row evaluator, and A 1 on every row."""
    co, ce = W.affine_triangle(2)
    L = 15
    N = 1 << L
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    assert s == u == (N + 1) * (N + 2) // 2
    x = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 8, x)
    y = torch.empty_like(x)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    pts = _samples_2d(N, rng, n=2000)
    ml = np.hstack([np.zeros((len(pts), 1), np.int64), pts])
    err, scale, _ = _check_sampled(co, ce, m, L, y, 8, ml, None)
    assert err.max() <= 1e-12 * scale
    x.fill_(1.0)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    wsum = np.abs(P.mesh_stencil(m, L, 0)).sum()
    y[y == 1.0] = 0.0  # Dirichlet rows
    assert float(y.abs().max()) <= 1e-12 * wsum


def test_3d_level11_largest_supported_level():
    """Level 11 (one tetrahedron: 1,435,853,825 DoFs, 11.5 GB per FP64 vector)
    is the largest 3D level: slice offsets exceed 2^30.  Sampled rows against
    the oracle's row evaluator, and A 1 on every row."""
    co, ce = W.unit_tet()
    J, t = W.random_affine(3, 7)
    co = W.apply_affine(co, J, t)
    L = 11
    N = 1 << L
    m = P.create_macro_mesh(co, ce, L)
    s, u = P.mesh_num_dofs(m, L)
    assert s == u == (N + 1) * (N + 2) * (N + 3) // 6
    x = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 9, x)
    y = torch.empty_like(x)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(45)
    ml = _samples_3d(N, 1, rng, n=2000)
    err, scale, _ = _check_sampled(co, ce, m, L, y, 9, ml, None)
    assert err.max() <= 1e-12 * scale
    x.fill_(1.0)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    wsum = np.abs(P.mesh_stencil(m, L, 0)).sum()
    y[y == 1.0] = 0.0  # Dirichlet rows
    assert float(y.abs().max()) <= 1e-12 * wsum


def _local_coords(dim, N, nmac):
    """Macro-local lattice coordinates (x, y, z) of every storage point of a
    level (macros stored one after the other), as int64 tensors."""
    def tri(S):
        rows = torch.arange(S + 1, device="cuda", dtype=torch.int64)
        lengths = S + 1 - rows
        y = torch.repeat_interleave(rows, lengths)
        x = torch.arange(int(lengths.sum()), device="cuda", dtype=torch.int64) - (torch.cumsum(lengths, 0) - lengths)[y]
        return x, y
    if dim == 2:
        x, y = tri(N)
        z = torch.zeros_like(x)
    else:
        parts = [tri(N - k) + (torch.full(((N - k + 1) * (N - k + 2) // 2,), k, device="cuda", dtype=torch.int64),)
                 for k in range(N + 1)]
        x, y, z = (torch.cat([p[i] for p in parts]) for i in range(3))
    return x.repeat(nmac), y.repeat(nmac), z.repeat(nmac)


@pytest.mark.parametrize("dim,L,dtype", [(2, 15, torch.float64), (3, 8, torch.float32), (3, 8, torch.float64)])
def test_transfers_full_size(dim, L, dtype):
    """Prolongation and restriction over every point of the largest 2D level
    and the benchmark cube, by properties exact in floating point: the P1
    interpolant of an integer linear function of the macro-local coordinates
    (every non-Dirichlet fine point gets the function's value, Dirichlet
    points keep theirs), and the restriction of the constant 1 (interior
    coarse points gather 1 + 6/2 in 2D, 1 + 14/2 in 3D)."""
    co, ce = W.affine_triangle(2) if dim == 2 else W.kuhn_cube()
    m = P.create_macro_mesh(co, ce, L)
    nmac = len(ce)
    Nf, Nc = 1 << L, 1 << (L - 1)
    sf, _ = P.mesh_num_dofs(m, L)
    sc, _ = P.mesh_num_dofs(m, L - 1)
    xc, yc, zc = _local_coords(dim, Nc, nmac)
    ec = (6 * xc + 10 * yc + 14 * zc).to(dtype)
    del xc, yc, zc
    xf = torch.zeros(sf, dtype=dtype, device="cuda")
    P.prolong_add(m, L, ec, xf)
    torch.cuda.synchronize()
    fx, fy, fz = _local_coords(dim, Nf, nmac)
    want = (3 * fx + 5 * fy + 7 * fz).to(dtype)
    # Dirichlet fine points: the domain boundary, where prolongation leaves x alone
    ones = torch.ones(sf, dtype=dtype, device="cuda")
    dirichlet = torch.empty_like(ones)
    P.mesh_set_dirichlet(m, L, None, dirichlet.copy_(ones))
    dirichlet = dirichlet == 0
    assert bool((xf[~dirichlet] == want[~dirichlet]).all())
    assert bool((xf[dirichlet] == 0).all())
    del want, dirichlet
    bc = torch.full((sc,), float("nan"), dtype=dtype, device="cuda")
    P.restrict_residual(m, L, ones, bc)
    torch.cuda.synchronize()
    del fx, fy, fz
    xc, yc, zc = _local_coords(dim, Nc, nmac)
    inner = (xc >= 1) & (yc >= 1) & (xc + yc + zc <= Nc - 1)
    if dim == 3:
        inner &= zc >= 1
    assert bool(torch.isfinite(bc).all())
    assert bool((bc[inner] == (4.0 if dim == 2 else 8.0)).all())


@pytest.mark.parametrize("order", ["canonical", "random"])
def test_3d_level8_cube_fp32(order):
    """The FP32 3D apply (the mixed solver's sweeps) on the benchmark cube:
    sampled rows against the oracle's FP64 rows of the same (FP32-rounded)
    keyed input, within 16 u32 of the row's absolute weight sum."""
    co, ce = W.kuhn_cube(order, 5)
    L = 8
    N = 1 << L
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    x = torch.empty(s, dtype=torch.float32, device="cuda")
    P.mesh_fill_random(m, L, 4, x)
    y = torch.empty_like(x)
    P.apply_stencil(m, L, x, y)
    torch.cuda.synchronize()
    rng = np.random.default_rng(46)
    ml = _samples_3d(N, 6, rng)
    err, scale, _ = _check_sampled(co, ce, m, L, y, 4, ml, None)
    w = max(np.abs(P.mesh_stencil(m, L, c)).sum() for c in range(6))
    # the oracle evaluates the FP64 input; FP32 rounding of x (u32 |x|) and of
    # the 15-term sums stays within a few u32 of sum |w|
    assert err.max() <= 16 * U32 * w, (err.max(), w)
