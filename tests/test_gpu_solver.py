"""GPU multigrid solves through the C ABI, checked by the oracle.

A solve is accepted when the oracle's own CSR recomputes its FP64 residual
||b - A x|| / ||b|| <= rtol (to rounding), and, for the manufactured problem
on meshes where the discrete solution has a closed form, when x matches that
solution within kappa * rtol.
"""
import numpy as np
import pytest

import harness
import paper_2305_15116_amd as P
from oracle.oracle import OracleMesh, solve
from paper_2305_15116_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    yield
    torch.cuda.synchronize()


def _manufactured(co, ce, L):
    """b = lumped mass * d pi^2 u* with u* = prod sin(pi x_k) (zero on the
    unit square / cube boundary), in storage layout, and the oracle mesh."""
    m = P.create_macro_mesh(co, ce, L)
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    xyz = om.xyz()
    dim = co.shape[1]
    us = np.prod(np.sin(np.pi * xyz), axis=1)
    bu = om.lumped_mass() * dim * np.pi ** 2 * us
    bu[om.boundary()] = 0.0
    return m, om, s2u, bu, us


@pytest.mark.parametrize("mesh,L,mode", [("cube", 4, 0), ("cube", 4, 1), ("cube", 5, 1), ("square", 6, 0),
                                         ("square", 6, 1), ("cube", 4, 2), ("cube", 5, 3), ("square", 6, 2),
                                         ("square", 6, 3), ("cube", 4, 4), ("cube", 5, 5), ("square", 6, 4),
                                         ("square", 6, 5)])
def test_manufactured_solution(mesh, L, mode):
    co, ce = W.kuhn_cube() if mesh == "cube" else W.two_triangle_square()
    m, om, s2u, bu, us = _manufactured(co, ce, L)
    b = torch.as_tensor(bu[s2u], device="cuda")
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10)
    torch.cuda.synchronize()
    assert rc == P.MF_OK and rel <= 1e-10
    xs = x.cpu().numpy()
    assert harness.copies_consistent(xs, s2u)
    xu = np.zeros(om.n)
    xu[s2u] = xs
    r = bu - om.spmv(xu)
    res = np.linalg.norm(r) / np.linalg.norm(bu)
    assert res <= 1.01e-10
    # every mode reports the true residual b - A x, not a recurred one
    assert abs(rel - res) <= 1e-2 * res, (rel, res)
    h = 1.0 / om.N
    uh = us * (np.pi ** 2 * h ** 2 / 4) / np.sin(np.pi * h / 2) ** 2
    uh[om.boundary()] = 0.0
    # kappa(A) <= ~ (4/(pi h))^2 bounds the error of a 1e-10 residual
    kappa = (4.0 / (np.pi * h)) ** 2
    assert np.abs(xu - uh).max() <= 2 * kappa * 1e-10 * np.abs(uh).max()


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_random_mesh_against_oracle_solve(mode):
    co, ce = W.kuhn_cube("random", 5)
    J, t = W.random_affine(3, 8)
    co = W.apply_affine(co, J, t)
    L = 4
    m = P.create_macro_mesh(co, ce, L)
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 31, b)
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    # stretched (cond J up to 10), randomly ordered tets slow point-Jacobi
    # multigrid down, but it still converges
    rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10, max_iter=2000)
    torch.cuda.synchronize()
    assert rc == P.MF_OK, (it, rel)
    bo = om.keyed_random(31)
    uo = solve(om, bo, tol=1e-14)
    xu = np.zeros(om.n)
    xu[s2u] = x.cpu().numpy()
    r = bo - om.spmv(xu)
    res = np.linalg.norm(r) / np.linalg.norm(bo)
    assert res <= 1.01e-10
    assert abs(rel - res) <= 1e-2 * res, (rel, res)
    # Dirichlet values are exactly b's
    bnd = om.boundary()
    assert np.array_equal(xu[bnd], bo[bnd])
    kappa_bound = 1e5
    assert np.abs(xu - uo).max() <= kappa_bound * 1e-10 * max(1.0, np.abs(uo).max())


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_tail_levels_in_lds_and_in_global_memory(mode):
    """16 triangles at level 5: the one-workgroup bottom of the cycle takes
    levels 2-4 (240, 720 and 2,448 storage points), whose b, x and t need
    81,792 bytes in FP64 cycles (more than the 64 KiB the kernel keeps in LDS:
    they stay in global memory, modes 0 and 2) and 40,896 bytes in FP32 cycles
    (held in LDS, modes 1 and 3).  Both forms must solve to the tolerance on
    the oracle's matrix."""
    co, ce = W.strip_2d(16)
    J, t = W.random_affine(2, 12)
    co = W.apply_affine(co, J, t)
    L = 5
    m = P.create_macro_mesh(co, ce, L)
    assert [P.mesh_num_dofs(m, k)[0] for k in (2, 3, 4, 5)] == [240, 720, 2448, 8976]
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 33, b)
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10, max_iter=2000)
    torch.cuda.synchronize()
    assert rc == P.MF_OK, (it, rel)
    bo = om.keyed_random(33)
    xu = np.zeros(om.n)
    xu[s2u] = x.cpu().numpy()
    res = np.linalg.norm(bo - om.spmv(xu)) / np.linalg.norm(bo)
    assert res <= 1.01e-10
    assert abs(rel - res) <= 1e-2 * res, (rel, res)


# refinement (modes 0, 1) takes any sweep counts; conjugate gradients (modes
# 2, 3) needs a symmetric preconditioner, so equal pre- and post-sweeps
CYCLES = [("strip2d", 6, 0, 2, None, 1), ("strip2d", 6, 1, 1, 1, 0), ("strip2d", 6, 3, 3, None, 3),
          ("strip2d", 6, 2, 0, 3, 0), ("strip3d", 5, 0, 2, None, 1), ("strip3d", 5, 1, 1, 1, 3),
          ("strip3d", 5, 3, 2, 3, 0), ("strip3d", 4, 2, 2, 0, 2)]


@pytest.mark.parametrize("mesh,L,pre,post,lc,mode", CYCLES)
def test_cycle_shapes_against_oracle(mesh, L, pre, post, lc, mode):
    """Odd, zero and unequal sweep counts and other coarse levels: the small
    levels of these meshes run in the one-workgroup bottom of the cycle, the
    larger ones as separate launches."""
    co, ce = W.strip_2d(5) if mesh == "strip2d" else W.strip_3d(3)
    J, t = W.random_affine(co.shape[1], 4)
    co = W.apply_affine(co, J, t)
    m = P.create_macro_mesh(co, ce, L)
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 41, b)
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    rc, it, rel, sec = P.vcycle_solve(m, L, b, x, ws, mode=mode, pre=pre, post=post, coarse_level=lc, rtol=1e-10,
                                      max_iter=1000)
    torch.cuda.synchronize()
    assert rc == P.MF_OK, (it, rel)
    bo = om.keyed_random(41)
    xu = np.zeros(om.n)
    xs = x.cpu().numpy()
    assert harness.copies_consistent(xs, s2u)
    xu[s2u] = xs
    r = bo - om.spmv(xu)
    assert np.linalg.norm(r) / np.linalg.norm(bo) <= 1.01e-10
    bnd = om.boundary()
    assert np.array_equal(xu[bnd], bo[bnd])
    uo = solve(om, bo, tol=1e-14)
    assert np.abs(xu - uo).max() <= 1e5 * 1e-10 * max(1.0, np.abs(uo).max())


def test_split_solve_equals_single_solve():
    """Checkpoint/resume (iterative refinement): k/2 + k/2 iterations from the saved x equal k
    iterations, bitwise."""
    co, ce = W.strip_3d(7)
    L = 4
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 5, b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, 1), dtype=torch.uint8, device="cuda")
    x1 = torch.zeros_like(b)
    rc, it, rel, _ = P.vcycle_solve(m, L, b, x1, ws, mode=1, rtol=0.0, max_iter=6)
    assert rc == P.MF_NOT_CONVERGED and it == 6
    x2 = torch.zeros_like(b)
    P.vcycle_solve(m, L, b, x2, ws, mode=1, rtol=0.0, max_iter=3)
    P.vcycle_solve(m, L, b, x2, ws, mode=1, rtol=0.0, max_iter=3)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2)


def test_cg_rejects_a_non_symmetric_cycle():
    co, ce = W.two_triangle_square()
    m = P.create_macro_mesh(co, ce, 3)
    s, _ = P.mesh_num_dofs(m, 3)
    b = torch.ones(s, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, 3, 2), dtype=torch.uint8, device="cuda")
    for mode in (2, 3, 4, 5):
        with pytest.raises(P.MFError) as e:
            P.vcycle_solve(m, 3, b, x, ws, mode=mode, pre=2, post=1)
        assert e.value.code == P.MF_EINVAL
        with pytest.raises(P.MFError) as e:
            P.batch_create(1, mode=mode, pre=1, post=2)
        assert e.value.code == P.MF_EINVAL
    # MINRES is not batched
    for mode in (4, 5):
        with pytest.raises(P.MFError) as e:
            P.batch_create(1, mode=mode)
        assert e.value.code == P.MF_EINVAL
    # refinement takes any sweep counts
    rc, it, rel, _ = P.vcycle_solve(m, 3, b, x, ws, mode=0, pre=2, post=1, rtol=1e-8)
    torch.cuda.synchronize()
    assert rc == P.MF_OK and rel <= 1e-8


def test_nan_rhs_is_reported():
    co, ce = W.two_triangle_square()
    L = 4
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.zeros(s, dtype=torch.float64, device="cuda")
    b[s // 2] = float("nan")
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, 0), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.MFError) as e:
        P.vcycle_solve(m, L, b, x, ws, mode=0)
    assert e.value.code == P.MF_ENUMERIC


def test_zero_rhs_converges_immediately():
    co, ce = W.kuhn_cube()
    m = P.create_macro_mesh(co, ce, 3)
    s, _ = P.mesh_num_dofs(m, 3)
    b = torch.zeros(s, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, 3, 1), dtype=torch.uint8, device="cuda")
    rc, it, rel, _ = P.vcycle_solve(m, 3, b, x, ws, mode=1)
    assert rc == P.MF_OK and it == 0 and float(x.abs().max()) == 0.0


@pytest.mark.parametrize("L", [0, 1, 2])
def test_coarse_levels_solve_directly(L):
    co, ce = W.strip_2d(6)
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 3, b)
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, 0), dtype=torch.uint8, device="cuda")
    rc, it, rel, _ = P.vcycle_solve(m, L, b, x, ws, mode=0, rtol=1e-12)
    assert rc == P.MF_OK and it <= 2


@pytest.mark.parametrize("mode", [2, 3])
def test_pcg_needs_fewer_iterations_on_a_stretched_mesh(mode):
    """Conjugate gradients around the V-cycle against refinement with the same
    V-cycle on a stretched 2D strip: same tolerance, fewer iterations."""
    co, ce = W.strip_2d(4)
    J, t = W.random_affine(2, 2)
    co = W.apply_affine(co, J, t)
    L = 7
    m = P.create_macro_mesh(co, ce, L)
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 9, b)
    P.mesh_set_dirichlet(m, L, None, b)
    its = {}
    for md in (mode - 2, mode):
        x = torch.zeros_like(b)
        ws = torch.empty(P.mesh_workspace_bytes(m, L, md), dtype=torch.uint8, device="cuda")
        rc, it, rel, _ = P.vcycle_solve(m, L, b, x, ws, mode=md, rtol=1e-8, max_iter=300)
        assert rc == P.MF_OK and rel <= 1e-8
        its[md] = it
    assert its[mode] < its[mode - 2]


@pytest.mark.parametrize("mode", [4, 5])
def test_minres_stopped_early_reports_the_true_residual(mode):
    """MINRES cut off after a few iterations: MF_NOT_CONVERGED, and rel_res
    is the FP64 residual of the returned x as the oracle's matrix gives it;
    more iterations give a smaller residual (MINRES minimises sqrt(r . M r),
    M the V-cycle, over a growing Krylov space)."""
    co, ce = W.kuhn_cube("random", 7)
    L = 4
    m = P.create_macro_mesh(co, ce, L)
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 35, b)
    bo = om.keyed_random(35)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    rels = []
    for k in (2, 4, 8):
        x = torch.zeros_like(b)
        rc, it, rel, _ = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-14, max_iter=k)
        torch.cuda.synchronize()
        assert rc == P.MF_NOT_CONVERGED and it == k
        xu = np.zeros(om.n)
        xu[s2u] = x.cpu().numpy()
        res = np.linalg.norm(bo - om.spmv(xu)) / np.linalg.norm(bo)
        assert abs(rel - res) <= 1e-6 * res, (k, rel, res)
        rels.append(res)
    assert rels[0] > rels[1] > rels[2], rels


def test_minres_and_cg_take_similar_iterations():
    """On this symmetric positive definite operator MINRES with the V-cycle
    needs about as many iterations as CG with it (both minimise over the same
    Krylov space, in different norms)."""
    co, ce = W.kuhn_cube()
    m, om, s2u, bu, us = _manufactured(co, ce, 5)
    b = torch.as_tensor(bu[s2u], device="cuda")
    its = {}
    for mode in (2, 4, 3, 5):
        x = torch.zeros_like(b)
        ws = torch.empty(P.mesh_workspace_bytes(m, 5, mode), dtype=torch.uint8, device="cuda")
        rc, it, rel, _ = P.vcycle_solve(m, 5, b, x, ws, mode=mode, rtol=1e-10)
        torch.cuda.synchronize()
        assert rc == P.MF_OK and rel <= 1e-10
        its[mode] = it
    assert abs(its[4] - its[2]) <= 3 and abs(its[5] - its[3]) <= 3, its


@pytest.mark.parametrize("mode", [4, 5])
def test_minres_from_a_nonzero_guess_is_deterministic(mode):
    """MINRES from a random initial guess on a randomly mapped 2D strip: the
    oracle's matrix gives a residual within the tolerance, the Dirichlet
    entries are b's, and a second solve from the same guess is bitwise the
    same (every reduction has a fixed order)."""
    co, ce = W.strip_2d(6)
    J, t = W.random_affine(2, 21)
    co = W.apply_affine(co, J, t)
    L = 6
    m = P.create_macro_mesh(co, ce, L)
    om = OracleMesh(co, ce, L)
    s2u = harness.storage_to_unique(P.mesh_dof_keys(m, L), om.keys())
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, L, 37, b)
    x0 = torch.empty_like(b)
    P.mesh_fill_random(m, L, 38, x0)
    ws = torch.empty(P.mesh_workspace_bytes(m, L, mode), dtype=torch.uint8, device="cuda")
    xs = []
    for _ in range(2):
        x = x0.clone()
        rc, it, rel, _ = P.vcycle_solve(m, L, b, x, ws, mode=mode, rtol=1e-10, max_iter=500)
        torch.cuda.synchronize()
        assert rc == P.MF_OK, (it, rel)
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
    bo = om.keyed_random(37)
    xu = np.zeros(om.n)
    xu[s2u] = xs[0].cpu().numpy()
    res = np.linalg.norm(bo - om.spmv(xu)) / np.linalg.norm(bo)
    assert res <= 1.01e-10
    bnd = om.boundary()
    assert np.array_equal(xu[bnd], bo[bnd])
