"""Serving loop on the GPU: batched and plain servers return what solving
each request alone returns, bitwise; oversize requests are rejected."""
import pytest

import paper_2305_15116_amd as P
from paper_2305_15116_amd import loadgen, serving

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    yield
    torch.cuda.synchronize()


def _alone(r, mode, max_iter):
    m = P.create_macro_mesh(r.coords, r.cells, r.level)
    s, _ = P.mesh_num_dofs(m, r.level)
    b = torch.empty(s, dtype=torch.float64, device="cuda")
    P.mesh_fill_random(m, r.level, r.rhs_seed, b)
    P.mesh_set_dirichlet(m, r.level, None, b)
    x = torch.zeros_like(b)
    ws = torch.empty(P.mesh_workspace_bytes(m, r.level, mode), dtype=torch.uint8, device="cuda")
    rc, it, rel, _ = P.vcycle_solve(m, r.level, b, x, ws, mode=mode, rtol=r.tol, max_iter=max_iter)
    torch.cuda.synchronize()
    return rc, it, x


@pytest.mark.parametrize("batched,split", [(True, 4_000_000), (True, 3000), (False, 0)])
def test_server_equals_solving_alone(batched, split):
    """split: requests of at least that many storage DoFs step in the second lane."""
    reqs = loadgen.requests(n=14, rate=500.0, levels2=(2, 6), levels3=(1, 4), kmax=7, tol=1e-8, seed_arrival=3,
                            seed_req=4)
    srv = serving.Server(4 << 30, batched=batched, max_batch=6, max_iter=200, split_dofs=split)
    futs, _, _ = loadgen.replay(srv, reqs)
    out = [f.result(timeout=100) for f in futs]
    srv.close()
    assert srv.completed == len(reqs) and srv.rejected == 0
    if batched and split == 3000:
        assert min(srv.lane_busy_s) > 0.0  # both lanes served requests
    for r, (x, info) in zip(reqs, out):
        rc, it, xa = _alone(r, srv.mode, 200)
        assert (info["status"], info["iters"]) == (rc, it)
        assert torch.equal(x, xa)
        assert info["t_done"] >= info["t_admit"] >= info["t_arrival"] - 1e-3


def test_oversize_request_is_rejected():
    reqs = loadgen.requests(n=3, rate=500.0, levels2=(4, 4), levels3=(3, 3), kmax=2)
    srv = serving.Server(1 << 20, batched=True)
    futs, _, _ = loadgen.replay(srv, reqs)
    for f in futs:
        with pytest.raises(P.MFError) as e:
            f.result(timeout=30)
        assert e.value.code == P.MF_ENOMEM
    srv.close()
    assert srv.rejected == 3
