"""Host-side parts of the serving loop: workload generator and admission footprint."""
import numpy as np
import pytest

import paper_2305_15116_amd as P
from paper_2305_15116_amd import loadgen, serving


def test_requests_are_seeded_and_shaped():
    a = loadgen.requests(n=50, rate=200.0)
    b = loadgen.requests(n=50, rate=200.0)
    assert [(r.t, r.dim, r.k, r.level, r.rhs_seed) for r in a] == [(r.t, r.dim, r.k, r.level, r.rhs_seed) for r in b]
    assert all(np.array_equal(x.coords, y.coords) for x, y in zip(a, b))
    t = np.array([r.t for r in a])
    assert np.all(np.diff(t) > 0)
    for r in a:
        assert r.dim in (2, 3) and 1 <= r.k <= 64 and 5 <= r.level <= 11
        assert r.cells.shape == (r.k, r.dim + 1)
        assert r.tol == 1e-8
    capped = loadgen.requests(n=200, levels3=(5, 8))
    assert max(r.level for r in capped if r.dim == 3) <= 8


def test_mean_gap_matches_rate():
    r = loadgen.requests(n=2000, rate=200.0)
    assert abs(r[-1].t / 2000 - 1 / 200.0) < 0.1 / 200.0


@pytest.mark.parametrize("dim,k,level", [(2, 1, 3), (2, 7, 6), (3, 1, 2), (3, 5, 4), (3, 13, 5)])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_footprint_covers_what_the_solver_needs(dim, k, level, mode):
    from paper_2305_15116_amd import workloads as W
    co, ce = W.strip_2d(k) if dim == 2 else W.strip_3d(k)
    m = P.create_macro_mesh(co, ce, level, flags=P.MF_FLAG_DIRICHLET | P.MF_FLAG_HOST_ONLY)
    s, _ = P.mesh_num_dofs(m, level)
    assert s == serving.storage_dofs(dim, k, level)
    need = 16 * s + P.mesh_workspace_bytes(m, level, mode)
    fp = serving.footprint_bytes(dim, k, level, mode)
    assert need <= fp <= 1.35 * need + (2 << 20) + 4096 * k * (level + 1)
