"""residual_noalloc (norm partials in the library's static device scratch)
against residual (partials in the mesh's buffers), through the C ABI.

Both run the same kernels over the same partial layout, so r and the norm
must agree bitwise.  Two calls in a row, the second on a smaller input (the
scratch keeps the first call's contents, which the second must not read),
then a level whose partials exceed the scratch maximum.
"""
import ctypes as C

import pytest

import paper_2305_15116_amd as P
from paper_2305_15116_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _vectors(m, L, dtype, seed):
    s, _ = P.mesh_num_dofs(m, L)
    b = torch.empty(s, dtype=dtype, device="cuda")
    x = torch.empty_like(b)
    P.mesh_fill_random(m, L, seed, b)
    P.mesh_fill_random(m, L, seed + 1, x)
    return b, x


def _call(name, m, L, b, x, r):
    n2 = C.c_double(float("nan"))
    code = P.MF_F64 if x.dtype == torch.float64 else P.MF_F32
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(P.lib(), name)(m, L, code, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                C.c_void_p(r.data_ptr()), C.byref(n2), stream)
    return rc, n2.value


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_residual_equals_residual(dtype):
    cases = [(W.kuhn_cube("random", 5), 6), (W.strip_2d(3), 5)]  # the second input is smaller
    for (co, ce), L in cases:
        m = P.create_macro_mesh(co, ce, L)
        b, x = _vectors(m, L, dtype, 90 + L)
        r0 = torch.full_like(b, float("nan"))
        r1 = torch.full_like(b, float("nan"))
        rc0, n0 = _call("residual", m, L, b, x, r0)
        rc1, n1 = _call("residual_noalloc", m, L, b, x, r1)
        torch.cuda.synchronize()
        assert rc0 == P.MF_OK and rc1 == P.MF_OK, P.mf_last_error()
        assert torch.equal(r0, r1)
        assert n0 == n1 and n0 > 0.0
        assert P.residual_noalloc(m, L, b, x, r1) == n0


def test_noalloc_rejects_partials_beyond_the_scratch():
    co, ce = W.affine_triangle(2)
    L = 15  # 271,196 partial pairs in FP64, above the 131,071 the scratch holds
    m = P.create_macro_mesh(co, ce, L)
    b, x = _vectors(m, L, torch.float64, 3)
    r = torch.zeros_like(b)
    rc, _ = _call("residual_noalloc", m, L, b, x, r)
    assert rc == P.MF_ENOMEM
    assert "scratch" in P.mf_last_error()
    assert float(r.abs().max()) == 0.0  # rejected before any launch
    # a smaller level of the same mesh still runs
    rc, n = _call("residual_noalloc", m, 10, b, x, r)
    assert rc == P.MF_OK and n > 0.0
