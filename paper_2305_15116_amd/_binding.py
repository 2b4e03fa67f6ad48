"""ctypes binding of libmfstencil.so with the same names as the C ABI.

Argument marshalling only: every computation runs in the library's HIP
kernels.  Vectors are torch tensors on the current HIP device (storage
layout, float64 or float32); streams default to torch's current stream.
There is no fallback: if the shared library is missing, loading fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_PKG, "libmfstencil.so")

MF_OK, MF_NOT_CONVERGED = 0, 1
MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_ENOTSUP, MF_ENUMERIC = -1, -2, -3, -4, -5
MF_F64, MF_F32 = 0, 1
MF_FLAG_DIRICHLET, MF_FLAG_HOST_ONLY = 1, 2

#: every symbol include/mf_stencil.h declares
EXPORTS = ["mf_last_error", "create_macro_mesh", "destroy_macro_mesh", "mesh_info", "mesh_num_dofs",
           "mesh_dof_keys", "mesh_dof_index", "mesh_stencil", "mesh_workspace_bytes", "mesh_fill_random",
           "mesh_set_dirichlet", "apply_stencil", "apply_p2", "apply_varcoef", "apply_blended", "smooth", "residual", "residual_noalloc", "restrict_residual", "prolong_add",
           "vcycle_solve", "device_copy", "batch_create", "batch_destroy", "batch_size", "batch_add", "batch_step"]


class MFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("pre", C.c_int), ("post", C.c_int), ("coarse_level", C.c_int),
                ("max_iter", C.c_int), ("omega", C.c_double), ("rtol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("rel_res", C.c_double), ("seconds", C.c_double)]


_lib = None


def lib():
    """Load the library; raises OSError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise OSError(f"{LIBPATH} is missing: run __graft_entry__.build() (no fallback exists)")
        L = C.CDLL(LIBPATH)
        vp, i64, i32, dbl, i = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int
        L.mf_last_error.restype = C.c_char_p
        L.create_macro_mesh.argtypes = [i, i64, vp, i64, vp, i, i, C.POINTER(vp)]
        L.destroy_macro_mesh.argtypes = [vp]
        L.mesh_info.argtypes = [vp, C.POINTER(i), C.POINTER(i64), C.POINTER(i)]
        L.mesh_num_dofs.argtypes = [vp, i, C.POINTER(i64), C.POINTER(i64)]
        L.mesh_dof_keys.argtypes = [vp, i, vp, vp]
        L.mesh_dof_index.argtypes = [vp, i, i64, vp, vp]
        L.mesh_stencil.argtypes = [vp, i, i64, vp]
        L.mesh_workspace_bytes.argtypes = [vp, i, i, C.POINTER(i64)]
        L.mesh_fill_random.argtypes = [vp, i, i, C.c_uint64, vp, vp]
        L.mesh_set_dirichlet.argtypes = [vp, i, i, vp, vp, vp]
        L.apply_stencil.argtypes = [vp, i, i, vp, vp, vp]
        L.smooth.argtypes = [vp, i, i, dbl, i, vp, vp, vp, vp]
        L.residual.argtypes = [vp, i, i, vp, vp, vp, C.POINTER(dbl), vp]
        L.residual_noalloc.argtypes = [vp, i, i, vp, vp, vp, C.POINTER(dbl), vp]
        L.restrict_residual.argtypes = [vp, i, i, vp, vp, vp]
        L.prolong_add.argtypes = [vp, i, i, vp, vp, vp]
        L.vcycle_solve.argtypes = [vp, i, vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.device_copy.argtypes = [vp, vp, i64, vp]
        L.batch_create.argtypes = [C.POINTER(SolveOpts), i, C.POINTER(vp)]
        L.batch_destroy.argtypes = [vp]
        L.batch_size.argtypes = [vp, C.POINTER(i)]
        L.batch_add.argtypes = [vp, vp, i, vp, vp, vp, dbl, i64]
        L.batch_step.argtypes = [vp, vp, vp, vp, C.POINTER(SolveInfo), C.POINTER(i)]
        for name in EXPORTS[1:]:
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def mf_last_error() -> str:
    return lib().mf_last_error().decode()


def _check(rc, allow=(MF_OK,)):
    if rc not in allow:
        raise MFError(rc, mf_last_error())
    return rc


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return MF_F64
    if t.dtype == torch.float32:
        return MF_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


class Mesh:
    """Owner of an mf_mesh*; destroyed with the object."""

    def __init__(self, handle, dim, n_macros, max_level):
        self.handle = handle
        self.dim, self.n_macros, self.max_level = dim, n_macros, max_level

    def close(self):
        if self.handle:
            lib().destroy_macro_mesh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return C.c_void_p(self.handle)


def create_macro_mesh(coords, cells, max_level: int, flags: int = MF_FLAG_DIRICHLET) -> Mesh:
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    dim = coords.shape[1]
    out = C.c_void_p()
    _check(lib().create_macro_mesh(dim, coords.shape[0], coords.ctypes.data, cells.shape[0], cells.ctypes.data,
                                   max_level, flags, C.byref(out)))
    return Mesh(out.value, dim, cells.shape[0], max_level)


def destroy_macro_mesh(mesh: Mesh):
    mesh.close()


def mesh_info(mesh: Mesh):
    d, n, l = C.c_int(), C.c_int64(), C.c_int()
    _check(lib().mesh_info(mesh, C.byref(d), C.byref(n), C.byref(l)))
    return d.value, n.value, l.value


def mesh_num_dofs(mesh: Mesh, level: int):
    s, u = C.c_int64(), C.c_int64()
    _check(lib().mesh_num_dofs(mesh, level, C.byref(s), C.byref(u)))
    return s.value, u.value


def mesh_dof_keys(mesh: Mesh, level: int):
    n, _ = mesh_num_dofs(mesh, level)
    d1 = mesh.dim + 1
    v = np.empty((n, d1), np.int64)
    w = np.empty((n, d1), np.int32)
    _check(lib().mesh_dof_keys(mesh, level, v.ctypes.data, w.ctypes.data))
    return v, w


def mesh_dof_index(mesh: Mesh, level: int, macro_lattice):
    ml = np.ascontiguousarray(macro_lattice, dtype=np.int64)
    out = np.empty(ml.shape[0], np.int64)
    _check(lib().mesh_dof_index(mesh, level, ml.shape[0], ml.ctypes.data, out.ctypes.data))
    return out


def mesh_stencil(mesh: Mesh, level: int, macro: int):
    w = np.empty(7 if mesh.dim == 2 else 15)
    _check(lib().mesh_stencil(mesh, level, macro, w.ctypes.data))
    return w


def mesh_workspace_bytes(mesh: Mesh, level: int, mode: int) -> int:
    b = C.c_int64()
    _check(lib().mesh_workspace_bytes(mesh, level, mode, C.byref(b)))
    return b.value


def mesh_fill_random(mesh: Mesh, level: int, seed: int, x, stream=None):
    _check(lib().mesh_fill_random(mesh, level, _dtype_code(x), seed, C.c_void_p(x.data_ptr()), _stream(stream)))


def mesh_set_dirichlet(mesh: Mesh, level: int, b, y, stream=None):
    """y = b at Dirichlet DoFs (b=None: 0 there); other entries unchanged."""
    _check(lib().mesh_set_dirichlet(mesh, level, _dtype_code(y), None if b is None else C.c_void_p(b.data_ptr()),
                                    C.c_void_p(y.data_ptr()), _stream(stream)))


def apply_stencil(mesh: Mesh, level: int, x, y, stream=None):
    _check(lib().apply_stencil(mesh, level, _dtype_code(x), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                               _stream(stream)))


def apply_varcoef(mesh: Mesh, level: int, k, x, y, stream=None):
    """y = A(k) x for -div(k grad u) (P1, 2D or 3D; k nodal, same layout and dtype as x)."""
    if k.dtype != x.dtype:
        raise MFError(MF_EINVAL, "k and x must have the same dtype")
    _check(lib().apply_varcoef(mesh, level, _dtype_code(x), C.c_void_p(k.data_ptr()), C.c_void_p(x.data_ptr()),
                               C.c_void_p(y.data_ptr()), _stream(stream)))


def apply_blended(mesh: Mesh, level: int, bubble, x, y, stream=None):
    """y = A x on blended 2D macros (FP64); bubble: (n_macros, 2) float64 on the device."""
    if bubble.dtype != x.dtype or _dtype_code(x) != MF_F64:
        raise MFError(MF_EINVAL, "apply_blended takes float64 bubble, x and y")
    if bubble.numel() != 2 * mesh.n_macros or not bubble.is_contiguous():
        raise MFError(MF_EINVAL, f"apply_blended needs a contiguous ({mesh.n_macros}, 2) bubble")
    _check(lib().apply_blended(mesh, level, C.c_void_p(bubble.data_ptr()), C.c_void_p(x.data_ptr()),
                               C.c_void_p(y.data_ptr()), _stream(stream)))


def apply_p2(mesh: Mesh, level: int, x, y, stream=None):
    """y = A x for the 2D P2 operator of `level`; x and y have the storage
    layout of level + 1 (its lattice holds the vertex and edge-midpoint DoFs)."""
    _check(lib().apply_p2(mesh, level, _dtype_code(x), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                          _stream(stream)))


def smooth(mesh: Mesh, level: int, omega: float, sweeps: int, b, x, tmp, stream=None):
    _check(lib().smooth(mesh, level, _dtype_code(x), omega, sweeps, C.c_void_p(b.data_ptr()),
                        C.c_void_p(x.data_ptr()), C.c_void_p(tmp.data_ptr()), _stream(stream)))


def residual(mesh: Mesh, level: int, b, x, r, norm: bool = False, stream=None):
    """r = b - A x; returns ||r||_2 over unique DoFs if norm=True (synchronises)."""
    n2 = C.c_double()
    _check(lib().residual(mesh, level, _dtype_code(x), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                          C.c_void_p(r.data_ptr()), C.byref(n2) if norm else None, _stream(stream)))
    return n2.value if norm else None


def residual_noalloc(mesh: Mesh, level: int, b, x, r, stream=None):
    """r = b - A x and ||r||_2 over unique DoFs (synchronises), with the norm
    partials in the library's static device scratch (no allocation)."""
    n2 = C.c_double()
    _check(lib().residual_noalloc(mesh, level, _dtype_code(x), C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                  C.c_void_p(r.data_ptr()), C.byref(n2), _stream(stream)))
    return n2.value


def device_copy(dst, src, stream=None):
    """dst = src (same byte size, a multiple of 16): the library's streaming copy."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("dst and src differ in size")
    _check(lib().device_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nb, _stream(stream)))


def restrict_residual(mesh: Mesh, level: int, rf, bc, stream=None):
    _check(lib().restrict_residual(mesh, level, _dtype_code(rf), C.c_void_p(rf.data_ptr()),
                                   C.c_void_p(bc.data_ptr()), _stream(stream)))


def prolong_add(mesh: Mesh, level: int, ec, xf, stream=None):
    _check(lib().prolong_add(mesh, level, _dtype_code(ec), C.c_void_p(ec.data_ptr()), C.c_void_p(xf.data_ptr()),
                             _stream(stream)))


def vcycle_solve(mesh: Mesh, level: int, b, x, workspace, mode: int = 0, pre: int = 2, post: int = 2,
                 coarse_level: int | None = None, max_iter: int = 50, omega: float = 2.0 / 3.0,
                 rtol: float = 1e-10, stream=None):
    """Returns (status, iters, rel_res, seconds); status is MF_OK or MF_NOT_CONVERGED."""
    o = SolveOpts(mode, pre, post, min(2, level) if coarse_level is None else coarse_level, max_iter, omega, rtol)
    info = SolveInfo()
    rc = _check(lib().vcycle_solve(mesh, level, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(workspace.data_ptr()), C.byref(o), C.byref(info), _stream(stream)),
                allow=(MF_OK, MF_NOT_CONVERGED))
    return rc, info.iters, info.rel_res, info.seconds


class Batch:
    """Owner of an mf_batch* (continuous batching of solves); destroyed with the object."""

    def __init__(self, handle, capacity):
        self.handle = handle
        self.capacity = capacity

    def close(self):
        if self.handle:
            lib().batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def _as_parameter_(self):
        return C.c_void_p(self.handle)


def batch_create(capacity: int, mode: int = 1, pre: int = 2, post: int = 2, coarse_level: int = -1,
                 max_iter: int = 50, omega: float = 2.0 / 3.0) -> Batch:
    o = SolveOpts(mode, pre, post, coarse_level, max_iter, omega, 0.0)
    out = C.c_void_p()
    _check(lib().batch_create(C.byref(o), capacity, C.byref(out)))
    return Batch(out.value, capacity)


def batch_destroy(batch: Batch):
    batch.close()


def batch_size(batch: Batch) -> int:
    n = C.c_int()
    _check(lib().batch_size(batch, C.byref(n)))
    return n.value


def batch_add(batch: Batch, mesh: Mesh, level: int, b, x, workspace, rtol: float, tag: int):
    _check(lib().batch_add(batch, mesh, level, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                           C.c_void_p(workspace.data_ptr()), rtol, tag))


def batch_step(batch: Batch, stream=None):
    """One outer iteration for every member; returns [(tag, status, iters, rel_res, seconds)] of those done."""
    cap = max(1, batch.capacity)
    tags = np.empty(cap, np.int64)
    status = np.empty(cap, np.int32)
    infos = (SolveInfo * cap)()
    n = C.c_int()
    _check(lib().batch_step(batch, _stream(stream), tags.ctypes.data, status.ctypes.data, infos, C.byref(n)))
    return [(int(tags[k]), int(status[k]), infos[k].iters, infos[k].rel_res, infos[k].seconds)
            for k in range(n.value)]
