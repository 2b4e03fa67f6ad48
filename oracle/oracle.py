"""Python face of the oracle (test infrastructure only).

Wraps oracle/liboracle.so (plain C++ FP64 CSR assembly and SpMV, written from
the definition of the P1 stiffness matrix, and of the 2D P2 one) and adds the two solves the tests
need: a dense solve at tiny levels and conjugate gradients on the interior
block, both textbook routines on the oracle's own CSR.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIBPATH)
        L.or_last_error.restype = C.c_char_p
        L.or_splitmix64.restype = C.c_uint64
        L.or_splitmix64.argtypes = [C.c_uint64]
        L.or_build.restype = C.c_void_p
        L.or_build.argtypes = [C.c_int, C.c_int64, f64p, C.c_int64, i64p, C.c_int]
        L.or_free.argtypes = [C.c_void_p]
        L.or_num_unique.restype = C.c_int64
        L.or_num_unique.argtypes = [C.c_void_p]
        L.or_get_keys.argtypes = [C.c_void_p, i64p, i32p]
        L.or_get_coords.argtypes = [C.c_void_p, f64p]
        L.or_get_boundary.argtypes = [C.c_void_p, i8p]
        L.or_keyed_random.argtypes = [C.c_void_p, C.c_uint64, f64p]
        L.or_elements.restype = C.c_int64
        L.or_elements.argtypes = [C.c_void_p, C.c_void_p]
        L.or_assemble.restype = C.c_int64
        L.or_assemble.argtypes = [C.c_void_p, C.c_int]
        L.or_assemble_blended.restype = C.c_int64
        L.or_assemble_blended.argtypes = [C.c_void_p, C.c_int, f64p]
        L.or_assemble_varcoef.restype = C.c_int64
        L.or_assemble_varcoef.argtypes = [C.c_void_p, C.c_int, f64p]
        L.or_assemble_p2.restype = C.c_int64
        L.or_assemble_p2.argtypes = [C.c_void_p, C.c_int]
        L.or_get_csr.argtypes = [C.c_void_p, i64p, i64p, f64p]
        L.or_spmv.argtypes = [C.c_void_p, f64p, f64p]
        L.or_apply_elementwise.restype = C.c_int
        L.or_apply_elementwise.argtypes = [C.c_void_p, C.c_int, f64p, f64p]
        L.or_lumped_mass.restype = C.c_int
        L.or_lumped_mass.argtypes = [C.c_void_p, f64p]
        L.or_sample_rows.restype = C.c_int
        L.or_sample_rows.argtypes = [C.c_int, C.c_int64, f64p, C.c_int64, i64p, C.c_int, C.c_int,
                                     C.c_uint64, C.c_int64, i64p, i64p, f64p, i8p]
        L.or_sample_rows_blended.restype = C.c_int
        L.or_sample_rows_blended.argtypes = [C.c_int64, f64p, C.c_int64, i64p, C.c_int, C.c_int, C.c_uint64, f64p,
                                             C.c_int64, i64p, i64p, f64p, i8p]
        L.or_sample_rows_varcoef.restype = C.c_int
        L.or_sample_rows_varcoef.argtypes = [C.c_int, C.c_int64, f64p, C.c_int64, i64p, C.c_int, C.c_int, C.c_uint64,
                                             C.c_uint64, C.c_double, C.c_int64, i64p, i64p, f64p, i8p]
        L.or_keyed_points.restype = C.c_int
        L.or_keyed_points.argtypes = [C.c_int, C.c_int64, i64p, C.c_int, C.c_uint64, C.c_int64, i64p, i64p, f64p]
        L.or_prolongation.restype = C.c_int64
        L.or_prolongation.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_time_spmv.restype = C.c_int
        L.or_time_spmv.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, f64p]
        _lib = L
    return _lib


def splitmix64(z: int) -> int:
    return int(lib().or_splitmix64(z))


def _err():
    return lib().or_last_error().decode()


class OracleMesh:
    """The refined macro mesh at one level, with unique DoFs identified by keys."""

    def __init__(self, coords, cells, level: int):
        coords = np.ascontiguousarray(coords, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        self.dim = coords.shape[1]
        self.level = level
        self.N = 1 << level
        self.coords, self.cells = coords, cells
        h = lib().or_build(self.dim, coords.shape[0], coords.ravel(), cells.shape[0], cells.ravel(), level)
        if not h:
            raise ValueError(_err())
        self._h = h
        self.n = int(lib().or_num_unique(h))
        self._csr = {}
        self._native_state = None
        self._native_nnz = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_free(h)
            self._h = None

    def keys(self):
        d1 = self.dim + 1
        v = np.empty(self.n * d1, np.int64)
        w = np.empty(self.n * d1, np.int32)
        lib().or_get_keys(self._h, v, w)
        return v.reshape(self.n, d1), w.reshape(self.n, d1)

    def xyz(self):
        out = np.empty(self.n * self.dim)
        lib().or_get_coords(self._h, out)
        return out.reshape(self.n, self.dim)

    def boundary(self):
        out = np.empty(self.n, np.int8)
        lib().or_get_boundary(self._h, out)
        return out.astype(bool)

    def keyed_random(self, seed: int):
        out = np.empty(self.n)
        lib().or_keyed_random(self._h, seed, out)
        return out

    def elements(self):
        ne = lib().or_elements(self._h, None)
        out = np.empty(ne * (self.dim + 1), np.int64)
        lib().or_elements(self._h, out.ctypes.data_as(C.c_void_p))
        return out.reshape(ne, self.dim + 1)

    def _native(self, dirichlet: bool) -> int:
        """Assemble the native CSR with the requested boundary rows; returns nnz."""
        if self._native_state != bool(dirichlet):
            nnz = lib().or_assemble(self._h, int(dirichlet))
            if nnz < 0:
                raise ValueError(_err())
            self._native_state = bool(dirichlet)
            self._native_nnz = int(nnz)
        return self._native_nnz

    def csr_blended(self, d, dirichlet: bool = True) -> sp.csr_matrix:
        """P1 stiffness matrix of the micro mesh whose lattice points macro c
        maps by F_c(xi) = affine(xi) + xi0 xi1 xi2 d[c] (2D; d: n_cells x 2)."""
        d = np.ascontiguousarray(d, dtype=np.float64).reshape(-1)
        nnz = lib().or_assemble_blended(self._h, int(dirichlet), d)
        if nnz < 0:
            raise ValueError(_err())
        self._native_state = ("blended", None)
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(nnz, np.int64)
        va = np.empty(nnz)
        lib().or_get_csr(self._h, rp, ci, va)
        return sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))

    def csr_varcoef(self, k, dirichlet: bool = True) -> sp.csr_matrix:
        """Stiffness matrix of -div(k grad u), k the P1 interpolant of the
        nodal values k (one per unique DoF)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        nnz = lib().or_assemble_varcoef(self._h, int(dirichlet), k)
        if nnz < 0:
            raise ValueError(_err())
        self._native_state = ("varcoef", None)
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(nnz, np.int64)
        va = np.empty(nnz)
        lib().or_get_csr(self._h, rp, ci, va)
        return sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))

    def csr_p2(self, dirichlet: bool = True) -> sp.csr_matrix:
        """P2 stiffness matrix of level self.level - 1 (2D) on this mesh's DoFs:
        the vertices and edge midpoints of that level's micro-triangles are the
        lattice points of this level."""
        key = ("p2", bool(dirichlet))
        if key not in self._csr:
            nnz = lib().or_assemble_p2(self._h, int(dirichlet))
            if nnz < 0:
                raise ValueError(_err())
            self._native_state = key
            rp = np.empty(self.n + 1, np.int64)
            ci = np.empty(nnz, np.int64)
            va = np.empty(nnz)
            lib().or_get_csr(self._h, rp, ci, va)
            self._csr[key] = sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))
        return self._csr[key]

    def spmv_p2(self, x, dirichlet: bool = True):
        """y = A x for the P2 matrix of csr_p2, with the oracle's own CSR row loop."""
        key = ("p2", bool(dirichlet))
        if self._native_state != key:
            if lib().or_assemble_p2(self._h, int(dirichlet)) < 0:
                raise ValueError(_err())
            self._native_state = key
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        lib().or_spmv(self._h, x, y)
        return y

    def csr(self, dirichlet: bool = True) -> sp.csr_matrix:
        key = bool(dirichlet)
        if key not in self._csr:
            nnz = self._native(dirichlet)
            rp = np.empty(self.n + 1, np.int64)
            ci = np.empty(nnz, np.int64)
            va = np.empty(nnz)
            lib().or_get_csr(self._h, rp, ci, va)
            self._csr[key] = sp.csr_matrix((va, ci, rp), shape=(self.n, self.n))
        return self._csr[key]

    def spmv(self, x, dirichlet: bool = True):
        """y = A x with the oracle's own CSR row loop."""
        self._native(dirichlet)
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        lib().or_spmv(self._h, x, y)
        return y

    def apply_elementwise(self, x, dirichlet: bool = True):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        if lib().or_apply_elementwise(self._h, int(dirichlet), x, y) != 0:
            raise ValueError(_err())
        return y

    def lumped_mass(self):
        out = np.empty(self.n)
        if lib().or_lumped_mass(self._h, out) != 0:
            raise ValueError(_err())
        return out

    def time_spmv(self, nthreads: int, warmup: int, reps: int):
        """Per-rep seconds of the CSR row loop, and the thread count it used."""
        self._native(True)
        t = np.empty(reps)
        used = lib().or_time_spmv(self._h, nthreads, warmup, reps, t)
        return t, used


def prolongation(fine: OracleMesh, coarse: OracleMesh) -> sp.csr_matrix:
    nnz = lib().or_prolongation(fine._h, coarse._h, None, None, None)
    if nnz < 0:
        raise ValueError(_err())
    rp = np.empty(fine.n + 1, np.int64)
    ci = np.empty(nnz, np.int64)
    va = np.empty(nnz)
    r = lib().or_prolongation(fine._h, coarse._h, rp.ctypes.data_as(C.c_void_p),
                              ci.ctypes.data_as(C.c_void_p), va.ctypes.data_as(C.c_void_p))
    if r < 0:
        raise ValueError(_err())
    return sp.csr_matrix((va, ci, rp), shape=(fine.n, coarse.n))


def sample_rows(coords, cells, level: int, seed: int, sample_cell, sample_lat, dirichlet: bool = True):
    """Rows of A at sampled (cell, lattice point) pairs for x = keyed random(seed),
    with no global build.  Returns (y, is_boundary)."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    sc = np.ascontiguousarray(sample_cell, dtype=np.int64)
    sl = np.ascontiguousarray(sample_lat, dtype=np.int64).ravel()
    ns = sc.shape[0]
    y = np.empty(ns)
    b = np.empty(ns, np.int8)
    r = lib().or_sample_rows(coords.shape[1], coords.shape[0], coords.ravel(), cells.shape[0], cells.ravel(),
                             level, int(dirichlet), seed, ns, sc, sl, y, b)
    if r != 0:
        raise ValueError(_err())
    return y, b.astype(bool)


def sample_rows_blended(coords, cells, level: int, seed: int, bubble, sample_cell, sample_lat, dirichlet: bool = True):
    """Rows of the blended 2D operator (csr_blended) at sampled (cell, lattice
    point) pairs for x = keyed random(seed), with no global build."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    bub = np.ascontiguousarray(bubble, dtype=np.float64).reshape(-1)
    sc = np.ascontiguousarray(sample_cell, dtype=np.int64)
    sl = np.ascontiguousarray(sample_lat, dtype=np.int64).ravel()
    ns = sc.shape[0]
    y = np.empty(ns)
    b = np.empty(ns, np.int8)
    r = lib().or_sample_rows_blended(coords.shape[0], coords.ravel(), cells.shape[0], cells.ravel(), level,
                                     int(dirichlet), seed, bub, ns, sc, sl, y, b)
    if r != 0:
        raise ValueError(_err())
    return y, b.astype(bool)


def sample_rows_varcoef(coords, cells, level: int, seed: int, kseed: int, kshift: float, sample_cell, sample_lat,
                        dirichlet: bool = True):
    """Rows of the variable-coefficient operator (csr_varcoef with k = keyed
    random(kseed) + kshift) at sampled (cell, lattice point) pairs for
    x = keyed random(seed), with no global build."""
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    sc = np.ascontiguousarray(sample_cell, dtype=np.int64)
    sl = np.ascontiguousarray(sample_lat, dtype=np.int64).ravel()
    ns = sc.shape[0]
    y = np.empty(ns)
    b = np.empty(ns, np.int8)
    r = lib().or_sample_rows_varcoef(coords.shape[1], coords.shape[0], coords.ravel(), cells.shape[0], cells.ravel(),
                                     level, int(dirichlet), seed, kseed, float(kshift), ns, sc, sl, y, b)
    if r != 0:
        raise ValueError(_err())
    return y, b.astype(bool)


def keyed_points(cells, dim: int, level: int, seed: int, sample_cell, sample_lat):
    """Keyed input values at sampled (cell, lattice point) pairs."""
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    sc = np.ascontiguousarray(sample_cell, dtype=np.int64)
    sl = np.ascontiguousarray(sample_lat, dtype=np.int64).ravel()
    out = np.empty(sc.shape[0])
    if lib().or_keyed_points(dim, cells.shape[0], cells.ravel(), level, seed, sc.shape[0], sc, sl, out) != 0:
        raise ValueError(_err())
    return out


def solve(mesh: OracleMesh, b, tol: float = 1e-13, maxiter: int = 100000):
    """Solution of A u = b with identity Dirichlet rows (u = b on the boundary).

    The boundary columns are moved to the right-hand side and the interior
    block (SPD) is solved by a dense solve at levels <= 3, else by plain
    conjugate gradients to ||r|| <= tol ||b_I||.
    """
    A = mesh.csr(dirichlet=False)
    bnd = mesh.boundary()
    inn = ~bnd
    u = np.zeros(mesh.n)
    u[bnd] = b[bnd]
    rhs = b[inn] - A[inn][:, bnd] @ u[bnd]
    AII = A[inn][:, inn].tocsr()
    if mesh.level <= 3:
        u[inn] = np.linalg.solve(AII.toarray(), rhs)
        return u
    x = np.zeros(AII.shape[0])
    r = rhs.copy()
    p = r.copy()
    rr = r @ r
    stop = (tol * np.linalg.norm(rhs)) ** 2
    for _ in range(maxiter):
        if rr <= stop:
            break
        q = AII @ p
        a = rr / (p @ q)
        x += a * p
        r -= a * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    u[inn] = x
    return u


def key_order(vids, wts):
    """Permutation that sorts DoF keys (rows of vids/wts) lexicographically."""
    cols = []
    for k in range(vids.shape[1] - 1, -1, -1):
        cols.append(wts[:, k])
        cols.append(vids[:, k])
    return np.lexsort(cols)
