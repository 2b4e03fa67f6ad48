// Host-side launchers of the HIP kernels (stencil_kernels.hip,
// vector_kernels.hip).  All are asynchronous on `stream` and return an MF_*
// status.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kargs.hpp"
#include "mesh.hpp"

namespace mf {

// One launch of the whole operator: interior rows of every macro (wave
// tiles) and macro-boundary rows (interface groups).  mode: kApply, kJacobi,
// kResidual, kNormB.  part (nullable; kResidual / kNormB) receives sums of
// squares at [0, np) and maxima at [np, 2 np), np = stencil_partials(L)
// (at most L.n_partials(), which sizes the buffers).
int64_t stencil_partials(const Level& L, int dtype);
int launch_stencil(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                   double omega, double* part, hipStream_t s);

// Interface groups only, for kExchangeSum (y = sum of x over copies;
// Dirichlet -> 0) and kDirichletSet (y = b at Dirichlet DoFs).
int launch_iface(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                 hipStream_t s);

// 2D only: y at every shared, non-Dirichlet DoF of L = the sum of its copies'
// partial rows, written to every copy (the exchange step of an apply).
int launch_exchange_apply(const Level& L, int dtype, void* y, hipStream_t s);

// P2 operator of a 2D mesh at `level` (vector layout: storage of level + 1):
// interior rows by fused wave tiles, macro-boundary rows from the element
// matrices (identity at Dirichlet DoFs), then the exchange.
int launch_p2_apply(const mf_mesh* m, int level, int dtype, const void* x, void* y, hipStream_t s);

// Variable-coefficient 2D apply y = A(k) x (k: nodal coefficient, same
// layout as x), including the exchange of shared DoFs.
int launch_varcoef_apply(const mf_mesh* m, const Level& L, int dtype, const void* k, const void* x, void* y,
                         hipStream_t s);

// Blended-macro 2D apply (FP64): bubble holds n_macros x 2 doubles (device).
int launch_blended_apply(const mf_mesh* m, const Level& L, const double* bubble, const double* x, double* y,
                         hipStream_t s);

// result[0] = sum part[0..np), result[1] = max part[np..2np), fixed order.
int launch_reduce(const double* part, int64_t np, double* result, hipStream_t s);

int launch_fill_random(const mf_mesh* m, const Level& L, int dtype, uint64_t seed, void* x, hipStream_t s);
int launch_restrict(const mf_mesh* m, const Level& fine, const Level& coarse, int dtype, const void* rf, void* bc,
                    hipStream_t s);
int launch_prolong_add(const mf_mesh* m, const Level& fine, const Level& coarse, int dtype, const void* ec,
                       void* xf, hipStream_t s);
int launch_coarse_solve(const Level& L, int dtype, const void* b, void* x, hipStream_t s);
// y = omega D^-1 b at every storage DoF (0 at Dirichlet DoFs): a Jacobi sweep
// whose iterate is zero, bitwise equal to launch_stencil(kJacobi) with x = 0.
int launch_jacobi0(const mf_mesh* m, const Level& L, int dtype, double omega, const void* b, void* y,
                   hipStream_t s);

// The V-cycle below level lc + nlev - 1 (nlev = tail_levels(...) >= 1) in one
// workgroup: vectors per level as in the solver workspace (b, x, t indexed
// by level).  Same steps and arithmetic as vcycle() on those levels.
template <typename T>
TailArgs<T> tail_args(const mf_mesh* m, int lc, int nlev, int pre, int post, double omega,
                      const std::vector<void*>& b, const std::vector<void*>& x, const std::vector<void*>& t);
int launch_vcycle_tail(const mf_mesh* m, int lc, int nlev, int dtype, int pre, int post, double omega,
                       const std::vector<void*>& b, const std::vector<void*>& x, const std::vector<void*>& t,
                       hipStream_t s);
int launch_tail_batch(const BatchOp& op, const char* table, hipStream_t s);

// Plain vector kernels over n entries.
int launch_fill(int dtype, void* x, double v, int64_t n, hipStream_t s);
int launch_copy(int dtype, void* dst, const void* src, int64_t n, hipStream_t s);
int launch_axpy(int dtype, void* y, const void* x, double a, int64_t n, hipStream_t s);    // y += a x
// The mixed solver's pair: b = float((1 / res[1]) r) and x += res[1] double(e),
// res = (sum of squares, max |.|) of r on the device.
int launch_scale_to_f32(const double* r, float* b, const double* res, int64_t n, hipStream_t s);
int launch_axpy_f32(double* x, const float* e, const double* res, int64_t n, hipStream_t s);

// Preconditioned conjugate gradients (scalars in res, see PcgArgs):
// z = s e (s = res[sslot] for FP32 e) and partials of r . z (edtype: type of
// e; z == e: not written); x += alpha p, r -= alpha q and partials of r . r,
// max |r|, with r32 also r32 = float(r / res[1]) and *sout = res[1] (both or
// neither); p = z + beta p.  Partials: L.lin_blocks() slots.
int launch_pcg_zdot(const mf_mesh* m, const Level& L, int edtype, const double* r, const void* e, double* z,
                    const double* res, double* part, hipStream_t s, int sslot = 1);
int launch_pcg_update(const mf_mesh* m, const Level& L, double* x, double* r, double* p, const double* q,
                      const double* res, double* part, hipStream_t s, float* r32 = nullptr, double* sout = nullptr);
// p = z + beta p; zdtype MF_F32: z is given as the FP32 V-cycle output e and
// formed as res[sslot] e (as launch_pcg_zdot forms it).
int launch_pcg_dir(double* p, const void* z, const double* res, int64_t n, hipStream_t s, int zdtype = MF_F64,
                   int sslot = 1);
// y = a y + b x1 + c x2 (x2 nullable) over n entries in nblk blocks of 256
// threads; part (nullable, 2 nblk doubles) receives zero sums and per-block
// maxima of |y| for launch_reduce.
int launch_lin3(double* y, const double* x1, const double* x2, double a, double b, double c, int64_t n, double* part,
                int nblk, hipStream_t s);
// result (2 doubles) = (sum, previous result[0]) of part[0, np)
int launch_reduce_shift(const double* part, int64_t np, double* result, hipStream_t s);

// Batched launches (one kernel over many requests; table = device base of
// the op's argument table).  Stencil, exchange, iface and reduce ops:
int launch_stencil_batch(const BatchOp& op, const char* table, hipStream_t s);
// Transfer, coarse-solve and vector ops:
int launch_vector_batch(const BatchOp& op, const char* table, hipStream_t s);

}  // namespace mf
