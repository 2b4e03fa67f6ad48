// Kernel argument records and batched launches.
//
// Every kernel of the library takes one Launch<A>: either the arguments of a
// single request by value (nseg == 0), or a device table of per-request
// arguments, in which request r owns the launch's workgroups
// [wg0[r], wg0[r+1]).  A batched launch therefore runs the same kernel over
// the tiles of many requests at once (continuous batching of solves), and
// each request's work is decomposed exactly as in its own launch, so its
// results are bitwise the same.
#pragma once

#include <cstdint>

#include "mesh.hpp"

namespace mf {

template <class A>
struct Launch {
  A one;               // nseg == 0: the single request's arguments
  const A* many;       // nseg > 0: per-request arguments (device)
  const int32_t* wg0;  // nseg > 0: nseg + 1 workgroup offsets (device), wg0[0] = 0
  int nseg;
  int nwg;             // workgroups of the whole launch
};

// The request that owns workgroup g: the last r with wg0[r] <= g (requests
// with no workgroups share their offset with the next one and are skipped).
MF_HD int find_seg(const int32_t* wg0, int nseg, int g) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wg0[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// stencil_kernel: every point of every macro of one level.
template <typename T>
struct StencilArgs {
  const Tile* tiles;
  int ntiles;  // wave tiles (one partial slot each)
  int nwg;     // workgroups of tiles (natural order)
  const MacroDev* md;
  const T* X;
  T* Y;
  const T* B;
  T omega;
  double* part;  // sums at [0, np), maxima at [np, 2 np)
  int np;
  // exchange list, read by group tiles (levels whose launch finishes shared DoFs)
  const int32_t* xptr;
  const Copy* xcopies;
  const int64_t* xcidx;
  const double* xinv;
  const float* xinvf;
};

// exchange_kernel / iface_kernel: groups of copies of macro-boundary DoFs.
template <typename T>
struct GroupArgs {
  int ngroups;
  const int32_t* gptr;
  const Copy* copies;
  const int64_t* cidx;  // storage index of each copy
  const uint8_t* gflag;  // all-groups list only
  const double* ginv;    // exchange list only
  const float* ginvf;
  const MacroDev* md;
  const T* X;
  T* Y;
  const T* B;
  T omega;
  double* part;  // block partials at [0, nblk), maxima at [np, ...)
  int np;
};

// restrict_kernel / prolong_add_kernel: per-point segments of one level.
template <typename T>
struct TransferArgs {
  const Tile* segs;
  int nseg;
  int nblk;  // blocks of this request: each wave loops over segments with stride 4 nblk
  const MacroDev* mdc;
  const MacroDev* mdf;
  const T* src;
  T* dst;
  const int32_t* sbc;  // slice bases of the coarse and the fine level (3D segment kernels)
  const int32_t* sbf;
};

// coarse_solve_kernel
template <typename T>
struct CoarseArgs {
  int n;
  const T* Ainv;
  const int32_t* first;
  const int32_t* cptr;
  const int64_t* cidx;
  const T* B;
  T* X;
};

// The first Jacobi sweep of a V-cycle level, whose iterate is zero, in two
// launches: jacobi0_stream_kernel writes the interior formula to every point
// of every macro (nmac macros of P points, bpm blocks each), then
// jacobi0_fix_kernel rewrites the macro-boundary DoFs: blocks [0, nblk_all)
// take the all-groups list (Dirichlet and unshared DoFs), blocks
// [nblk_all, nblk_all + nblk_grp) the shared non-Dirichlet ones (the
// exchange list), one group per thread.
template <typename T>
struct Jacobi0Args {
  int nmac, bpm;
  int64_t P;
  int nall, nblk_all;  // all macro-boundary DoFs
  const int32_t* aptr;
  const Copy* acopies;
  int ngroups, nblk_grp;  // exchange list
  const int32_t* gptr;
  const Copy* copies;
  const int64_t* gidx;  // storage index of each exchange-list copy
  const double* ginv;
  const float* ginvf;
  const MacroDev* md;
  const T* B;
  T* Y;
  T omega;
};
constexpr int kJ0Points = 2048;  // points per block of the streaming pass (a multiple of the block size)

// vcycle_tail_kernel: the bottom of a V-cycle — the coarse solve and up to
// kTailLevels - 1 levels above it, each of at most kTailMaxPoints storage
// points — run by one workgroup of kTailWG threads with barriers between the
// steps, instead of about a dozen launches per level whose time is latency.
// The point limit is where one CU stops beating the whole chip: measured on
// cube and triangle solves, 3D levels of 990 points gain and of 5,814 points
// lose (the single CU's load bandwidth; also with the level's FP32 vectors
// in LDS), 2D levels of 2,145 points gain.
#ifndef MF_TAIL_LEVELS
#define MF_TAIL_LEVELS 4
#endif
#ifndef MF_TAIL_MAX_POINTS
#define MF_TAIL_MAX_POINTS 4096
#endif
constexpr int kTailLevels = MF_TAIL_LEVELS;
constexpr int kTailWG = 1024;
constexpr int64_t kTailMaxPoints = MF_TAIL_MAX_POINTS;
constexpr int kTailMaxCoarse = 256;  // coarse unknowns (the dense solve runs on one CU)

template <typename T>
struct TailLevel {
  int nx;  // exchange list: shared non-Dirichlet DoFs
  const int32_t* xptr;
  const Copy* xcopies;
  const int64_t* xcidx;
  const double* xinv;
  const float* xinvf;
  int ng;  // all macro-boundary DoFs
  const int32_t* gptr;
  const Copy* copies;
  const int64_t* gcidx;
  const uint8_t* gflag;
  const MacroDev* md;
  int64_t storage;  // nmac macros of side N, stored one after the other
  int N, nmac;
  T* b;  // right-hand side, iterate and ping-pong vector of the cycle
  T* x;
  T* t;
};

template <typename T>
struct TailArgs {
  int nlev;  // levels lc .. lc + nlev - 1 in lv[0 .. nlev)
  int pre, post;
  T omega;
  CoarseArgs<T> coarse;
  TailLevel<T> lv[kTailLevels];
  int lds;  // bytes of LDS holding the levels' b, x and t (0: they stay in global memory)
};

// The tail keeps its levels' vectors in LDS when they fit in kTailLdsMax
// bytes: three per level (b, x, t), each rounded up to 16 bytes.
#ifndef MF_TAIL_LDS_MAX
#define MF_TAIL_LDS_MAX (64 * 1024)
#endif
constexpr int kTailLdsMax = MF_TAIL_LDS_MAX;
MF_HD constexpr int64_t tail_lds_vec(int64_t storage, int elem) { return (storage * elem + 15) / 16 * 16; }

// Plain vector kernels (fill, copy, axpy and the FP32 <-> FP64 pair of the
// mixed solver, whose scale comes from a device norm result).
struct VecArgs {
  void* y;
  const void* x;
  const double* res;  // result pair (sum of squares, max |.|) of a reduction
  int64_t n;
  double a;
  int nblk;   // grid-stride blocks of this request
  int sslot;  // PCG direction: res slot of the FP32 preconditioner's scale (1, or 8 in mixed CG)
};

// reduce_kernel: one block per request.
struct ReduceArgs {
  const double* part;
  int64_t np;
  double* result;  // 2 doubles: (sum, max), or (sum, previous sum) with shift
  double* copy;    // nullable: a second copy of the 2 doubles
  int shift;       // 1: result[1] takes the previous result[0] instead of the max
  int pad_;
};

// Vector kernels of preconditioned conjugate gradients: FP64 vectors,
// grid-stride over the storage index with nblk blocks, one (sum, max)
// partial per block; sums count each unique DoF once (its owner copy, from
// the level's owner bits).  Scalars live on the device in res:
// [0] r.r  [1] max |r|  [2] r.z  [3] previous r.z  [4] p.A p.
struct PcgArgs {
  int64_t n;
  const uint32_t* own;  // owner bits of the storage DoFs
  double* x;            // update: x += alpha p
  double* r;            // zdot: read; update: r -= alpha q
  double* p;            // update: read
  const double* q;      // update: A p
  const void* e;        // zdot: preconditioner output (FP32 or FP64)
  double* z;            // zdot: z = s e (not written when z == e)
  const double* res;    // scalars
  double* part;         // sums at [0, nblk), maxima at [nblk, 2 nblk)
  float* r32;           // update (nullable): the next preconditioner input, float(r / res[1])
  double* sout;         // update with r32: receives res[1], the scale r32 was formed with
  int nblk;
  int sslot;            // zdot: res slot of the FP32 preconditioner's scale s (1, or 8 in mixed CG)
};

inline int vec_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------- builders
// The same records serve single launches and batch tables.
template <typename T>
constexpr int dtype_of() { return sizeof(T) == 4 ? MF_F32 : MF_F64; }

template <typename T>
StencilArgs<T> stencil_args(const Level& L, const void* x, void* y, const void* b, double omega, double* part) {
  constexpr int dt = dtype_of<T>();
  const bool f32 = dt == MF_F32 && !L.tiles_f32.empty();
  StencilArgs<T> a;
  a.tiles = f32 ? L.dev.tiles_f32 : L.dev.tiles;
  a.ntiles = (int)L.tiles_for(dt).size();
  a.nwg = a.ntiles / kWavesPerWG;
  a.md = L.dev.md;
  a.X = (const T*)x;
  a.Y = (T*)y;
  a.B = (const T*)b;
  a.omega = (T)omega;
  a.part = part;
  a.np = (int)L.n_partials(dt);
  a.xptr = L.dev.xgrp_ptr;
  a.xcopies = L.dev.xcopies;
  a.xcidx = L.dev.xcpidx;
  a.xinv = L.dev.xgrp_invdiag;
  a.xinvf = L.dev.xgrp_invdiagf;
  return a;
}

template <typename T>
GroupArgs<T> exchange_args(const Level& L, const void* x, void* y, const void* b, double omega, double* part) {
  GroupArgs<T> g;
  g.ngroups = (int)L.nxgroups();
  g.gptr = L.dev.xgrp_ptr;
  g.copies = L.dev.xcopies;
  g.cidx = L.dev.xcpidx;
  g.gflag = nullptr;
  g.ginv = L.dev.xgrp_invdiag;
  g.ginvf = L.dev.xgrp_invdiagf;
  g.md = L.dev.md;
  g.X = (const T*)x;
  g.Y = (T*)y;
  g.B = (const T*)b;
  g.omega = (T)omega;
  g.part = part ? part + L.tiles_for(dtype_of<T>()).size() / kWavesPerWG : nullptr;
  g.np = (int)L.n_partials(dtype_of<T>());
  return g;
}
inline int exchange_blocks(const Level& L) { return (int)L.xgroup_blocks(); }
// stencil passes of levels whose launch finishes shared DoFs need no exchange launch
inline bool exchange_in_launch(const Level& L) { return L.xfused; }

template <typename T>
GroupArgs<T> iface_args(const Level& L, const void* x, void* y, const void* b) {
  GroupArgs<T> g;
  g.ngroups = (int)L.ngroups();
  g.gptr = L.dev.grp_ptr;
  g.copies = L.dev.copies;
  g.cidx = L.dev.cpidx;
  g.gflag = L.dev.grp_flag;
  g.ginv = nullptr;
  g.ginvf = nullptr;
  g.md = L.dev.md;
  g.X = (const T*)x;
  g.Y = (T*)y;
  g.B = (const T*)b;
  g.omega = T(0);
  g.part = nullptr;
  g.np = 0;
  return g;
}
inline int iface_blocks(const Level& L) { return (int)L.iface_blocks(); }

// restriction: coarse points gather fine values; prolongation: fine points.
// At most kTransferBlocks workgroups; each wave walks several segments.
constexpr int kTransferBlocks = 8192;
inline int transfer_blocks(int nseg) {
  return std::min(kTransferBlocks, (nseg + kWavesPerWG - 1) / kWavesPerWG);
}
template <typename T>
TransferArgs<T> restrict_args(const Level& F, const Level& C, const void* rf, void* bc) {
  const int n = (int)C.psegs.size();
  return TransferArgs<T>{C.dev.psegs, n, transfer_blocks(n), C.dev.md, F.dev.md, (const T*)rf, (T*)bc,
                         C.dev.sbase, F.dev.sbase};
}
template <typename T>
TransferArgs<T> prolong_args(const Level& F, const Level& C, const void* ec, void* xf) {
  // 3D prolongations walk runs of slice segments, 2D single segments
  const bool runs = !F.pruns.empty();
  const int n = (int)(runs ? F.pruns.size() : F.psegs.size());
  return TransferArgs<T>{runs ? F.dev.pruns : F.dev.psegs, n, transfer_blocks(n), C.dev.md, F.dev.md,
                         (const T*)ec, (T*)xf, C.dev.sbase, F.dev.sbase};
}

template <typename T>
CoarseArgs<T> coarse_args(const Level& L, const void* b, void* x);
template <>
inline CoarseArgs<double> coarse_args<double>(const Level& L, const void* b, void* x) {
  return CoarseArgs<double>{(int)L.ncoarse, L.dev.cinv, L.dev.cfirst, L.dev.cptr, L.dev.cidx, (const double*)b,
                            (double*)x};
}
template <>
inline CoarseArgs<float> coarse_args<float>(const Level& L, const void* b, void* x) {
  return CoarseArgs<float>{(int)L.ncoarse, L.dev.cinvf, L.dev.cfirst, L.dev.cptr, L.dev.cidx, (const float*)b,
                           (float*)x};
}
inline int coarse_blocks(const Level& L) { return (int)((L.ncoarse + kWavesPerWG - 1) / kWavesPerWG); }

template <typename T>
Jacobi0Args<T> jacobi0_args(const Level& L, const void* b, void* y, double omega) {
  Jacobi0Args<T> a;
  a.nmac = (int)L.base.size();
  a.P = a.nmac > 0 ? L.storage / a.nmac : 0;
  a.bpm = (int)((a.P + kJ0Points - 1) / kJ0Points);
  a.nall = (int)L.ngroups();
  a.nblk_all = (a.nall + kWG - 1) / kWG;
  a.aptr = L.dev.grp_ptr;
  a.acopies = L.dev.copies;
  a.ngroups = (int)L.nxgroups();
  a.nblk_grp = (a.ngroups + kWG - 1) / kWG;
  a.gptr = L.dev.xgrp_ptr;
  a.copies = L.dev.xcopies;
  a.gidx = L.dev.xcpidx;
  a.ginv = L.dev.xgrp_invdiag;
  a.ginvf = L.dev.xgrp_invdiagf;
  a.md = L.dev.md;
  a.B = (const T*)b;
  a.Y = (T*)y;
  a.omega = (T)omega;
  return a;
}
template <typename T>
int jacobi0_stream_blocks(const Jacobi0Args<T>& a) { return a.nmac * a.bpm; }
template <typename T>
int jacobi0_fix_blocks(const Jacobi0Args<T>& a) { return a.nblk_all + a.nblk_grp; }

template <typename T>
TailLevel<T> tail_level(const Level& L, void* b, void* x, void* t) {
  TailLevel<T> v;
  v.nx = (int)L.nxgroups();
  v.xptr = L.dev.xgrp_ptr;
  v.xcopies = L.dev.xcopies;
  v.xcidx = L.dev.xcpidx;
  v.xinv = L.dev.xgrp_invdiag;
  v.xinvf = L.dev.xgrp_invdiagf;
  v.ng = (int)L.ngroups();
  v.gptr = L.dev.grp_ptr;
  v.copies = L.dev.copies;
  v.gcidx = L.dev.cpidx;
  v.gflag = L.dev.grp_flag;
  v.md = L.dev.md;
  v.storage = L.storage;
  v.N = L.N;
  v.nmac = (int)L.base.size();
  v.b = (T*)b;
  v.x = (T*)x;
  v.t = (T*)t;
  return v;
}

// Levels the tail of a V-cycle from `level` down to lc takes (0: none).
inline int tail_levels(const mf_mesh* m, int level, int lc) {
  if (kTailLevels < 1 || m->levels[lc].ncoarse > kTailMaxCoarse || m->levels[lc].storage > kTailMaxPoints) return 0;
  int n = 1;
  while (n < kTailLevels && lc + n <= level && m->levels[lc + n].storage <= kTailMaxPoints) ++n;
  return n;
}

inline VecArgs vec_args(void* y, const void* x, const double* res, int64_t n, double a) {
  return VecArgs{y, x, res, n, a, vec_blocks(n), 1};
}

inline PcgArgs pcg_args(const Level& L, double* x, double* r, double* p, const double* q, const void* e, double* z,
                        const double* res, double* part) {
  return PcgArgs{L.storage, L.dev.own_bits, x, r, p, q, e, z, res, part, nullptr, nullptr, (int)L.lin_blocks(), 1};
}
inline int pcg_blocks(const Level& L) { return (int)L.lin_blocks(); }

// ---------------------------------------------------------------- batch ops
enum OpKind : int {
  kOpStencil = 0,  // StencilArgs<T>, mode = kApply / kJacobi / kResidual / kNormB
  kOpExchange,     // GroupArgs<T>, same modes
  kOpIface,        // GroupArgs<T>, mode = kExchangeSum / kDirichletSet
  kOpReduce,       // ReduceArgs
  kOpRestrict,     // TransferArgs<T>
  kOpProlong,      // TransferArgs<T>
  kOpCoarse,       // CoarseArgs<T>
  kOpFill,         // VecArgs: y = a
  kOpCopy,         // VecArgs: y = x
  kOpAxpy,         // VecArgs: y += a x
  kOpScaleF32,     // VecArgs: float y = x / res[1]
  kOpAxpyF32,      // VecArgs: double y += res[1] * float x
  kOpPcgZDot,      // PcgArgs, dtype = type of e: z = s e, partials of r . z
  kOpPcgDir,       // VecArgs: y = x + beta y, beta = res[2] / res[3] (0 if res[3] == 0)
  kOpPcgUpdate,    // PcgArgs: x += alpha p, r -= alpha q, alpha = res[2] / res[4]; partials of r . r
  kOpJacobi0,      // Jacobi0Args<T>: y = omega D^-1 b (the first sweep from a zero iterate);
                   // mode 0: streaming pass over all points, mode 1: macro-boundary DoFs
  kOpTail,         // TailArgs<T>: the V-cycle below a level, one workgroup per request
};

// One batched launch: a table of nseg argument records at args_off and nseg+1
// workgroup offsets at wg0_off, inside the batch's device table.
struct BatchOp {
  int kind, dtype, dim, mode;
  int nseg, nwg;
  int64_t args_off, wg0_off;
  int variant;  // stencil ops: 3D tile shape of the members' levels (kPenZ or kPenSeg); tail ops: dynamic LDS bytes
  int pad_;
};

}  // namespace mf
