// Device helpers shared by the stencil, transfer and V-cycle tail kernels:
// precision-specific macro constants, the per-point partial stencil sum and
// row finish of the stencil kernels, argument resolution of batched
// launches, and the per-segment transfer and zero-iterate Jacobi steps.
#pragma once

#include <hip/hip_runtime.h>

#include "kargs.hpp"

namespace mf {

template <typename T>
struct Prec;

template <>
struct Prec<double> {
  static __device__ __forceinline__ double w(const MacroDev& M, int mask, int i) { return M.wm[mask][i]; }
  static __device__ __forceinline__ double invd(const MacroDev& M) { return M.inv_diag; }
  static __device__ __forceinline__ double ginv(const double* d, const float*, int g) { return d[g]; }
  static __device__ __forceinline__ const double* K(const MacroDev& M, int t) { return M.K[t]; }
};

template <>
struct Prec<float> {
  static __device__ __forceinline__ float w(const MacroDev& M, int mask, int i) { return M.wmf[mask][i]; }
  static __device__ __forceinline__ float invd(const MacroDev& M) { return M.inv_diagf; }
  static __device__ __forceinline__ float ginv(const double*, const float* f, int g) { return f[g]; }
  static __device__ __forceinline__ const float* K(const MacroDev& M, int t) { return M.Kf[t]; }
};

// Ordinary (write-back) stores: partial lines at wave boundaries merge in L2.
#ifndef MF_NT_STORE
#define MF_NT_STORE 0
#endif
template <typename T>
__device__ __forceinline__ void st(T* p, T v) {
  if (MF_NT_STORE) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// A macro's 16 x 16 partial-stencil table (row = support mask).  The stencil
// kernels keep a copy in LDS, so that the per-lane lookups of boundary lanes
// are LDS reads and never wait on the vector-memory counter that paces the
// row loads in flight; the V-cycle tail reads the macro record directly.
template <typename T>
using WTab = T (*)[16];

// Partial stencil sum for a point with support `mask`: neighbours outside
// the macro (whose values in v are clamped stand-ins) are dropped by
// selects, so the code is branch-free.
template <typename T, int DIM>
__device__ __forceinline__ T partial_sum(const WTab<T> W, int mask, int N, int x, int y, int z, const T* v) {
  constexpr StencilTable ST = stencil_table(DIM);
  T acc = T(0);
#pragma unroll
  for (int o = 0; o < ST.n; ++o) {
    const int nx = x + ST.off[o][0], ny = y + ST.off[o][1], nz = z + ST.off[o][2];
    const bool in = nx >= 0 && ny >= 0 && nz >= 0 && nx + ny + nz <= N;
    acc = fma(W[mask][o], in ? v[o] : T(0), acc);
  }
  return acc;
}

// Norm / dot partials of one finished row value `out` (xc = the point's x).
template <typename T, int MODE>
__device__ __forceinline__ void accum(double& ss, double& mx, T out, T xc) {
  if (MODE == kResidual || MODE == kNormB) {
    ss += (double)out * (double)out;
    mx = fmax(mx, fabs((double)out));
  } else if (MODE == kApplyDot) {
    ss += (double)xc * (double)out;  // (no maximum: only the dot product is used)
  }
}

// Finish the row of one point.  acc is its (partial) stencil value, xc and bv
// its x and b entries.  Interior points, Dirichlet points (identity rows) and
// points no other macro shares are finished here; shared non-Dirichlet points
// get their partial row for the exchange (KEEP_SHARED), or nothing where the
// same launch computes their whole rows (group_rows3).  Norm partials count
// each unique DoF once (Dirichlet DoFs on shared primitives only in their
// owner).
template <typename T, int DIM, int MODE, bool KEEP_SHARED = true>
__device__ __forceinline__ void finish(const MacroDev& M, const WTab<T> W, int mask, T acc, T xc, T bv, T omega,
                                       T* yp, double& ss, double& mx) {
  constexpr int FM = full_mask(DIM);
  constexpr StencilTable ST = stencil_table(DIM);
  const bool full = mask == FM;
  const bool dir = !full && ((M.dir_mask >> mask) & 1);
  const bool shared = !full && ((M.shared_mask >> mask) & 1);
  if (dir) {
    const T out = MODE == kResidual ? bv - xc : (MODE == kNormB ? bv : xc);
    if (MODE != kNormB) st(yp, out);
    if ((M.own_mask >> mask) & 1) accum<T, MODE>(ss, mx, out, xc);
  } else if (full || !shared) {
    T out;
    if (MODE == kApply || MODE == kApplyDot) out = acc;
    else if (MODE == kJacobi) out = fma(omega * (full ? Prec<T>::invd(M) : T(1) / W[mask][ST.centre]), bv - acc, xc);
    else if (MODE == kResidual) out = bv - acc;
    else out = bv;
    if (MODE != kNormB) st(yp, out);
    accum<T, MODE>(ss, mx, out, xc);
  } else if (MODE != kNormB && KEEP_SHARED) {
    st(yp, acc);
  }
}

// Argument tables are read-only for the whole launch: reading them through
// the constant address space lets the compiler use scalar loads, so the
// request's arguments stay in scalar registers as a by-value argument does.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* as_const(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

__device__ __forceinline__ int find_seg_c(const int32_t* wg0, int nseg, int g) {
  const auto* w = as_const(wg0);
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (w[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Resolves workgroup g of a launch to its request's arguments and the
// workgroup index inside that request.
template <class A>
__device__ __forceinline__ int resolve(const Launch<A>& L, int g, A& a) {
  if (L.nseg == 0) {
    a = L.one;
    return g;
  }
  const int r = find_seg_c(L.wg0, L.nseg, g);
#if defined(__HIP_DEVICE_COMPILE__)
  a = as_const(L.many)[r];
#else
  a = L.many[r];  // the host pass only type-checks device code
#endif
  return g - as_const(L.wg0)[r];
}

template <int DIM>
__device__ __forceinline__ int64_t lidx(int N, int x, int y, int z) {
  return DIM == 2 ? idx2(N, x, y) : idx3(N, x, y, z);
}

// Restriction r_c = P^T r_f on one macro: a coarse point P gathers the fine
// point 2P (weight 1) and the fine points 2P + d for the stencil offsets d
// (weight 1/2) — the fine points whose interpolation uses P — counting only
// fine points this macro owns, so that the later exchange sums each fine DoF
// once.  Dirichlet fine points are skipped.
// Segment and macro records are read-only for the launch: read them through
// the constant address space (scalar loads, scalar registers).
__device__ __forceinline__ Tile load_seg(const Tile* segs, int si) {
#if defined(__HIP_DEVICE_COMPILE__)
  return as_const(segs)[si];
#else
  return segs[si];
#endif
}

struct MacroC {
  int64_t base;
  int32_t N;
  uint16_t own_mask, dir_mask;
};

__device__ __forceinline__ MacroC load_macro(const MacroDev* md, int m) {
#if defined(__HIP_DEVICE_COMPILE__)
  const auto* p = as_const(md) + m;
  return MacroC{p->base, p->N, p->own_mask, p->dir_mask};
#else
  return MacroC{md[m].base, md[m].N, md[m].own_mask, md[m].dir_mask};
#endif
}

// Storage offsets of the 15 stencil neighbours of a 3D point (x, y, z),
// relative to the point, in stencil-table order; exact for neighbours inside
// the macro.  Slice z has side S = N - z and row y of it d = S + 1 - y
// points: rows y +- 1 start d after / end d + 1 before the point's column,
// and (x, y, z + 1) / (x, y, z - 1) lie T(S) - y after / T(S + 1) - y
// before it (T(s) = (s + 1)(s + 2) / 2 points in a slice of side s).
__device__ __forceinline__ void nbr_offsets3(int N, int y, int z, int (&o)[15]) {
  const int S = N - z, d = S + 1 - y;
  const int up = (S + 1) * (S + 2) / 2 - y;
  const int dn = y - (S + 2) * (S + 3) / 2;
  const int t[15] = {dn, dn + 1, dn + d + 1, dn + d, -d - 1, -d, -1, 0, 1, d - 1, d, up - d, up - d + 1, up - 1, up};
#pragma unroll
  for (int k = 0; k < 15; ++k) o[k] = t[k];
}

template <typename T, int DIM>
__device__ __forceinline__ void restrict_point(const TransferArgs<T>& a, int macro, int x, int y, int z) {
  constexpr StencilTable ST = stencil_table(DIM);
  constexpr int full = DIM == 2 ? 7 : 15;
  const MacroC C = load_macro(a.mdc, macro);
  const MacroC F = load_macro(a.mdf, macro);
  const int Nc = C.N, Nf = F.N;
  const bool live = x + y + z <= Nc;
  // 3D: the fine neighbours' indices as offsets from that of 2P
  int off[15];
  int64_t fc = 0;
  if constexpr (DIM == 3) {
    nbr_offsets3(Nf, live ? 2 * y : 0, 2 * z, off);
    fc = live ? lidx<3>(Nf, 2 * x, 2 * y, 2 * z) : 0;
  }
  // branch-free: every lane takes all offsets; fine points outside the macro
  // read the centre instead and contribute nothing
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < ST.n; ++s) {
    const int fx = 2 * x + ST.off[s][0], fy = 2 * y + ST.off[s][1], fz = DIM == 3 ? 2 * z + ST.off[s][2] : 0;
    const bool in = live && fx >= 0 && fy >= 0 && fz >= 0 && fx + fy + fz <= Nf;
    const int mask = support_mask(DIM, Nf, fx, fy, fz);
    const bool owned = mask == full || ((F.own_mask >> mask) & 1);
    const bool dir = mask != full && ((F.dir_mask >> mask) & 1);
    const bool use = in && owned && !dir;
    const int64_t i = in ? (DIM == 3 ? fc + off[s] : lidx<DIM>(Nf, fx, fy, fz)) : 0;
    const T r = a.src[F.base + i];
    const T w = s == ST.centre ? T(1) : T(0.5);
    acc += use ? w * r : T(0);
  }
  if (live) a.dst[C.base + lidx<DIM>(Nc, x, y, z)] = acc;
}
// (x, y) of slice-local index r in a 3D slice of side S <= 2048, r <
// (S+1)(S+2)/2: y is the smaller root of y^2 - (2S + 3) y + 2r = 0 (row y
// starts at y (2S + 3 - y) / 2), rounded down and corrected by one step
// either way.  The FP32 discriminant is exact or within an ulp and the
// hardware root within an ulp, far inside that correction.
__device__ __forceinline__ void slice_xy3(int S, int r, int& x, int& y) {
  const float b = 2.0f * (float)S + 3.0f;
  int yy = (int)((b - __builtin_amdgcn_sqrtf(b * b - 8.0f * (float)r)) * 0.5f);
  yy = min(max(yy, 0), S);
  if (row_start(S, yy) > r) --yy;
  else if (yy < S && row_start(S, yy + 1) <= r) ++yy;
  y = yy;
  x = r - row_start(S, yy);
}

// This lane's point of slice segment sg ({macro, first slice-local index, 0,
// z}) in a macro of side N: the slice of side S = N - z holds (S+1)(S+2)/2
// points, row y starting at y (2S + 3 - y) / 2, so y is the smaller root of
// y^2 - (2S + 3) y + 2r = 0, rounded down and corrected by one step either
// way.  Lanes past the slice's end get x = S + 1 (no point: x + y + z > N).
template <int DIM>
__device__ __forceinline__ void slice_point(const Tile& sg, int N, int& x, int& y, int& z) {
  z = DIM == 3 ? sg.z : 0;
  const int S = N - z;
  const int r = sg.x0 + (int)(threadIdx.x & (kWave - 1));
  if (r >= (S + 1) * (S + 2) / 2) {
    x = S + 1;
    y = 0;
    return;
  }
  if (DIM == 3) {
    slice_xy3(S, r, x, y);
    return;
  }
  // 2D: the discriminant reaches 2^32, exact in a double
  const double b = 2.0 * (double)S + 3.0;
  int yy = (int)((b - sqrt(b * b - 8.0 * (double)r)) * 0.5);
  yy = min(max(yy, 0), S);
  if (row_start(S, yy) > r) --yy;
  else if (yy < S && row_start(S, yy + 1) <= r) ++yy;
  y = yy;
  x = r - row_start(S, yy);
}

// Restriction over one 3D slice segment of coarse points: the same sum as
// restrict_point, in the same order, with cheaper index work.  Slice bases
// come from the per-level tables; the storage index of fine point 2P + d is
// formed from that of 2P (slice 2z of side S = Nf - 2z, row 2y of
// l = S + 1 - 2y points): +-1 along the row, l after / l + 1 before it for
// rows 2y +- 1, T(S) - 2y after and T(S + 1) - 2y before it for slices
// 2z +- 1 (T(s) = (s + 1)(s + 2) / 2 points in a slice of side s), all as
// 32-bit offsets from the first point of slice 2z - 1.  Whether 2P + d lies
// in the macro, and its support mask, follow from P's position:
// 2x + dx = 0 only for x = 0 and dx = 0, and Nf - |2P + d| =
// 2 (Nc - |P|) - |d| vanishes only on P's far face with |d| = 0.
// The lane's coarse point is slice-local index r of slice sg.z (in_run:
// inside its run of points).
template <typename T>
__device__ __forceinline__ T restrict_seg3(const TransferArgs<T>& a, const Tile sg, int r, bool in_run, int64_t& di,
                                           bool& wr) {
  constexpr StencilTable ST = stencil_table(3);
  constexpr int full = 15;
  const MacroC C = load_macro(a.mdc, sg.macro);
  const MacroC F = load_macro(a.mdf, sg.macro);
  const int Nc = C.N, Nf = F.N;
  const int z = sg.z;
  int x = Nc - z + 1, y = 0;  // lanes past the run or the slice: no point
  if (in_run && r < (Nc - z + 1) * (Nc - z + 2) / 2) slice_xy3(Nc - z, r, x, y);
  const bool live = x + y + z <= Nc;
  const bool x0 = x == 0, y0 = y == 0, z0 = z == 0, far = x + y + z == Nc;
  const int zf = 2 * z, S = Nf - zf, yf = live ? 2 * y : 0, xf = live ? 2 * x : 0;
  const int za = zf > 0 ? zf - 1 : 0;
  const T* __restrict__ Fa = a.src + F.base + as_const(a.sbf)[za];  // anchor: slice 2z - 1 (slice 0 at z = 0)
  const int tb = as_const(a.sbf)[zf] - as_const(a.sbf)[za];         // points of slice 2z - 1 (0 at z = 0)
  const int c = tb + row_start(S, yf) + xf;
  const int l = S + 1 - yf;
  const int up = c + (S + 1) * (S + 2) / 2 - yf;
  const int dn = c - tb + yf;
  const int rel[15] = {dn,     dn + 1,     dn + l + 1, dn + l, c - l - 1, c - l, c - 1, c,
                       c + 1,  c + l - 1,  c + l,      up - l, up - l + 1, up - 1, up};
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < ST.n; ++s) {
    const int dx = ST.off[s][0], dy = ST.off[s][1], dz = ST.off[s][2], sd = dx + dy + dz;
    const bool in = live && (dx >= 0 || !x0) && (dy >= 0 || !y0) && (dz >= 0 || !z0) && (sd <= 0 || !far);
    const int mask = ((sd == 0 && far) ? 0 : 1) | ((dx == 0 && x0) ? 0 : 2) | ((dy == 0 && y0) ? 0 : 4) |
                     ((dz == 0 && z0) ? 0 : 8);
    const bool owned = mask == full || ((F.own_mask >> mask) & 1);
    const bool dir = mask != full && ((F.dir_mask >> mask) & 1);
    const bool use = in && owned && !dir;
    // points outside the macro read the anchor (value unused)
    const T r = Fa[in ? (unsigned)rel[s] : 0u];
    const T w = s == ST.centre ? T(1) : T(0.5);
    acc += use ? w * r : T(0);
  }
  di = C.base + as_const(a.sbc)[z] + r;
  wr = live;
  return acc;
}

// 2D: one 64-point segment of coarse points.
template <typename T, int DIM>
__device__ __forceinline__ void restrict_segment(const TransferArgs<T>& a, const Tile sg) {
  int x, y, z;
  slice_point<DIM>(sg, load_macro(a.mdc, sg.macro).N, x, y, z);
  restrict_point<T, DIM>(a, sg.macro, x, y, z);
}

// x_f += P e_c: even fine points take the coarse value, the others the mean
// of the two coarse endpoints of the coarse micro-edge they bisect; the
// edge direction follows from the coordinate parities.  Dirichlet points are
// left unchanged.
template <typename T, int DIM>
__device__ __forceinline__ void prolong_point(const TransferArgs<T>& a, int macro, int x, int y, int z) {
  constexpr int full = DIM == 2 ? 7 : 15;
  const MacroC C = load_macro(a.mdc, macro);
  const MacroC F = load_macro(a.mdf, macro);
  const int Nc = C.N, Nf = F.N;
  const bool live = x + y + z <= Nf;
  const int mask = support_mask(DIM, Nf, x, y, z);
  const bool dir = mask != full && ((F.dir_mask >> mask) & 1);
  // direction s of the coarse micro-edge the point bisects: the parity
  // pattern, with the middle odd coordinate negated for two or three odd
  // coordinates ((1,1,0) -> e1 - e2, (1,0,1) -> e1 - e3, (0,1,1) -> e2 - e3,
  // (1,1,1) -> e1 - e2 + e3); even points have s = 0 and take the coarse
  // value itself (the two reads coincide)
  // (lanes past the macro's far face read the coarse point (0, 0, 0))
  const int xl = live ? x : 0, yl = live ? y : 0, zl = live ? z : 0;
  const int px = xl & 1, py = yl & 1, pz = zl & 1;
  const int sx = px;
  const int sy = (px && py) ? -1 : py;
  const int sz = (pz && (px ^ py)) ? -1 : pz;
  const T u = a.src[C.base + lidx<DIM>(Nc, (xl - sx) >> 1, (yl - sy) >> 1, (zl - sz) >> 1)];
  const T v = a.src[C.base + lidx<DIM>(Nc, (xl + sx) >> 1, (yl + sy) >> 1, (zl + sz) >> 1)];
  if (live && !dir) a.dst[F.base + lidx<DIM>(Nf, x, y, z)] += T(0.5) * (u + v);
}
// Prolongation over one 3D slice segment of fine points: prolong_point's
// update, with the slice bases from the per-level tables and the coarse
// points addressed by 32-bit offsets from the first point of coarse slice
// z / 2 (the other coarse slice, (z + 1) / 2, follows it), the fine point by
// its slice-local index.
// The lane's fine point is slice-local index r of slice sg.z (in_run: inside
// its run of points).
template <typename T>
__device__ __forceinline__ void prolong_seg3(const TransferArgs<T>& a, const Tile sg, int r, bool in_run,
                                             int64_t& di, T& u, T& v, bool& wr) {
  constexpr int full = 15;
  const MacroC C = load_macro(a.mdc, sg.macro);
  const MacroC F = load_macro(a.mdf, sg.macro);
  const int Nc = C.N, Nf = F.N;
  const int z = sg.z;
  int x = Nf - z + 1, y = 0;  // lanes past the run or the slice: no point
  if (in_run && r < (Nf - z + 1) * (Nf - z + 2) / 2) slice_xy3(Nf - z, r, x, y);
  const bool live = x + y + z <= Nf;
  const int mask = support_mask(3, Nf, x, y, z);
  const bool dir = mask != full && ((F.dir_mask >> mask) & 1);
  // dead lanes read the coarse points of (0, 0, z)
  const int xl = live ? x : 0, yl = live ? y : 0;
  const int px = xl & 1, py = yl & 1, pz = z & 1;
  const int sx = px;
  const int sy = (px && py) ? -1 : py;
  const int sz = (pz && (px ^ py)) ? -1 : pz;
  // coarse slices (z - sz) / 2 and (z + sz) / 2 are z / 2 or (z + 1) / 2
  const int zl = z >> 1, zh = (z + 1) >> 1;
  const T* __restrict__ Cl = a.src + C.base + as_const(a.sbc)[zl];
  const int dh = as_const(a.sbc)[zh] - as_const(a.sbc)[zl];
  const int zu = sz < 0 ? zh : zl, zv = sz > 0 ? zh : zl;
  u = Cl[(unsigned)((sz < 0 ? dh : 0) + row_start(Nc - zu, (yl - sy) >> 1) + ((xl - sx) >> 1))];
  v = Cl[(unsigned)((sz > 0 ? dh : 0) + row_start(Nc - zv, (yl + sy) >> 1) + ((xl + sx) >> 1))];
  // dead lanes name the macro's first point (a valid address, never written)
  di = F.base + (live ? as_const(a.sbf)[z] + r : 0);
  wr = live && !dir;
}

// 2D: one 64-point segment of fine points.
template <typename T, int DIM>
__device__ __forceinline__ void prolong_segment(const TransferArgs<T>& a, const Tile sg) {
  int x, y, z;
  slice_point<DIM>(sg, load_macro(a.mdf, sg.macro).N, x, y, z);
  prolong_point<T, DIM>(a, sg.macro, x, y, z);
}

// First Jacobi sweep of a V-cycle level.  The iterate is zero there, so
// x' = x + omega D^-1 (b - A x) reduces to omega D^-1 b, with D the diagonal
// of the row the sweep would finish: the macro's interior centre weight, the
// partial stencil's centre at a boundary point no other macro shares, the
// assembled diagonal of a shared DoF (exchange list), and x' = x = 0 at
// Dirichlet DoFs.  The arithmetic is that of the stencil and exchange
// kernels with x = 0 (fma(omega d, b - 0, 0)), so the result is bitwise
// the same, in one pass that reads b once and needs no exchange.
template <typename T>
__device__ __forceinline__ T centre_inv(const MacroDev& M, int mask, int full, int centre) {
  if constexpr (sizeof(T) == 8) return mask == full ? M.inv_diag : 1.0 / M.wm[mask][centre];
  else return mask == full ? M.inv_diagf : 1.0f / M.wmf[mask][centre];
}

template <typename T, int DIM>
__device__ __forceinline__ void jacobi0_point(const Jacobi0Args<T>& a, int macro, int x, int y, int z) {
  constexpr int full = DIM == 2 ? 7 : 15;
  constexpr int centre = stencil_table(DIM).centre;
  const MacroDev& M = a.md[macro];
  const MacroC C = load_macro(a.md, macro);
  const int N = C.N;
  if (x + y + z > N) return;
  const int mask = support_mask(DIM, N, x, y, z);
  const bool dir = mask != full && ((C.dir_mask >> mask) & 1);
  const bool shared = mask != full && !dir && ((M.shared_mask >> mask) & 1);
  if (shared) return;  // finished by the group part
  const int64_t i = C.base + lidx<DIM>(N, x, y, z);
  a.Y[i] = dir ? T(0) : fma(a.omega * centre_inv<T>(M, mask, full, centre), a.B[i], T(0));
}

template <int DIM>
__device__ __forceinline__ int64_t copy_index(const MacroDev& M, const Copy& c) {
  return M.base + (DIM == 2 ? idx2(M.N, c.x, c.y) : idx3(M.N, c.x, c.y, c.z));
}

// One DoF shared by several macros and not Dirichlet (exchange list): its
// copies in Y hold partial rows; sum them in fixed macro order, finish the
// row and write it to every copy.  Returns the row value; i0 = index of the
// first copy.
template <typename T, int DIM, int MODE>
__device__ __forceinline__ T exchange_row(const GroupArgs<T>& a, int g, int64_t& i0) {
  const int c0 = a.gptr[g], c1 = a.gptr[g + 1];
  i0 = a.cidx[c0];
  T out;
  if (MODE == kNormB) {
    out = a.B[i0];
  } else {
    T acc = T(0);
    for (int c = c0; c < c1; ++c) acc += a.Y[a.cidx[c]];
    if (MODE == kApply || MODE == kApplyDot) out = acc;
    else if (MODE == kJacobi) out = fma(a.omega * Prec<T>::ginv(a.ginv, a.ginvf, g), a.B[i0] - acc, a.X[i0]);
    else out = a.B[i0] - acc;
    for (int c = c0; c < c1; ++c) a.Y[a.cidx[c]] = out;
  }
  return out;
}

// One macro-boundary DoF (all-groups list): y = the sum of x over its copies
// (0 at Dirichlet DoFs), written to every copy (in place allowed).
template <typename T, int DIM>
__device__ __forceinline__ void iface_sum_row(const GroupArgs<T>& a, int g) {
  const int c0 = a.gptr[g], c1 = a.gptr[g + 1];
  const bool dir = a.gflag[g] & 1;
  T out = T(0);
  if (!dir)
    for (int c = c0; c < c1; ++c) out += a.X[a.cidx[c]];
  for (int c = c0; c < c1; ++c) a.Y[a.cidx[c]] = out;
}

// Coarse direct solve, unknown i, one wavefront (lane = its lane):
// x(copies of i) = sum_j Ainv[i][j] b(first copy of j).
template <typename T>
__device__ __forceinline__ void coarse_row(const CoarseArgs<T>& a, int i, int lane) {
  T acc = T(0);
  for (int j = lane; j < a.n; j += kWave) acc = fma(a.Ainv[(int64_t)i * a.n + j], a.B[a.first[j]], acc);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  for (int c = a.cptr[i] + lane; c < a.cptr[i + 1]; c += kWave) a.X[a.cidx[c]] = acc;
}

// The zero-iterate Jacobi row of shared non-Dirichlet DoF g (exchange list),
// written to every copy.
template <typename T, int DIM>
__device__ __forceinline__ void jacobi0_group(const Jacobi0Args<T>& a, int g) {
  const int c0 = a.gptr[g], c1 = a.gptr[g + 1];
  const T b = a.B[a.gidx[c0]];
  T d;
  if constexpr (sizeof(T) == 8) d = a.ginv[g];
  else d = a.ginvf[g];
  const T out = fma(a.omega * d, b, T(0));
  for (int c = c0; c < c1; ++c) a.Y[a.gidx[c]] = out;
}

}  // namespace mf
