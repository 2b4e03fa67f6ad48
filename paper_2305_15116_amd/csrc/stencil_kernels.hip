// Constant-stencil kernels for CDNA4 (gfx950): the operator's rows for every
// point of every macro (apply, weighted Jacobi, residual + norm partials),
// the exchange that completes rows of DoFs shared by several macros, and the
// deterministic norm reduction.
//
// The paper's vertex-to-vertex kernel (Performance Modeling section) walks
// one triangle row by row, x fastest, reading seven neighbours with constant
// weights; on a CPU its speed depends on whether three source rows plus the
// destination row fit in a cache level (the layer condition).  Here the same
// reuse is kept in registers: a 64-lane wavefront owns 64 consecutive
// columns and walks rows upward (2D), or walks a pencil of rows upward
// through the slices (3D), holding the rows the stencil needs and taking the
// x+-1 neighbours from adjacent lanes through DPP shifts, so each source
// value is read from memory once per tile; future rows are loaded ahead to
// keep enough bytes in flight for HBM3E.  No matrix cores: the path is
// HBM-bound.
//
// Macro-boundary DoFs are handled in the same walk (the paper leaves them to
// interface primitives, Performance Modeling, experiment description): a
// point on a face, edge or vertex of its macro uses the partial stencil of
// its support mask — only the micro-elements on its side — and a DoF shared
// by several macros is finished by the exchange kernel, which sums the
// copies' partial rows in fixed macro order and writes the result to every
// copy.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "rows.hpp"
#include "wave.hpp"

namespace mf {

namespace {


using wave::dn1;
using wave::up1;
using wave::xcd_wg;


__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

#ifndef MF_RING_U2
#define MF_RING_U2 8
#endif
constexpr int kU2 = MF_RING_U2;  // rows loaded ahead (2D)
static_assert(kTileH2 % kU2 == 0, "ring depth must divide the tile height");
static_assert(kTileH2F % kRingU2F == 0, "ring depth must divide the tile height");

// 2D tile height and load-ring depth per precision.
template <typename T>
struct Tile2 {
  static constexpr int H = kTileH2, U = kU2;
};
template <>
struct Tile2<float> {
  static constexpr int H = kTileH2F, U = kRingU2F;
};


// Copies the 16 x 16 partial-stencil table of macro M into W with `nthreads`
// threads starting at `first` (a wave or the whole workgroup).
template <typename T>
__device__ __forceinline__ void load_wtab(const MacroDev& M, WTab<T> W, int first, int nthreads) {
  for (int i = (int)threadIdx.x - first; i < 256; i += nthreads)
    if (i >= 0) W[i >> 4][i & 15] = Prec<T>::w(M, i >> 4, i & 15);
}




// Interior finish of one row value (full stencil, interior point).
template <typename T, int MODE>
__device__ __forceinline__ void finish_interior(const MacroDev& M, T acc, T xc, T bv, T omega, T* yp, double& ss,
                                                double& mx) {
  T out;
  if (MODE == kApply || MODE == kApplyDot) out = acc;
  else if (MODE == kJacobi) out = fma(omega * Prec<T>::invd(M), bv - acc, xc);
  else if (MODE == kResidual) out = bv - acc;
  else out = bv;
  if (MODE != kNormB) st(yp, out);
  accum<T, MODE>(ss, mx, out, xc);
}

// Support masks of the boundary lanes of rows off the y = 0 (and, in 3D,
// z = 0) faces: the row's first point (x = 0), its last (far face) or both.
template <int DIM>
struct RowMasks {
  static constexpr int L = full_mask(DIM) & ~2;   // x = 0
  static constexpr int F = full_mask(DIM) & ~1;   // far face
  static constexpr int LF = full_mask(DIM) & ~3;  // both
};

// Row of one point from its neighbour values v (xc = its x, bv = its b).
// may_face (a compile-time constant after unrolling) marks the rows that can
// lie on the y = 0 / z = 0 faces: those go through the general per-lane
// path.  In other rows a boundary lane is the row's first point (x = 0, only
// in tiles starting at x0 = 0, tile_left), its last (on the far face
// x + y + z = N), or both.  A row without such a lane takes the interior
// stencil from scalar registers, and so does a row whose boundary lanes are
// all Dirichlet points (they copy x).  Any other row takes, in every lane,
// the partial stencil of the lane's own support mask from the LDS table
// (interior lanes read the full stencil there, the same weights); the
// neighbours such a lane lacks (x - 1 for x = 0, the offsets of coordinate
// sum +1 on the far face) have weight 0 in its table row, and their
// stand-in values are replaced by 0 so that those terms add exactly nothing.
// The terms are summed in table order in every case, so a boundary row is
// the sum over the neighbours it has, in that order.  Jacobi needs bid =
// 1 / centre weight of the L, F and LF masks.
template <typename T, int DIM, int MODE, bool KEEP_SHARED = true>
__device__ __forceinline__ void point_row(const MacroDev& M, const WTab<T> W, const T* wi, bool inside, int N, int x,
                                          int y, int z, const T* v, T xc, T bv, T omega, T* yp, double& ss,
                                          double& mx, bool may_face, bool tile_left, const T* bid) {
  constexpr StencilTable ST = stencil_table(DIM);
  constexpr int FM = full_mask(DIM);
  constexpr int NO = ST.n;
  if (may_face && (y == 0 || (DIM == 3 && z == 0))) {
    // a row on the y = 0 or z = 0 face: every lane is a boundary point
    if (__builtin_amdgcn_ballot_w64(inside)) {
      const int mask = support_mask(DIM, N, x, y, z);
      const T acc = partial_sum<T, DIM>(W, inside ? mask : FM, N, x, y, z, v);
      if (inside) finish<T, DIM, MODE, KEEP_SHARED>(M, W, mask, acc, xc, bv, omega, yp, ss, mx);
    }
    return;
  }
  const bool far = inside && x + y + z == N;
  const bool left = tile_left && inside && x == 0;
  if (!__builtin_amdgcn_ballot_w64(far || left)) {
    T acc = wi[0] * v[0];
#pragma unroll
    for (int o = 1; o < NO; ++o) acc = fma(wi[o], v[o], acc);
    if (inside) finish_interior<T, MODE>(M, acc, xc, bv, omega, yp, ss, mx);
    return;
  }
  const bool bnd = far || left;
  const int bm = FM & ~(far ? 1 : 0) & ~(left ? 2 : 0);
  const bool dir = bnd && ((M.dir_mask >> bm) & 1);
  T a = T(0);
  if (!__builtin_amdgcn_ballot_w64(bnd && !dir)) {
    // the row's boundary lanes are all Dirichlet (they copy x): the others
    // take the interior stencil
    a = wi[0] * v[0];
#pragma unroll
    for (int o = 1; o < NO; ++o) a = fma(wi[o], v[o], a);
  } else {
    const T* wr = W[bm];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      T vo = v[o];
      if (ST.off[o][0] + ST.off[o][1] + ST.off[o][2] > 0) vo = far ? T(0) : vo;
      if (ST.off[o][0] < 0) vo = left ? T(0) : vo;
      a = o == 0 ? wr[0] * vo : fma(wr[o], vo, a);
    }
  }
  const bool shared = bnd && !dir && ((M.shared_mask >> bm) & 1);
  const bool own = !bnd || ((M.own_mask >> bm) & 1);
  T out;
  if (MODE == kApply || MODE == kApplyDot) {
    out = dir ? xc : a;
  } else if (MODE == kJacobi) {
    const T id = !bnd ? Prec<T>::invd(M) : far ? (left ? bid[2] : bid[1]) : bid[0];
    out = dir ? xc : (shared ? a : fma(omega * id, bv - a, xc));
  } else if (MODE == kResidual) {
    out = dir ? bv - xc : (shared ? a : bv - a);
  } else {
    out = bv;
  }
  if (inside) {
    if (MODE != kNormB && (KEEP_SHARED || !shared)) st(yp, out);
    if (dir ? own : !shared) accum<T, MODE>(ss, mx, out, xc);
  }
}

// ------------------------------------------------------------------ row loads
// Start of row y in a triangle of side S in 32-bit arithmetic (exact for
// every supported level: S <= 32768).
__device__ __forceinline__ int rs32(int S, int y) { return y * (S + 2) - ((y * (y + 1)) >> 1); }

// Value at column xc (>= 0) of row r of a triangle of side S stored at base,
// with the row clamped to [0, last] and the column into the row: a valid
// point for every lane, so loads need no predicate and the unrolled loops
// stay straight-line code (clamped values are never used).  The row address
// is wave-uniform (scalar registers); only the unsigned column offset is per
// lane.
template <typename T>
__device__ __forceinline__ T ldrow(const T* __restrict__ base, int S, int r, int last, int xc) {
  // the row is clamped into [0, S] as well: `last` may name the row past the
  // triangle's apex, and the column offset must stay non-negative
  const int rr = min(max(r, 0), min(last, S));
  const unsigned byte = (unsigned)min(xc, S - rr) * (unsigned)sizeof(T);
  return *(const T*)((const char*)(base + rs32(S, rr)) + byte);
}

// ------------------------------------------------------------------ 2D tile
template <typename T, int MODE>
__device__ __forceinline__ void tile2d(const int x0, const int y0, const MacroDev& M, WTab<T> W,
                                       const T* __restrict__ X, T* __restrict__ Y, const T* __restrict__ B,
                                       T omega, double& ss, double& mx) {
  constexpr int FM = full_mask(2);
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int x = x0 - 1 + lane;
  constexpr int kH = Tile2<T>::H, kU = Tile2<T>::U;
  const int y1 = min(y0 + kH, N - x0 + 1);  // rows y0 .. y1-1 (x0 + y <= N)
  X += M.base;
  Y += M.base;
  if (MODE != kApply) B += M.base;
  T wi[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) wi[o] = Prec<T>::w(M, FM, o);
  T bid[3] = {T(0), T(0), T(0)};
  if (MODE == kJacobi) {
    constexpr int c = stencil_table(2).centre;
    bid[0] = T(1) / W[RowMasks<2>::L][c];
    bid[1] = T(1) / W[RowMasks<2>::F][c];
    bid[2] = T(1) / W[RowMasks<2>::LF][c];
  }

  const int xc = max(x, 0);
  T am = ldrow(X, N, y0 - 1, y1, xc);
  T a0 = ldrow(X, N, y0, y1, xc);
  T am_r = dn1(am), a0_l = up1(a0), a0_r = dn1(a0);
  T q[kU], qb[kU];
#pragma unroll
  for (int k = 0; k < kU; ++k) {
    q[k] = ldrow(X, N, y0 + 1 + k, y1, xc);                    // x rows y0+1 ..
    if (MODE != kApply) qb[k] = ldrow(B, N, y0 + k, y1 - 1, xc);  // b rows = output rows
  }
  // The tile's rows are fully unrolled so that the load ring needs no
  // register copies at a loop back-edge (which would wait for every load in
  // flight).  Loads are unconditional; rows past the tile's end only skip
  // the arithmetic (a uniform branch).
  const int nrows = y1 - y0;
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    const int yy = y0 + k;
    const T ap = q[k % kU];
    const T bv = MODE != kApply ? qb[k % kU] : T(0);
    // (compile-time guards: a ring slot is refilled only if a later row of
    // this tile reads it)
    if (k + kU < kH) q[k % kU] = ldrow(X, N, y0 + 1 + k + kU, y1, xc);
    if (MODE != kApply && k + kU < kH) qb[k % kU] = ldrow(B, N, y0 + k + kU, y1 - 1, xc);
    if (k >= nrows) continue;
    const T ap_l = up1(ap), ap_r = dn1(ap);
    const T v[7] = {am, am_r, a0_l, a0, a0_r, ap_l, ap};
    const bool inside = lane >= 1 && lane <= kTileW && x + yy <= N;
    point_row<T, 2, MODE>(M, W, wi, inside, N, x, yy, 0, v, a0, bv, omega, Y + rs32(N, yy) + (unsigned)xc, ss, mx,
                          k == 0, x0 == 0, bid);
    am = a0;
    am_r = a0_r;
    a0 = ap;
    a0_l = ap_l;
    a0_r = ap_r;
  }
}

// Interior 2D tile: every row y0-1 .. y0+H exists and holds every column
// x0-1 .. x0+62, and no output point lies on the macro's boundary.  Row
// addresses are then advanced incrementally (row y+1 starts N+1-y entries
// after row y) with no clamping, and every output lane takes the interior
// finish.
template <typename T>
__device__ __forceinline__ bool tile2d_inner(int x0, int y0, int N) {
  return x0 >= 1 && y0 >= 1 && x0 + y0 + kTileW + Tile2<T>::H <= N;
}

template <typename T, int MODE>
__device__ __forceinline__ void tile2d_fast(const int x0, const int y0, const MacroDev& M, const T* __restrict__ X,
                                            T* __restrict__ Y, const T* __restrict__ B, T omega, double& ss,
                                            double& mx) {
  constexpr int kH = Tile2<T>::H, kU = Tile2<T>::U;
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const bool out_lane = (unsigned)(lane - 1) < (unsigned)kTileW;
  const unsigned col = (unsigned)(x0 - 1 + lane) * (unsigned)sizeof(T);
  T wi[7];
#pragma unroll
  for (int o = 0; o < 7; ++o) wi[o] = Prec<T>::w(M, full_mask(2), o);
  // cursors: byte address of the next row and the byte step to the one after
  const char* px = (const char*)(X + M.base + rs32(N, y0 - 1));
  int sx = (N + 2 - y0) * (int)sizeof(T);
  char* py = (char*)(Y + M.base + rs32(N, y0));
  int sy = (N + 1 - y0) * (int)sizeof(T);
  const char* pb = MODE != kApply ? (const char*)(B + M.base + rs32(N, y0)) : nullptr;
  int sb = sy;
  auto ldx = [&]() -> T {
    const T v = *(const T*)(px + col);
    px += sx;
    sx -= (int)sizeof(T);
    return v;
  };
  auto ldb = [&]() -> T {
    const T v = *(const T*)(pb + col);
    pb += sb;
    sb -= (int)sizeof(T);
    return v;
  };
  T am = ldx();
  T a0 = ldx();
  T am_r = dn1(am), a0_l = up1(a0), a0_r = dn1(a0);
  T q[kU], qb[kU];
#pragma unroll
  for (int k = 0; k < kU; ++k) {
    q[k] = ldx();
    if (MODE != kApply) qb[k] = ldb();
  }
#pragma unroll
  for (int k = 0; k < kH; ++k) {
    const T ap = q[k % kU];
    const T bv = MODE != kApply ? qb[k % kU] : T(0);
    if (k + 1 + kU <= kH) q[k % kU] = ldx();
    if (MODE != kApply && k + kU < kH) qb[k % kU] = ldb();
    const T ap_l = up1(ap), ap_r = dn1(ap);
    const T v[7] = {am, am_r, a0_l, a0, a0_r, ap_l, ap};
    T acc = wi[0] * v[0];
#pragma unroll
    for (int o = 1; o < 7; ++o) acc = fma(wi[o], v[o], acc);
    if (out_lane) finish_interior<T, MODE>(M, acc, a0, bv, omega, (T*)(py + col), ss, mx);
    py += sy;
    sy -= (int)sizeof(T);
    am = a0;
    am_r = a0_r;
    a0 = ap;
    a0_l = ap_l;
    a0_r = ap_r;
  }
}

// ------------------------------------------------------------------ 3D pencil
// Slice z of a tetrahedral macro is a triangle of side S = N - z.  Output row
// y of slice z reads rows y, y+1 of slice z-1, rows y-1..y+1 of slice z and
// rows y-1, y of slice z+1.  A wave keeps rows y0-1 .. y0+kPenR of five
// consecutive slices in registers (z-1, z, z+1 and two in flight) and walks
// z upward, so each value is loaded once per pencil.  Rows, columns and
// slices outside the macro are clamped to a valid point (values never used).
template <typename T, int MODE, int PZ>
__device__ __forceinline__ void pencil3d(const int x0, const int y0, const int z0, const MacroDev& M, WTab<T> W,
                                         const T* __restrict__ X, T* __restrict__ Y, const T* __restrict__ B,
                                         T omega, double& ss, double& mx) {
  constexpr int FM = full_mask(3);
  constexpr int NS = 5;
  constexpr int NR = kPenR + 2;
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int x = x0 - 1 + lane;
  const int nz = min(PZ, N + 1 - x0 - y0 - z0);  // output slices z0 .. z0+nz-1
  X += M.base;
  Y += M.base;
  if (MODE != kApply) B += M.base;
  T wi[15];
#pragma unroll
  for (int o = 0; o < 15; ++o) wi[o] = Prec<T>::w(M, FM, o);
  T bid[3] = {T(0), T(0), T(0)};
  if (MODE == kJacobi) {
    constexpr int c = stencil_table(3).centre;
    bid[0] = T(1) / W[RowMasks<3>::L][c];
    bid[1] = T(1) / W[RowMasks<3>::F][c];
    bid[2] = T(1) / W[RowMasks<3>::LF][c];
  }
  const int xc = max(x, 0);
  // Slice z of a macro starts at sum_{k<z} (S_k+1)(S_k+2)/2, S_k = N - k;
  // bases are advanced incrementally (slices past N are clamped to slice N).
  auto next_base = [&](int64_t zb, int zp) -> int64_t {  // base of slice zp+1 given base of zp
    const int S = N - zp;
    return zp >= N ? zb : zb + ((int64_t)(S + 1) * (S + 2) >> 1);
  };
  auto ld = [&](const T* __restrict__ base, int64_t zb, int zp, int y) -> T {
    const int S = N - min(zp, N);
    return ldrow(base + zb, S, y, S, xc);
  };
  T s[NS][NR];
  int64_t lb = z0 > 0 ? slice_base(N, z0 - 1) : 0;  // base of the next slice to load
  int lz = max(z0 - 1, 0);                          // its (clamped) index
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int j = 0; j < NR; ++j) s[i][j] = ld(X, lb, lz, y0 - 1 + j);
    if (z0 - 1 + i >= 0) {
      lb = next_base(lb, lz);
      lz = min(lz + 1, N);
    }
  }
  int64_t zb = slice_base(N, z0);  // output slice base
  T bq[2][kPenR];
  if (MODE != kApply) {
#pragma unroll
    for (int j = 0; j < kPenR; ++j) bq[0][j] = ld(B, zb, z0, y0 + j);
  }
#pragma unroll
  for (int k = 0; k < PZ; ++k) {
    const int z = z0 + k;
    const int64_t zb1 = next_base(zb, min(z, N));
    if (MODE != kApply && k + 1 < PZ) {
#pragma unroll
      for (int j = 0; j < kPenR; ++j) bq[(k + 1) % 2][j] = ld(B, zb1, z + 1, y0 + j);
    }
    const T* A = s[k % NS];
    const T* Bs = s[(k + 1) % NS];
    const T* C = s[(k + 2) % NS];
    if (k < nz) {
      const int S = N - z;
      T* Yz = Y + zb;
#pragma unroll
      for (int j = 1; j <= kPenR; ++j) {
        const int y = y0 + j - 1;
        const T v[15] = {A[j],      dn1(A[j]),  A[j + 1],      up1(A[j + 1]), Bs[j - 1],
                         dn1(Bs[j - 1]), up1(Bs[j]), Bs[j],     dn1(Bs[j]),    up1(Bs[j + 1]),
                         Bs[j + 1], C[j - 1],   dn1(C[j - 1]), up1(C[j]),     C[j]};
        const bool inside = lane >= 1 && lane <= kTileW && x + y + z <= N;
        const T bv = MODE != kApply ? bq[k % 2][j - 1] : T(0);
        point_row<T, 3, MODE>(M, W, wi, inside, N, x, y, z, v, Bs[j], bv, omega, Yz + rs32(S, y) + (unsigned)xc, ss,
                              mx, j == 1 || k == 0, x0 == 0, bid);
      }
    }
    // slice z-1 is done: its slot takes the next slice (z+4)
#pragma unroll
    for (int j = 0; j < NR; ++j) s[k % NS][j] = ld(X, lb, lz, y0 - 1 + j);
    lb = next_base(lb, lz);
    lz = min(lz + 1, N);
    zb = zb1;
  }
}




// ------------------------------------------------------------ 3D slice runs
// A run of t.y0 consecutive points of slice z from slice-local index t.x0,
// one point per lane, 64 at a time.  Relative to the point's own index p in
// slice z (side S = N - z; row y holds d = S + 1 - y points): row y + 1 of
// the slice starts d after p's column, row y - 1 ends d + 1 before it; the
// point (x, y, z + 1) lies T(S) - y after p and (x, y, z - 1) lies
// T(S + 1) - y before it, T(s) = (s + 1)(s + 2) / 2 being the points of a
// slice of side s.  The 15 neighbours are therefore seven row positions and
// their +-1 columns.  Indices are formed relative to the first point of
// slice z - 1 (of slice 0 at z = 0), so every offset is a non-negative
// 32-bit value.  Lattice points outside the macro map to some index of the
// neighbouring slices; for 1 <= z <= N - 2 every such index stays inside
// the macro, elsewhere the indices are clamped into it.  Those values are
// stand-ins that the boundary rows never use (point_row).
template <typename T, int MODE>
__device__ __forceinline__ void seg3d(const Tile& t, const MacroDev& M, WTab<T> W, const T* __restrict__ X,
                                      T* __restrict__ Y, const T* __restrict__ B, T omega, double& ss, double& mx) {
  constexpr int FM = full_mask(3);
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N, z = t.z, S = N - z;
  T wi[15];
#pragma unroll
  for (int o = 0; o < 15; ++o) wi[o] = Prec<T>::w(M, FM, o);
  T bid[3] = {T(0), T(0), T(0)};
  if (MODE == kJacobi) {
    constexpr int c = stencil_table(3).centre;
    bid[0] = T(1) / W[RowMasks<3>::L][c];
    bid[1] = T(1) / W[RowMasks<3>::F][c];
    bid[2] = T(1) / W[RowMasks<3>::LF][c];
  }
  const int za = max(z - 1, 0);
  const int64_t ab = M.base + slice_base(N, za);
  const T* Xa = X + ab;
  const int Ts = (S + 1) * (S + 2) / 2;                 // points of slice z
  const int Tb = z > 0 ? (S + 2) * (S + 3) / 2 : 0;     // points of slice z - 1: offset of slice z
  const bool safe = z >= 1 && z + 2 <= N;
  // highest index of the three slices around z, inside the macro
  const int hi = (int)min(tet_count_small(N + 1) - slice_base(N, za) - 1, (int64_t)Tb + 2 * (int64_t)Ts);
  auto ld = [&](int i) -> T {
    if (!safe) i = min(max(i, 0), hi);
    return *(const T*)((const char*)Xa + (unsigned)i * (unsigned)sizeof(T));
  };
#pragma unroll
  for (int k = 0; k < kSegRun; ++k) {
    if (k * kWave >= t.y0) break;  // wave-uniform
    int r = t.x0 + k * kWave + lane;
    const bool live = k * kWave + lane < t.y0;
    if (!live) r = 0;
    int x, y;
    slice_xy3(S, r, x, y);
    const int d = S + 1 - y;
    const int p = Tb + r;
    const int pu = p + Ts - y;
    const int pd = r + y;
    const T v[15] = {ld(pd),         ld(pd + 1),     ld(pd + d + 1), ld(pd + d), ld(p - d - 1),
                     ld(p - d),      ld(p - 1),      ld(p),          ld(p + 1),  ld(p + d - 1),
                     ld(p + d),      ld(pu - d),     ld(pu - d + 1), ld(pu - 1), ld(pu)};
    const T bv = MODE != kApply ? B[ab + p] : T(0);
    point_row<T, 3, MODE, false>(M, W, wi, live, N, x, y, z, v, v[7], bv, omega, Y + ab + p, ss, mx, true, true, bid);
  }
}

// A group tile of a slice-run level: lane i finishes shared DoF t.x0 + i of
// the exchange list.  Each copy's partial row is formed as the walk forms it
// at a boundary point (the partial stencil of the copy's support mask in its
// own macro, neighbours outside that macro dropped, table order), the copies
// are summed in the list's fixed macro order and the row is finished as the
// exchange kernel finishes it, so the values are those of the run and
// exchange launches; the runs leave these DoFs alone (point_row with
// KEEP_SHARED = false).
template <typename T, int MODE>
__device__ __forceinline__ void group_rows3(const StencilArgs<T>& a, const Tile& t, double& ss, double& mx) {
  constexpr StencilTable ST = stencil_table(3);
  const int lane = threadIdx.x & (kWave - 1);
  if (lane >= t.y0) return;
  const int g = t.x0 + lane;
  const int c0 = a.xptr[g], c1 = a.xptr[g + 1];
  const int64_t i0 = a.xcidx[c0];
  T out;
  if (MODE == kNormB) {
    out = a.B[i0];
  } else {
    T acc = T(0);
    for (int c = c0; c < c1; ++c) {
      const Copy k = a.xcopies[c];
      const MacroDev& M = a.md[k.macro];
      const int N = M.N;
      const int64_t i = a.xcidx[c];
      int off[15];
      nbr_offsets3(N, k.y, k.z, off);
      const int mask = support_mask(3, N, k.x, k.y, k.z);
      T p = T(0);
#pragma unroll
      for (int o = 0; o < ST.n; ++o) {
        const int nx = k.x + ST.off[o][0], ny = k.y + ST.off[o][1], nz = k.z + ST.off[o][2];
        const bool in = nx >= 0 && ny >= 0 && nz >= 0 && nx + ny + nz <= N;
        const T v = a.X[in ? i + off[o] : i];
        p = fma(Prec<T>::w(M, mask, o), in ? v : T(0), p);
      }
      acc += p;
    }
    if (MODE == kApply || MODE == kApplyDot) out = acc;
    else if (MODE == kJacobi) out = fma(a.omega * Prec<T>::ginv(a.xinv, a.xinvf, g), a.B[i0] - acc, a.X[i0]);
    else out = a.B[i0] - acc;
    for (int c = c0; c < c1; ++c) a.Y[a.xcidx[c]] = out;
  }
  accum<T, MODE>(ss, mx, out, MODE == kApplyDot ? a.X[i0] : T(0));
}

// Whether a wave tile has output points on its macro's boundary (x = 0,
// y = 0, z = 0 or the far face x + y + z = N).
template <typename T, int DIM, int PZ>
__device__ __forceinline__ bool tile_on_boundary(const Tile& t, int N) {
  if (DIM == 2) return t.x0 == 0 || t.y0 == 0 || t.x0 + t.y0 + (kTileW - 1) + (Tile2<T>::H - 1) >= N;
  if (PZ == kPenSeg) return true;  // a run of 64 points or more reaches a row end
  return t.x0 == 0 || t.y0 == 0 || t.z == 0 || t.x0 + t.y0 + t.z + (kTileW - 1) + (kPenR - 1) + (PZ - 1) >= N;
}

template <typename T, int DIM, int MODE, int PZ>
__global__ __launch_bounds__(kWG) void stencil_kernel(const Launch<StencilArgs<T>> L) {
  constexpr bool kPart = has_partials(MODE);
  const int g = xcd_wg(L.nwg);
  if (g < 0) return;
  StencilArgs<T> a;
  const int n = resolve(L, g, a);
  // wave-uniform tile index: the tile and its macro constants load into scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ti = n * kWavesPerWG + wv;
  const Tile t = a.tiles[ti];
  __shared__ T wtab[kWavesPerWG][16][16];
  // The partial-stencil table is only read by tiles that reach the macro's
  // boundary.  The workgroup's four tiles usually share one macro: then one
  // table serves all waves (one load per thread), loaded only if one of the
  // four tiles needs it; otherwise each wave loads its own when it needs it.
  const int m0 = a.tiles[n * kWavesPerWG].macro, m3 = a.tiles[n * kWavesPerWG + kWavesPerWG - 1].macro;
  const bool same = m0 == m3;
  if (same) {
    bool need = false;
    if (m0 >= 0) {
      const int N0 = a.md[m0].N;
#pragma unroll
      for (int k = 0; k < kWavesPerWG; ++k) need = need || tile_on_boundary<T, DIM, PZ>(a.tiles[n * kWavesPerWG + k], N0);
    }
    if (need) {
      load_wtab<T>(a.md[m0], wtab[0], 0, kWG);
      __syncthreads();
    }
  } else if (t.macro >= 0 && tile_on_boundary<T, DIM, PZ>(t, a.md[t.macro].N)) {
    load_wtab<T>(a.md[t.macro], wtab[wv], wv * kWave, kWave);
    __builtin_amdgcn_wave_barrier();
  }
  double ss = 0.0, mx = 0.0;
  if (t.macro >= 0) {
    const MacroDev& M = a.md[t.macro];
    WTab<T> W = wtab[same ? 0 : wv];
    if (DIM == 2 && tile2d_inner<T>(t.x0, t.y0, M.N))
      tile2d_fast<T, MODE>(t.x0, t.y0, M, a.X, a.Y, a.B, a.omega, ss, mx);
    else if (DIM == 2)
      tile2d<T, MODE>(t.x0, t.y0, M, W, a.X, a.Y, a.B, a.omega, ss, mx);
    else if (PZ == kPenSeg)
      seg3d<T, MODE>(t, M, W, a.X, a.Y, a.B, a.omega, ss, mx);
    else
      pencil3d<T, MODE, PZ>(t.x0, t.y0, t.z, M, W, a.X, a.Y, a.B, a.omega, ss, mx);
  } else if (DIM == 3 && PZ == kPenSeg && t.macro == kGroupTile) {
    group_rows3<T, MODE>(a, t, ss, mx);
  }
  if (kPart && a.part != nullptr) {
    // one partial per workgroup: its four waves summed in a fixed order
    ss = wave_sum(ss);
    mx = wave_max(mx);
    __shared__ double s_ss[kWavesPerWG], s_mx[kWavesPerWG];
    if ((threadIdx.x & (kWave - 1)) == 0) {
      s_ss[wv] = ss;
      s_mx[wv] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double p = s_ss[0], q = s_mx[0];
#pragma unroll
      for (int k = 1; k < kWavesPerWG; ++k) {
        p += s_ss[k];
        q = fmax(q, s_mx[k]);
      }
      a.part[n] = p;
      a.part[a.np + n] = q;
    }
  }
}

// ------------------------------------------------------------------ exchange

// One DoF shared by several macros and not Dirichlet: its copies hold
// partial rows (written by stencil_kernel); sum them in fixed macro order,
// finish the row, and write it to every copy.
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(kIfaceWG) void exchange_kernel(const Launch<GroupArgs<T>> L) {
  GroupArgs<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int g = blk * kIfaceWG + threadIdx.x;
  double ss = 0.0, mx = 0.0;
  if (g < a.ngroups) {
    int64_t i0;
    const T out = exchange_row<T, DIM, MODE>(a, g, i0);
    accum<T, MODE>(ss, mx, out, MODE == kApplyDot ? a.X[i0] : T(0));
  }
  if (has_partials(MODE) && a.part != nullptr) {
    __shared__ double s_ss[kIfaceWG / kWave], s_mx[kIfaceWG / kWave];
    ss = wave_sum(ss);
    mx = wave_max(mx);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
      s_ss[w] = ss;
      s_mx[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double p = 0.0, q = 0.0;
      for (int i = 0; i < kIfaceWG / kWave; ++i) {
        p += s_ss[i];
        q = fmax(q, s_mx[i]);
      }
      a.part[blk] = p;
      a.part[a.np + blk] = q;
    }
  }
}

// Every macro-boundary DoF: kExchangeSum (y = sum of x over the copies,
// Dirichlet -> 0, in place allowed) or kDirichletSet (y = b at Dirichlet
// DoFs; b == NULL sets them to 0).
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(kIfaceWG) void iface_kernel(const Launch<GroupArgs<T>> L) {
  GroupArgs<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int g = blk * kIfaceWG + threadIdx.x;
  if (g >= a.ngroups) return;
  if (MODE == kDirichletSet) {
    const int c0 = a.gptr[g], c1 = a.gptr[g + 1];
    if (!(a.gflag[g] & 1)) return;
    const T v = a.B ? a.B[a.cidx[c0]] : T(0);
    for (int c = c0; c < c1; ++c) a.Y[a.cidx[c]] = v;
    return;
  }
  iface_sum_row<T, DIM>(a, g);
}

// result = (sum of part[0, np), max of part[np, 2 np)) in a fixed order; one
// block of kRedT threads per request, four loads in flight per thread.
constexpr int kRedT = 512;
__global__ __launch_bounds__(kRedT) void reduce_kernel(const Launch<ReduceArgs> L) {
  ReduceArgs r;
  resolve(L, (int)blockIdx.x, r);
  __shared__ double s[kRedT], m[kRedT];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, b = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 3 * kRedT < r.np; i += 4 * kRedT) {
    a0 += r.part[i];
    a1 += r.part[i + kRedT];
    a2 += r.part[i + 2 * kRedT];
    a3 += r.part[i + 3 * kRedT];
    b = fmax(fmax(b, fmax(r.part[r.np + i], r.part[r.np + i + kRedT])),
             fmax(r.part[r.np + i + 2 * kRedT], r.part[r.np + i + 3 * kRedT]));
  }
  for (; i < r.np; i += kRedT) {
    a0 += r.part[i];
    b = fmax(b, r.part[r.np + i]);
  }
  s[threadIdx.x] = (a0 + a1) + (a2 + a3);
  m[threadIdx.x] = b;
  __syncthreads();
  for (int w = kRedT / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s[threadIdx.x] += s[threadIdx.x + w];
      m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double second = r.shift ? r.result[0] : m[0];
    r.result[0] = s[0];
    r.result[1] = second;
    if (r.copy) {
      r.copy[0] = s[0];
      r.copy[1] = second;
    }
  }
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

inline int stencil_grid(int nwg) { return wave::xcd_grid(nwg); }

template <class A>
Launch<A> single(const A& a, int nwg) {
  Launch<A> l{};
  l.one = a;
  l.nseg = 0;
  l.nwg = nwg;
  return l;
}

template <class A>
Launch<A> batched(const BatchOp& op, const char* table) {
  Launch<A> l{};
  l.many = (const A*)(table + op.args_off);
  l.wg0 = (const int32_t*)(table + op.wg0_off);
  l.nseg = op.nseg;
  l.nwg = op.nwg;
  return l;
}

template <typename T, int DIM, int MODE>
void run_stencil(const Level& L, const void* x, void* y, const void* b, double omega, double* part,
                 hipStream_t s) {
  const StencilArgs<T> a = stencil_args<T>(L, x, y, b, omega, part);
  if (a.nwg > 0) {
    // the tile shape is a 3D notion: 2D uses one instance
    if (DIM == 3 && L.pen_z == kPenSeg) {
      if constexpr (DIM == 3)
        hipLaunchKernelGGL((stencil_kernel<T, DIM, MODE, kPenSeg>), dim3(stencil_grid(a.nwg)), dim3(kWG), 0, s,
                           single(a, a.nwg));
    } else {
      hipLaunchKernelGGL((stencil_kernel<T, DIM, MODE, kPenZ>), dim3(stencil_grid(a.nwg)), dim3(kWG), 0, s,
                         single(a, a.nwg));
    }
  }
  const int nblk = exchange_in_launch(L) ? 0 : exchange_blocks(L);
  if (nblk == 0) return;
  hipLaunchKernelGGL((exchange_kernel<T, DIM, MODE>), dim3(nblk), dim3(kIfaceWG), 0, s,
                     single(exchange_args<T>(L, x, y, b, omega, part), nblk));
}

template <typename T, int DIM, int MODE>
void run_iface(const Level& L, const void* x, void* y, const void* b, hipStream_t s) {
  const int nblk = iface_blocks(L);
  if (nblk == 0) return;
  hipLaunchKernelGGL((iface_kernel<T, DIM, MODE>), dim3(nblk), dim3(kIfaceWG), 0, s,
                     single(iface_args<T>(L, x, y, b), nblk));
}

template <typename T, int DIM>
void dispatch(int mode, const Level& L, const void* x, void* y, const void* b, double omega, double* part,
              hipStream_t s) {
  switch (mode) {
    case kApply: run_stencil<T, DIM, kApply>(L, x, y, b, omega, part, s); break;
    case kJacobi: run_stencil<T, DIM, kJacobi>(L, x, y, b, omega, part, s); break;
    case kResidual: run_stencil<T, DIM, kResidual>(L, x, y, b, omega, part, s); break;
    case kNormB: run_stencil<T, DIM, kNormB>(L, x, y, b, omega, part, s); break;
    case kApplyDot: run_stencil<T, DIM, kApplyDot>(L, x, y, b, omega, part, s); break;
    case kExchangeSum: run_iface<T, DIM, kExchangeSum>(L, x, y, b, s); break;
    default: run_iface<T, DIM, kDirichletSet>(L, x, y, b, s); break;
  }
}

int launch(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
           double omega, double* part, hipStream_t s) {
  if (dtype == MF_F64) {
    if (m->dim == 2) dispatch<double, 2>(mode, L, x, y, b, omega, part, s);
    else dispatch<double, 3>(mode, L, x, y, b, omega, part, s);
  } else {
    if (m->dim == 2) dispatch<float, 2>(mode, L, x, y, b, omega, part, s);
    else dispatch<float, 3>(mode, L, x, y, b, omega, part, s);
  }
  return check_launch();
}

// ---------------------------------------------------------------- batched
template <typename T, int DIM, int MODE>
void batch_stencil(const BatchOp& op, const char* table, hipStream_t s) {
  if (op.kind == kOpStencil && DIM == 3 && op.variant == kPenSeg) {
    if constexpr (DIM == 3)
      hipLaunchKernelGGL((stencil_kernel<T, DIM, MODE, kPenSeg>), dim3(stencil_grid(op.nwg)), dim3(kWG), 0, s,
                         batched<StencilArgs<T>>(op, table));
  } else if (op.kind == kOpStencil)
    hipLaunchKernelGGL((stencil_kernel<T, DIM, MODE, kPenZ>), dim3(stencil_grid(op.nwg)), dim3(kWG), 0, s,
                       batched<StencilArgs<T>>(op, table));
  else
    hipLaunchKernelGGL((exchange_kernel<T, DIM, MODE>), dim3(op.nwg), dim3(kIfaceWG), 0, s,
                       batched<GroupArgs<T>>(op, table));
}

template <typename T, int DIM>
void batch_dispatch(const BatchOp& op, const char* table, hipStream_t s) {
  if (op.kind == kOpIface) {
    if (op.mode == kExchangeSum)
      hipLaunchKernelGGL((iface_kernel<T, DIM, kExchangeSum>), dim3(op.nwg), dim3(kIfaceWG), 0, s,
                         batched<GroupArgs<T>>(op, table));
    else
      hipLaunchKernelGGL((iface_kernel<T, DIM, kDirichletSet>), dim3(op.nwg), dim3(kIfaceWG), 0, s,
                         batched<GroupArgs<T>>(op, table));
    return;
  }
  switch (op.mode) {
    case kApply: batch_stencil<T, DIM, kApply>(op, table, s); break;
    case kJacobi: batch_stencil<T, DIM, kJacobi>(op, table, s); break;
    case kResidual: batch_stencil<T, DIM, kResidual>(op, table, s); break;
    case kNormB: batch_stencil<T, DIM, kNormB>(op, table, s); break;
    default: batch_stencil<T, DIM, kApplyDot>(op, table, s); break;
  }
}

}  // namespace

int64_t stencil_partials(const Level& L, int dtype) { return L.n_partials(dtype); }

int launch_stencil(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                   double omega, double* part, hipStream_t s) {
  return launch(m, L, dtype, mode, x, y, b, omega, part, s);
}

int launch_iface(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                 hipStream_t s) {
  return launch(m, L, dtype, mode, x, y, b, 0.0, nullptr, s);
}

int launch_exchange_apply(const Level& L, int dtype, void* y, hipStream_t s) {
  const int nblk = exchange_blocks(L);
  if (nblk == 0) return MF_OK;
  if (dtype == MF_F64)
    hipLaunchKernelGGL((exchange_kernel<double, 2, kApply>), dim3(nblk), dim3(kIfaceWG), 0, s,
                       single(exchange_args<double>(L, nullptr, y, nullptr, 0.0, nullptr), nblk));
  else
    hipLaunchKernelGGL((exchange_kernel<float, 2, kApply>), dim3(nblk), dim3(kIfaceWG), 0, s,
                       single(exchange_args<float>(L, nullptr, y, nullptr, 0.0, nullptr), nblk));
  return check_launch();
}

int launch_reduce(const double* part, int64_t np, double* result, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedT), 0, s, single(ReduceArgs{part, np, result, nullptr, 0, 0}, 1));
  return check_launch();
}

int launch_reduce_shift(const double* part, int64_t np, double* result, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kRedT), 0, s, single(ReduceArgs{part, np, result, nullptr, 1, 0}, 1));
  return check_launch();
}

int launch_stencil_batch(const BatchOp& op, const char* table, hipStream_t s) {
  if (op.nwg <= 0) return MF_OK;
  if (op.kind == kOpReduce) {
    hipLaunchKernelGGL(reduce_kernel, dim3(op.nwg), dim3(kRedT), 0, s, batched<ReduceArgs>(op, table));
    return check_launch();
  }
  if (op.dtype == MF_F64) {
    if (op.dim == 2) batch_dispatch<double, 2>(op, table, s);
    else batch_dispatch<double, 3>(op, table, s);
  } else {
    if (op.dim == 2) batch_dispatch<float, 2>(op, table, s);
    else batch_dispatch<float, 3>(op, table, s);
  }
  return check_launch();
}

}  // namespace mf
