// Variable-coefficient 2D P1 apply (gfx950): y = A(k) x with A(k) the
// stiffness matrix of -div(k grad u), k the P1 interpolant of nodal values
// k_i (a vector in storage layout).  On a P1 element grad u . grad v is
// constant, so each element matrix is exactly mean_T(k) times the
// constant-coefficient one; the rows are formed on the fly from the macro's
// two element matrices and the coefficient, which the paper notes as the way
// to keep varying weights matrix-free at the price of extra arithmetic
// (comparison of matrix-free and sparse storage).  Traffic: k and x read,
// y written (24 B/DoF in FP64).
//
// Walk: as the constant-coefficient 2D walk, a wave owns 64 columns (62
// outputs) of a strip of rows and keeps three rows of x and k in registers.
// A point's row sums over its six micro-triangles: U(x,y), U(x-1,y),
// U(x,y-1) (up) and D(x-1,y), D(x-1,y-1), D(x,y-1) (down), where U(a,b) has
// vertices (a,b),(a+1,b),(a,b+1) and D(a,b) has (a+1,b),(a+1,b+1),(a,b+1).
// The triangle coefficients of one band of rows are computed once per lane
// and reused by the two rows that share the band.  Macro-boundary points sum
// only the triangles inside the macro (a partial row, completed for shared
// DoFs by the exchange kernel); Dirichlet points copy x.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "rows.hpp"
#include "wave.hpp"

namespace mf {

namespace {

using wave::dn1;
using wave::up1;

template <typename T>
struct VcTile {
  static constexpr int H = kTileH2, U = 4;
};
template <>
struct VcTile<float> {
  static constexpr int H = kTileH2F, U = 8;
};

// Column xc (>= 0) of row r of a triangle of side N stored at base, with the
// row clamped to [0, min(last, N)] and the column into the row.
template <typename T>
__device__ __forceinline__ T ld_row(const T* __restrict__ base, int N, int r, int last, int xc) {
  const int rr = min(max(r, 0), min(last, N));
  return base[row_start(N, rr) + min(xc, N - rr)];
}

// Coefficients of the up and down triangles with anchor (x, b), from k rows
// b and b+1 of this lane (kb, kb1) and of lane + 1.
template <typename T>
__device__ __forceinline__ void band_coef(T kb, T kb1, T third, T& ku, T& kd) {
  const T kbr = dn1(kb), kb1r = dn1(kb1);
  ku = (kb + kbr + kb1) * third;
  kd = (kbr + kb1r + kb1) * third;
}

template <typename T, bool INNER>
__device__ __forceinline__ void vc_tile(int x0, int y0, const MacroDev& M, const T* __restrict__ K,
                                        const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int kH = VcTile<T>::H, kU = VcTile<T>::U;
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int x = x0 - 1 + lane;
  const int xc = max(x, 0);
  const int y1 = min(y0 + kH, N - x0 + 1);  // output rows y0 .. y1-1
  K += M.base;
  X += M.base;
  Y += M.base;
  // element matrices: up (type 0) and down (type 1), local rows 0..2
  T ku[3][3], kd[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ku[i][j] = (T)M.K[0][i * 4 + j];
      kd[i][j] = (T)M.K[1][i * 4 + j];
    }
  const T third = T(1) / T(3);

  // x and k of rows y-1 (m), y (0), y+1 (p); triangle coefficients of bands
  // y-1 (between rows y-1 and y) and y
  T xm = ld_row(X, N, y0 - 1, y1, xc), x0v = ld_row(X, N, y0, y1, xc);
  T km = ld_row(K, N, y0 - 1, y1, xc), k0 = ld_row(K, N, y0, y1, xc);
  T kum, kdm;
  band_coef(km, k0, third, kum, kdm);
  T qx[kU], qk[kU];
#pragma unroll
  for (int j = 0; j < kU; ++j) {
    qx[j] = ld_row(X, N, y0 + 1 + j, y1, xc);
    qk[j] = ld_row(K, N, y0 + 1 + j, y1, xc);
  }
  const int nrows = y1 - y0;
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const int yy = y0 + j;
    const T xp = qx[j % kU], kp = qk[j % kU];
    qx[j % kU] = ld_row(X, N, y0 + 2 + j + kU - 1, y1, xc);
    qk[j % kU] = ld_row(K, N, y0 + 2 + j + kU - 1, y1, xc);
    if (j >= nrows) continue;
    T kup, kdp;  // band y
    band_coef(k0, kp, third, kup, kdp);
    const T xE = dn1(x0v), xW = up1(x0v), xNW = up1(xp), xSE = dn1(xm);
    const T t1 = ku[0][0] * x0v + ku[0][1] * xE + ku[0][2] * xp;
    const T t2 = ku[1][0] * xW + ku[1][1] * x0v + ku[1][2] * xNW;
    const T t3 = ku[2][0] * xm + ku[2][1] * xSE + ku[2][2] * x0v;
    const T t4 = kd[0][0] * x0v + kd[0][1] * xp + kd[0][2] * xNW;
    const T t5 = kd[1][0] * xm + kd[1][1] * x0v + kd[1][2] * xW;
    const T t6 = kd[2][0] * xSE + kd[2][1] * xE + kd[2][2] * x0v;
    const T c1 = kup, c2 = up1(kup), c3 = kum, c4 = up1(kdp), c5 = up1(kdm), c6 = kdm;
    T acc;
    const bool inside = lane >= 1 && lane <= kTileW && x + yy <= N;
    if (INNER) {
      acc = c1 * t1;
      acc = fma(c2, t2, acc);
      acc = fma(c3, t3, acc);
      acc = fma(c4, t4, acc);
      acc = fma(c5, t5, acc);
      acc = fma(c6, t6, acc);
      if (inside) Y[row_start(N, yy) + xc] = acc;
    } else {
      // triangles inside the macro (the point itself is inside)
      const bool in1 = x + yy <= N - 1, in2 = x >= 1, in3 = yy >= 1;
      const bool in4 = x >= 1 && x + yy <= N - 1, in5 = x >= 1 && yy >= 1, in6 = yy >= 1 && x + yy <= N - 1;
      acc = in1 ? c1 * t1 : T(0);
      acc = in2 ? fma(c2, t2, acc) : acc;
      acc = in3 ? fma(c3, t3, acc) : acc;
      acc = in4 ? fma(c4, t4, acc) : acc;
      acc = in5 ? fma(c5, t5, acc) : acc;
      acc = in6 ? fma(c6, t6, acc) : acc;
      if (inside) {
        const bool dir = (M.dir_mask >> support_mask(2, N, x, yy, 0)) & 1;
        Y[row_start(N, yy) + xc] = dir ? x0v : acc;
      }
    }
    xm = x0v;
    x0v = xp;
    k0 = kp;
    kum = kup;
    kdm = kdp;
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void varcoef_kernel(const Tile* __restrict__ tiles, int nwg, const MacroDev* md,
                                                      const T* __restrict__ K, const T* __restrict__ X,
                                                      T* __restrict__ Y) {
  const int g = wave::xcd_wg(nwg);
  if (g < 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Tile t = tiles[g * kWavesPerWG + wv];
  if (t.macro < 0) return;
  const MacroDev& M = md[t.macro];
  if (t.x0 >= 1 && t.y0 >= 1 && t.x0 + t.y0 + kTileW + VcTile<T>::H <= M.N)
    vc_tile<T, true>(t.x0, t.y0, M, K, X, Y);
  else
    vc_tile<T, false>(t.x0, t.y0, M, K, X, Y);
}

template <typename T>
int run_varcoef(const Level& L, const void* k, const void* x, void* y, hipStream_t s) {
  const bool f32 = sizeof(T) == 4 && !L.tiles_f32.empty();
  const Tile* tiles = f32 ? L.dev.tiles_f32 : L.dev.tiles;
  const int nwg = (int)((f32 ? L.tiles_f32.size() : L.tiles.size()) / kWavesPerWG);
  if (nwg > 0)
    hipLaunchKernelGGL(varcoef_kernel<T>, dim3(wave::xcd_grid(nwg)), dim3(kWG), 0, s, tiles, nwg, L.dev.md,
                       (const T*)k, (const T*)x, (T*)y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return launch_exchange_apply(L, dtype_of<T>(), y, s);
}


// ---------------------------------------------------------------- 3D
// Tetrahedral macros: a point's row sums over the micro-tets of its macro
// that contain it (24 for an interior point: each of the 6 element types
// with the point at each of its 4 vertices), each tet contributing
// mean_T(k) times its row of the constant-coefficient element matrix.  Every
// vertex of such a tet is the point itself or one of its 15 stencil
// neighbours, so one lane loads k and x at those 15 points (gathers within a
// few rows of 3 slices, served by L1/L2) and forms all contributions in
// registers.  One wave takes a 64-point slice segment (consecutive storage
// points of one slice, across row ends), so short rows leave no lane idle.

// Index into the 15 stencil offsets of lattice offset d (-1 if none).
__host__ __device__ constexpr int stencil_slot(int dx, int dy, int dz) {
  constexpr StencilTable ST = stencil_table(3);
  for (int o = 0; o < ST.n; ++o)
    if (ST.off[o][0] == dx && ST.off[o][1] == dy && ST.off[o][2] == dz) return o;
  return -1;
}

// Stencil slot of vertex u of a type-t tet whose vertex v is the point.
__host__ __device__ constexpr int tet_slot(int t, int v, int u) {
  constexpr ElemTable E = elem_table(3);
  return stencil_slot(E.off[t][u][0] - E.off[t][v][0], E.off[t][u][1] - E.off[t][v][1],
                      E.off[t][u][2] - E.off[t][v][2]);
}

__host__ __device__ constexpr bool tet_slots_valid() {
  for (int t = 0; t < 6; ++t)
    for (int v = 0; v < 4; ++v)
      for (int u = 0; u < 4; ++u)
        if (tet_slot(t, v, u) < 0) return false;
  return true;
}
static_assert(tet_slots_valid(), "every edge of a micro-tet is a stencil offset");

template <typename T>
__device__ __forceinline__ void vc3_point(const MacroDev& M, const T* __restrict__ K, const T* __restrict__ X,
                                          T* __restrict__ Y, int x, int y, int z) {
  constexpr StencilTable ST = stencil_table(3);
  constexpr ElemTable E = elem_table(3);
  const int N = M.N;
  const int S = N - z;
  // neighbours by offsets from the point's index, all taken relative to the
  // first point of slice z - 1 (slice 0 at z = 0) as 32-bit offsets
  const int za = z > 0 ? z - 1 : 0;
  const int64_t ab = M.base + slice_base(N, za);
  const int c = (z > 0 ? (S + 2) * (S + 3) / 2 : 0) + row_start(S, y) + x;
  int off[15];
  nbr_offsets3(N, y, z, off);
  const T* __restrict__ Ka = K + ab;
  const T* __restrict__ Xa = X + ab;
  T kv[ST.n], xv[ST.n];
#pragma unroll
  for (int o = 0; o < ST.n; ++o) {
    const int nx = x + ST.off[o][0], ny = y + ST.off[o][1], nz = z + ST.off[o][2];
    const bool in = nx >= 0 && ny >= 0 && nz >= 0 && nx + ny + nz <= N;
    // neighbours outside the macro read the point itself; no tet uses them
    const unsigned byte = (unsigned)(in ? c + off[o] : c) * (unsigned)sizeof(T);
    kv[o] = *(const T*)((const char*)Ka + byte);
    xv[o] = *(const T*)((const char*)Xa + byte);
  }
  const int mask = support_mask(3, N, x, y, z);
  if (mask != full_mask(3) && ((M.dir_mask >> mask) & 1)) {
    Y[ab + c] = xv[ST.centre];  // identity row
    return;
  }
  // the sums of the four vertex coefficients are used unscaled and the row
  // scaled by 1/4 once at the end: scaling by powers of two is exact, so this
  // equals summing mean_T(k) times the element rows.  The element matrices
  // are read in the kernel's precision (FP32 kernels: the macro's FP32 copy).
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < E.ntypes; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ax = x - E.off[t][v][0], ay = y - E.off[t][v][1], az = z - E.off[t][v][2];
      const bool exists = ax >= 0 && ay >= 0 && az >= 0 && ax + ay + az <= N - E.slack[t];
      const int s0 = tet_slot(t, v, 0), s1 = tet_slot(t, v, 1), s2 = tet_slot(t, v, 2), s3 = tet_slot(t, v, 3);
      const T ks = kv[s0] + kv[s1] + kv[s2] + kv[s3];
      const T* Kt = Prec<T>::K(M, t) + 4 * v;
      T r = Kt[0] * xv[s0];
      r = fma(Kt[1], xv[s1], r);
      r = fma(Kt[2], xv[s2], r);
      r = fma(Kt[3], xv[s3], r);
      acc = exists ? fma(ks, r, acc) : acc;
    }
  }
  // interior, unshared and shared points alike store their (partial) row;
  // the exchange kernel completes shared DoFs
  Y[ab + c] = acc * T(0.25);
}

template <typename T>
__global__ __launch_bounds__(kWG) void varcoef3d_kernel(const Tile* __restrict__ segs, int nwg, const MacroDev* md,
                                                        const T* __restrict__ K, const T* __restrict__ X,
                                                        T* __restrict__ Y) {
  const int g = wave::xcd_wg(nwg);
  if (g < 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Tile sg = load_seg(segs, g * kWavesPerWG + wv);
  if (sg.macro < 0) return;
  const MacroDev& M = md[sg.macro];
  int x, y, z;
  slice_point<3>(sg, M.N, x, y, z);
  if (x + y + z > M.N) return;  // lanes past the slice's last point
  vc3_point<T>(M, K, X, Y, x, y, z);
}

template <typename T>
int run_varcoef3d(const Level& L, const void* k, const void* x, void* y, hipStream_t s) {
  const int nwg = (int)(L.psegs.size() / kWavesPerWG);
  if (nwg > 0)
    hipLaunchKernelGGL(varcoef3d_kernel<T>, dim3(wave::xcd_grid(nwg)), dim3(kWG), 0, s, L.dev.psegs, nwg, L.dev.md,
                       (const T*)k, (const T*)x, (T*)y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return launch_exchange_apply(L, dtype_of<T>(), y, s);
}

}  // namespace

int launch_varcoef_apply(const mf_mesh* m, const Level& L, int dtype, const void* k, const void* x, void* y,
                         hipStream_t s) {
  if (m->dim == 3)
    return dtype == MF_F64 ? run_varcoef3d<double>(L, k, x, y, s) : run_varcoef3d<float>(L, k, x, y, s);
  return dtype == MF_F64 ? run_varcoef<double>(L, k, x, y, s) : run_varcoef<float>(L, k, x, y, s);
}

}  // namespace mf
