// Fused P2 operator for 2D macro meshes (gfx950): y = A x over the vertex
// and edge-midpoint DoFs in one pass (the paper's four P2 kernels,
// Performance Modeling section, fused as its Conclusion proposes).
//
// Interior DoFs: a 64-lane wavefront walks fine rows upward.  Lane i holds
// the fine columns xa = x0 - 2 + 2i (even) and xa + 1 of each row, so in an
// even row it computes a vertex row (19 neighbours) and a horizontal-edge row
// (9), in an odd row a vertical- and a diagonal-edge row (9 each).  Every
// neighbour is at most two columns and two rows away, i.e. in the lane itself
// or in lanes i +- 1 (DPP shifts), and in the five rows kept in registers, so
// each source value is read from memory once per tile.  Opposite neighbours
// share a weight (p2.hpp) and are added before the multiply.
//
// Macro-boundary DoFs (about 3 * 2^(l+1) per macro): one thread each sums the
// element-matrix rows of the micro-triangles of its macro that contain it (a
// partial row), or copies x at a Dirichlet DoF; the exchange kernel then
// completes shared DoFs exactly as for P1.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "p2.hpp"
#include "wave.hpp"

namespace mf {

namespace {

using wave::dn1;
using wave::up1;

template <typename T>
struct P2Tab;
template <>
struct P2Tab<double> {
  static __device__ __forceinline__ const double* w(const P2Macro& P) { return P.w; }
  static __device__ __forceinline__ const double* K(const P2Macro& P) { return P.K; }
};
template <>
struct P2Tab<float> {
  static __device__ __forceinline__ const float* w(const P2Macro& P) { return P.wf; }
  static __device__ __forceinline__ const float* K(const P2Macro& P) { return P.Kf; }
};

// One fine row as a lane sees it: its even column a, the odd column b after
// it, and the shifted copies the stencils use (ua: a of lane - 1, i.e. column
// xa - 2; da: a of lane + 1, column xa + 2; ub: b of lane - 1, column xa - 1).
template <typename T>
struct Row {
  T a, b, ua, da, ub;
};
template <typename T>
__device__ __forceinline__ Row<T> row_of(T a, T b) {
  return Row<T>{a, b, up1(a), dn1(a), up1(b)};
}

// Two adjacent entries, loaded or stored as one 16-byte (FP64) access; rows
// start at any entry, so only the element alignment is assumed (gfx950
// global memory accesses need dword alignment only).
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  typedef double V __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct Pair<float> {
  typedef float V __attribute__((ext_vector_type(2), aligned(4)));
};

// Columns xa and xa + 1 of row r of the fine triangle (side M), with the row
// clamped to [0, last] and the columns into the row: a valid point for every
// lane (clamped values only feed halo lanes and points that are not stored).
template <typename T>
__device__ __forceinline__ void ld_pair(const T* __restrict__ X, int M, int r, int last, int xa, T& a, T& b) {
  const int rr = min(max(r, 0), last);
  const int S = M - rr;
  const T* row = X + row_start(M, rr);
  if (sizeof(T) == 4) {
    // FP32: two 4-byte loads measured faster than one 8-byte pair load
    a = row[min(max(xa, 0), S)];
    b = row[min(max(xa + 1, 0), S)];
  } else if (S >= 1) {
    // one 2-element load at a start kept inside the row; a lane past the row
    // end takes the last element, a lane before its start the first
    const int st = min(max(xa, 0), S - 1);
    const typename Pair<T>::V v = *(const typename Pair<T>::V*)(row + st);
    a = xa >= S ? v.y : v.x;
    b = xa < 0 ? v.x : v.y;
  } else {
    a = row[0];
    b = a;
  }
}

constexpr int kP2U = 4;  // rows loaded ahead
static_assert(kP2H % 2 == 0 && kP2H >= kP2U, "tile height");

template <typename T>
__device__ __forceinline__ void p2_tile(int x0, int y0, const MacroDev& Md, const P2Macro& P, const T* __restrict__ X,
                                        T* __restrict__ Y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int M = Md.N;  // fine side
  const int xa = x0 - 2 + 2 * lane;
  const bool lane_out = lane >= 1 && lane <= kTileW;
  const int nrows = min(kP2H, M - y0);  // rows that can hold interior points (Y <= M - 1)
  const int last = min(y0 + nrows + 1, M);
  X += Md.base;
  Y += Md.base;
  const T* w = P2Tab<T>::w(P);
  T wt[kP2Weights];
#pragma unroll
  for (int k = 0; k < kP2Weights; ++k) wt[k] = w[k];

  Row<T> r0, r1, r2, r3;  // rows Y-2 .. Y+1 of the current output row Y
  {
    T a, b;
    ld_pair(X, M, y0 - 2, last, xa, a, b);
    r0 = row_of(a, b);
    ld_pair(X, M, y0 - 1, last, xa, a, b);
    r1 = row_of(a, b);
    ld_pair(X, M, y0, last, xa, a, b);
    r2 = row_of(a, b);
    ld_pair(X, M, y0 + 1, last, xa, a, b);
    r3 = row_of(a, b);
  }
  T qa[kP2U], qb[kP2U];  // raw rows y0+2 .. loaded ahead
#pragma unroll
  for (int k = 0; k < kP2U; ++k) ld_pair(X, M, y0 + 2 + k, last, xa, qa[k], qb[k]);

#pragma unroll
  for (int k = 0; k < kP2H; ++k) {
    const Row<T> r4 = row_of(qa[k % kP2U], qb[k % kP2U]);  // row Y+2
    if (k + kP2U + 1 <= kP2H) ld_pair(X, M, y0 + 2 + k + kP2U, last, xa, qa[k % kP2U], qb[k % kP2U]);
    if (k < nrows) {
      const int yy = y0 + k;
      T oa, ob;
      if ((k & 1) == 0) {
        // vertex at xa, horizontal edge at xa + 1
        oa = wt[0] * r2.a;
        oa = fma(wt[1], r2.da + r2.ua, oa);
        oa = fma(wt[2], r4.a + r0.a, oa);
        oa = fma(wt[3], r0.da + r4.ua, oa);
        oa = fma(wt[4], r2.b + r2.ub, oa);
        oa = fma(wt[5], r3.a + r1.a, oa);
        oa = fma(wt[6], r1.b + r3.ub, oa);
        oa = fma(wt[7], r3.b + r1.ub, oa);
        oa = fma(wt[8], r1.da + r3.ua, oa);
        oa = fma(wt[9], r0.b + r4.ub, oa);
        ob = wt[10] * r2.b;
        ob = fma(wt[11], r2.da + r2.a, ob);
        ob = fma(wt[12], r3.b + r1.b, ob);
        ob = fma(wt[13], r3.a + r1.da, ob);
        ob = fma(wt[14], r4.a + r0.da, ob);
      } else {
        // vertical edge at xa, diagonal edge at xa + 1
        oa = wt[15] * r2.a;
        oa = fma(wt[16], r3.a + r1.a, oa);
        oa = fma(wt[17], r1.da + r3.ua, oa);
        oa = fma(wt[18], r1.b + r3.ub, oa);
        oa = fma(wt[19], r2.b + r2.ub, oa);
        ob = wt[20] * r2.b;
        ob = fma(wt[21], r3.da + r1.a, ob);
        ob = fma(wt[22], r1.da + r3.a, ob);
        ob = fma(wt[23], r3.b + r1.b, ob);
        ob = fma(wt[24], r2.da + r2.a, ob);
      }
      // interior points only: X >= 1, Y >= 1, X + Y <= M - 1
      T* yrow = Y + row_start(M, yy);
      const bool va = lane_out && yy >= 1 && xa >= 1 && xa + yy <= M - 1;
      const bool vb = lane_out && yy >= 1 && xa + 1 + yy <= M - 1;
      if (va && vb) {
        typename Pair<T>::V v;
        v.x = oa;
        v.y = ob;
        *(typename Pair<T>::V*)(yrow + xa) = v;
      } else {
        if (va) yrow[xa] = oa;
        if (vb) yrow[xa + 1] = ob;
      }
    }
    r0 = r1;
    r1 = r2;
    r2 = r3;
    r3 = r4;
  }
}

template <typename T>
__global__ __launch_bounds__(kWG) void p2_kernel(const Tile* __restrict__ tiles, int nwg, const MacroDev* md,
                                                 const P2Macro* p2, const T* __restrict__ X, T* __restrict__ Y) {
  const int g = wave::xcd_wg(nwg);
  if (g < 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Tile t = tiles[g * kWavesPerWG + wv];
  if (t.macro < 0) return;
  p2_tile<T>(t.x0, t.y0, md[t.macro], p2[t.macro], X, Y);
}

// Macro-boundary DoF k of macro c: k in [0, M] on y = 0, (M, 2M] on x = 0
// (y = k - M), (2M, 3M) on the far edge x + y = M (y = k - 2M).
template <typename T>
__global__ __launch_bounds__(256) void p2_boundary_kernel(const MacroDev* md, const P2Macro* p2, int nmacro, int M,
                                                          const T* __restrict__ X, T* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int per = 3 * M;
  if (t >= (int64_t)nmacro * per) return;
  const int c = (int)(t / per), k = (int)(t % per);
  int x, y;
  if (k <= M) {
    x = k;
    y = 0;
  } else if (k <= 2 * M) {
    x = 0;
    y = k - M;
  } else {
    y = k - 2 * M;
    x = M - y;
  }
  const MacroDev& Md = md[c];
  const int64_t i = Md.base + idx2(M, x, y);
  if ((Md.dir_mask >> support_mask(2, M, x, y, 0)) & 1) {
    Y[i] = X[i];  // identity row
    return;
  }
  // partial row: the micro-triangles of this macro containing the point
  const T* K = P2Tab<T>::K(p2[c]);
  const int nc = M / 2;
  T acc = T(0);
  for (int up = 1; up >= 0; --up)
    for (int db = -1; db <= 0; ++db)
      for (int da = -1; da <= 0; ++da) {
        const int a = (x >> 1) + da, b = (y >> 1) + db;
        if (a < 0 || b < 0 || a + b > nc - 1 - (up ? 0 : 1)) continue;
        int px[6], py[6];
        if (up) {
          px[0] = 2 * a;     py[0] = 2 * b;
          px[1] = 2 * a + 2; py[1] = 2 * b;
          px[2] = 2 * a;     py[2] = 2 * b + 2;
        } else {
          px[0] = 2 * a + 2; py[0] = 2 * b + 2;
          px[1] = 2 * a;     py[1] = 2 * b + 2;
          px[2] = 2 * a + 2; py[2] = 2 * b;
        }
        px[3] = (px[0] + px[1]) >> 1; py[3] = (py[0] + py[1]) >> 1;
        px[4] = (px[1] + px[2]) >> 1; py[4] = (py[1] + py[2]) >> 1;
        px[5] = (px[0] + px[2]) >> 1; py[5] = (py[0] + py[2]) >> 1;
        int lp = -1;
        for (int q = 0; q < 6; ++q)
          if (px[q] == x && py[q] == y) lp = q;
        if (lp < 0) continue;
        for (int q = 0; q < 6; ++q) acc = fma(K[lp * 6 + q], X[Md.base + idx2(M, px[q], py[q])], acc);
      }
  Y[i] = acc;
}

template <typename T>
int run_p2(const mf_mesh* m, const Level& F, const void* x, void* y, hipStream_t s) {
  const int nwg = (int)(F.p2_tiles.size() / kWavesPerWG);
  if (nwg > 0)
    hipLaunchKernelGGL(p2_kernel<T>, dim3(wave::xcd_grid(nwg)), dim3(kWG), 0, s, F.dev.p2_tiles, nwg, F.dev.md,
                       m->p2_dev, (const T*)x, (T*)y);
  const int64_t nb = (int64_t)m->nc * 3 * F.N;
  hipLaunchKernelGGL(p2_boundary_kernel<T>, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, F.dev.md, m->p2_dev,
                     (int)m->nc, F.N, (const T*)x, (T*)y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return launch_exchange_apply(F, dtype_of<T>(), y, s);
}

}  // namespace

int launch_p2_apply(const mf_mesh* m, int level, int dtype, const void* x, void* y, hipStream_t s) {
  const Level& F = m->levels[level + 1];
  return dtype == MF_F64 ? run_p2<double>(m, F, x, y, s) : run_p2<float>(m, F, x, y, s);
}

}  // namespace mf
