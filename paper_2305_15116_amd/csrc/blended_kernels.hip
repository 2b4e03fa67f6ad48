// Blended (non-affine) 2D macros (gfx950): y = A x for the P1 operator of a
// micro mesh whose lattice points macro c maps by
//   F_c(xi) = P0 + (P1 - P0) xi1 + (P2 - P0) xi2 + xi0 xi1 xi2 d_c,
// xi = lattice point / N, xi0 = 1 - xi1 - xi2 (a cubic bubble that vanishes
// on the macro's edges, so neighbouring macros agree on shared points).  No
// two rows share a stencil, so every element matrix is formed on the fly from
// the mapped coordinates: the paper's remark that varying weights can be
// computed on the fly at an arithmetic cost, here taken to the point where
// the arithmetic (about 120 FP64 operations per DoF) rivals the 16 B/DoF of
// memory traffic.
//
// Walk: the constant-coefficient 2D tiles.  Per lane and band of two rows,
// the element matrices of the band's up triangle U(x,b) = {(x,b), (x+1,b),
// (x,b+1)} and down triangle D(x,b) = {(x+1,b), (x+1,b+1), (x,b+1)} are
// formed once (K = (1 / 2|det E|) adj(E^T E) on the two edge vectors, the
// vertex-0 row and column from zero row sums) and serve the two rows that
// border the band; the neighbouring lane's triangles come by DPP shifts.
// Boundary handling as in the variable-coefficient walk.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "wave.hpp"

namespace mf {

namespace {

using wave::dn1;
using wave::up1;

constexpr int kBlH = kTileH2, kBlU = 4;  // rows per tile, rows loaded ahead

// Symmetric P1 element matrix of the triangle (X0, X1, X2).
struct TriK {
  double k00, k01, k02, k11, k12, k22;
};
__device__ __forceinline__ TriK tri_k(double x0, double y0, double x1, double y1, double x2, double y2) {
  const double e1x = x1 - x0, e1y = y1 - y0, e2x = x2 - x0, e2y = y2 - y0;
  const double m11 = e1x * e1x + e1y * e1y, m12 = e1x * e2x + e1y * e2y, m22 = e2x * e2x + e2y * e2y;
  // 1 / (2 |det E|): the hardware reciprocal estimate refined by two Newton
  // steps s <- s + s (1 - t s) (each squares the relative error), which is
  // cheaper than the IEEE division sequence and within an ulp of it
  const double t = 2.0 * fabs(e1x * e2y - e1y * e2x);
  double s = __builtin_amdgcn_rcp(t);
  s = fma(s, fma(-t, s, 1.0), s);
  s = fma(s, fma(-t, s, 1.0), s);
  TriK k;
  k.k11 = m22 * s;
  k.k22 = m11 * s;
  k.k12 = -m12 * s;
  k.k01 = -(k.k11 + k.k12);
  k.k02 = -(k.k12 + k.k22);
  k.k00 = -(k.k01 + k.k02);
  return k;
}

// A band's two element matrices and the entries of the neighbouring lane's
// (lane - 1) ones that the rows use.
struct Band {
  TriK u, d;
  double u01l, u11l, u12l;              // U(x-1, b): row of its vertex 1
  double d00l, d01l, d02l, d11l, d12l;  // D(x-1, b): rows of its vertices 0 and 1
};

__device__ __forceinline__ Band make_band(double cx, double cy, double cx1, double cy1) {
  // (cx, cy): this lane's point in row b; (cx1, cy1): in row b + 1
  const double rx = dn1(cx), ry = dn1(cy), rx1 = dn1(cx1), ry1 = dn1(cy1);
  Band B;
  B.u = tri_k(cx, cy, rx, ry, cx1, cy1);
  B.d = tri_k(rx, ry, rx1, ry1, cx1, cy1);
  B.u01l = up1(B.u.k01);
  B.u11l = up1(B.u.k11);
  B.u12l = up1(B.u.k12);
  B.d00l = up1(B.d.k00);
  B.d01l = up1(B.d.k01);
  B.d02l = up1(B.d.k02);
  B.d11l = up1(B.d.k11);
  B.d12l = up1(B.d.k12);
  return B;
}

__device__ __forceinline__ double ld_row(const double* __restrict__ base, int N, int r, int last, int xc) {
  const int rr = min(max(r, 0), min(last, N));
  return base[row_start(N, rr) + min(xc, N - rr)];
}

template <bool INNER>
__device__ __forceinline__ void bl_tile(int x0, int y0, const MacroDev& M, const Geo2& G, double bx, double by,
                                        const double* __restrict__ X, double* __restrict__ Y) {
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int x = x0 - 1 + lane;
  const int xc = max(x, 0);
  const int y1 = min(y0 + kBlH, N - x0 + 1);  // output rows y0 .. y1-1
  X += M.base;
  Y += M.base;
  const double invN = 1.0 / (double)N;  // exact: N is a power of two
  const double a = (double)x * invN;
  auto map = [&](int r, double& fx, double& fy) {
    const double b = (double)r * invN;
    const double bub = (1.0 - a - b) * a * b;
    fx = G.p0[0] + G.e1[0] * a + G.e2[0] * b + bub * bx;
    fy = G.p0[1] + G.e1[1] * a + G.e2[1] * b + bub * by;
  };
  double cx, cy, cx1, cy1;
  map(y0 - 1, cx, cy);
  map(y0, cx1, cy1);
  Band bm = make_band(cx, cy, cx1, cy1);  // band y0-1
  cx = cx1;
  cy = cy1;
  double xm = ld_row(X, N, y0 - 1, y1, xc), x0v = ld_row(X, N, y0, y1, xc);
  double q[kBlU];
#pragma unroll
  for (int j = 0; j < kBlU; ++j) q[j] = ld_row(X, N, y0 + 1 + j, y1, xc);
  const int nrows = y1 - y0;
#pragma unroll
  for (int j = 0; j < kBlH; ++j) {
    const int yy = y0 + j;
    const double xp = q[j % kBlU];
    q[j % kBlU] = ld_row(X, N, y0 + 1 + j + kBlU, y1, xc);
    if (j >= nrows) continue;
    map(yy + 1, cx1, cy1);
    const Band bp = make_band(cx, cy, cx1, cy1);  // band y
    const double xE = dn1(x0v), xW = up1(x0v), xNW = up1(xp), xSE = dn1(xm);
    // the six triangles around (x, y), each with this point's row of its matrix
    const double t1 = bp.u.k00 * x0v + bp.u.k01 * xE + bp.u.k02 * xp;      // U(x, y), vertex 0
    const double t2 = bp.u01l * xW + bp.u11l * x0v + bp.u12l * xNW;         // U(x-1, y), vertex 1
    const double t3 = bm.u.k02 * xm + bm.u.k12 * xSE + bm.u.k22 * x0v;      // U(x, y-1), vertex 2
    const double t4 = bp.d00l * x0v + bp.d01l * xp + bp.d02l * xNW;         // D(x-1, y), vertex 0
    const double t5 = bm.d01l * xm + bm.d11l * x0v + bm.d12l * xW;          // D(x-1, y-1), vertex 1
    const double t6 = bm.d.k02 * xSE + bm.d.k12 * xE + bm.d.k22 * x0v;      // D(x, y-1), vertex 2
    const bool inside = lane >= 1 && lane <= kTileW && x + yy <= N;
    double acc;
    if (INNER) {
      acc = ((t1 + t2) + (t3 + t4)) + (t5 + t6);
      if (inside) Y[row_start(N, yy) + xc] = acc;
    } else {
      const bool in1 = x + yy <= N - 1, in2 = x >= 1, in3 = yy >= 1;
      const bool in4 = x >= 1 && x + yy <= N - 1, in5 = x >= 1 && yy >= 1, in6 = yy >= 1 && x + yy <= N - 1;
      const double s12 = (in1 ? t1 : 0.0) + (in2 ? t2 : 0.0);
      const double s34 = (in3 ? t3 : 0.0) + (in4 ? t4 : 0.0);
      const double s56 = (in5 ? t5 : 0.0) + (in6 ? t6 : 0.0);
      acc = (s12 + s34) + s56;
      if (inside) {
        const bool dir = (M.dir_mask >> support_mask(2, N, x, yy, 0)) & 1;
        Y[row_start(N, yy) + xc] = dir ? x0v : acc;
      }
    }
    xm = x0v;
    x0v = xp;
    cx = cx1;
    cy = cy1;
    bm = bp;
  }
}

__global__ __launch_bounds__(kWG) void blended_kernel(const Tile* __restrict__ tiles, int nwg, const MacroDev* md,
                                                      const Geo2* geo, const double* __restrict__ bubble,
                                                      const double* __restrict__ X, double* __restrict__ Y) {
  const int g = wave::xcd_wg(nwg);
  if (g < 0) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const Tile t = tiles[g * kWavesPerWG + wv];
  if (t.macro < 0) return;
  const MacroDev& M = md[t.macro];
  const Geo2& G = geo[t.macro];
  const double bx = bubble[2 * t.macro], by = bubble[2 * t.macro + 1];
  if (t.x0 >= 1 && t.y0 >= 1 && t.x0 + t.y0 + kTileW + kBlH <= M.N)
    bl_tile<true>(t.x0, t.y0, M, G, bx, by, X, Y);
  else
    bl_tile<false>(t.x0, t.y0, M, G, bx, by, X, Y);
}

}  // namespace

int launch_blended_apply(const mf_mesh* m, const Level& L, const double* bubble, const double* x, double* y,
                         hipStream_t s) {
  const int nwg = (int)(L.tiles.size() / kWavesPerWG);
  if (nwg > 0)
    hipLaunchKernelGGL(blended_kernel, dim3(wave::xcd_grid(nwg)), dim3(kWG), 0, s, L.dev.tiles, nwg, L.dev.md,
                       m->geo2_dev, bubble, x, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return launch_exchange_apply(L, MF_F64, y, s);
}

}  // namespace mf
