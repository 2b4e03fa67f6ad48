// Blended (non-affine) 2D macros (gfx950): y = A x for the P1 operator of a
// micro mesh whose lattice points macro c maps by
//   F_c(xi) = P0 + (P1 - P0) xi1 + (P2 - P0) xi2 + xi0 xi1 xi2 d_c,
// xi = lattice point / N, xi0 = 1 - xi1 - xi2 (a cubic bubble that vanishes
// on the macro's edges, so neighbouring macros agree on shared points).  No
// two rows share a stencil, so every element matrix is formed on the fly from
// the edge vectors between mapped lattice points: the paper's remark that varying weights can be
// computed on the fly at an arithmetic cost, here taken to the point where
// the arithmetic (about 85 vector instructions per DoF, most of them FP64)
// outweighs the 16 B/DoF of memory traffic.
//
// Walk: the constant-coefficient 2D tiles, in edge form.  A P1 element
// matrix has zero row sums, so a row is y_i = sum_j w_ij (x_i - x_j) over
// the six lattice edges at i, where w_ij sums -K_ij over the (up to two)
// micro-triangles that share the edge, and -K_ij = cot(theta_k) / 2 with
// theta_k the angle opposite the edge: (e_ki . e_kj) / (2 |det|).  Per lane
// and band of two rows, the up triangle U = {C, R, C1} and the down triangle
// D = {R, R1, C1} (C = (x,b), R = (x+1,b), C1 = (x,b+1), R1 = (x+1,b+1))
// give their three cotangent weights from five edge vectors; the band then
// holds the lane's vertical edge weight (x,b)-(x,b+1) (U's plus the left
// lane's D's) and diagonal edge weight (x+1,b)-(x,b+1) (U's plus D's), and
// the horizontal edge (x,b+1)-(x+1,b+1) collects D's weight now and the next
// band's U's.  A row then needs two weights from the left lane (DPP) and the
// two carried from the band below.  Triangles outside the macro get zero
// weights on tiles that touch the macro boundary; Dirichlet points copy x and
// the exchange kernel completes shared DoFs.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "wave.hpp"

namespace mf {

namespace {

using wave::dn1;
using wave::up1;

// rows per tile (the walk runs on the 16-row tiles of the FP32 passes, which
// halves the extra band each tile forms below its first row), rows loaded ahead
constexpr int kBlH = kTileH2F, kBlU = 4;

struct V2 {
  double x, y;
};
__device__ __forceinline__ V2 operator-(V2 a, V2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ double dot(V2 a, V2 b) { return fma(a.x, b.x, a.y * b.y); }
__device__ __forceinline__ double cross(V2 a, V2 b) { return fma(a.x, b.y, -(a.y * b.x)); }
__device__ __forceinline__ V2 dn1v(V2 a) { return {dn1(a.x), dn1(a.y)}; }

// 1 / (2 |d|): the hardware reciprocal estimate refined by two Newton steps
// s <- s + s (1 - t s) (each squares the relative error), cheaper than the
// IEEE division sequence and within an ulp of it
__device__ __forceinline__ double half_inv_abs(double d) {
  const double t = 2.0 * fabs(d);
  double s = __builtin_amdgcn_rcp(t);
  s = fma(s, fma(-t, s, 1.0), s);
  return fma(s, fma(-t, s, 1.0), s);
}

// What one band leaves for the rows above it.
struct Band {
  V2 h;           // edge vector (x, b+1) -> (x+1, b+1)
  double u_cr;    // U's -K on the horizontal edge (x,b)-(x+1,b)
  double wv, wd;  // weights of the edges (x,b)-(x,b+1) and (x+1,b)-(x,b+1)
  double d_top;   // D's -K on the horizontal edge (x,b+1)-(x+1,b+1)
};

// Band b from three edge vectors at the lane's point C = (x, b): h = C -> R,
// v = C -> C1 and h1 = C1 -> R1; R -> R1 is the right lane's v and R -> C1 is
// v - h.  in_u / in_d: whether U(x,b) / D(x,b) lie in the macro.
__device__ __forceinline__ Band make_band(V2 h, V2 v, V2 h1, bool in_u, bool in_d) {
  Band B;
  const V2 g = v - h, f = dn1v(v);
  // one reciprocal for both triangles: 1 / (2 |det U| |det D|); a triangle
  // outside the macro enters as 1, so a degenerate one cannot spoil the other
  const double tu = in_u ? fabs(cross(h, v)) : 1.0, td = in_d ? fabs(cross(f, g)) : 1.0;
  const double sp = half_inv_abs(tu * td);
  const double su = sp * td, sd = sp * tu;
  // -K per edge of U and D (cotangent of the opposite angle over two)
  const double u_cr = dot(v, g) * su, u_cc1 = -dot(h, g) * su, u_rc1 = dot(h, v) * su;
  const double d_rr1 = -dot(g, h1) * sd, d_rc1 = dot(f, h1) * sd, d_r1c1 = dot(f, g) * sd;
  B.u_cr = in_u ? u_cr : 0.0;
  const double d_rr1m = in_d ? d_rr1 : 0.0;
  B.wv = (in_u ? u_cc1 : 0.0) + up1(d_rr1m);
  B.wd = (in_u ? u_rc1 : 0.0) + (in_d ? d_rc1 : 0.0);
  B.d_top = in_d ? d_r1c1 : 0.0;
  B.h = h1;
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
  // Edge vectors between neighbouring mapped lattice points, formed from
  // lattice differences rather than as differences of O(1) mapped
  // coordinates (which would cost about log10(N) digits): with bubble
  // n(i, j) / N^3, n(i, j) = (N - i - j) i j, the differences
  // n(x+1, r) - n(x, r) = r (N - r - 2x - 1) and n(x, r+1) - n(x, r) =
  // x (N - x - 2r - 1) are exact integers, and the scalings by powers of two
  // are exact, so each component takes one rounding.
  const double invN = 1.0 / (double)N;  // exact: N is a power of two
  const double invN3 = invN * invN * invN;
  const double e1x = G.e1[0] * invN, e1y = G.e1[1] * invN, e2x = G.e2[0] * invN, e2y = G.e2[1] * invN;
  auto hv = [&](int r) -> V2 {  // F(x+1, r) - F(x, r)
    const double nb = (double)r * (double)(N - r - 2 * x - 1) * invN3;
    return {fma(nb, bx, e1x), fma(nb, by, e1y)};
  };
  auto vv = [&](int r) -> V2 {  // F(x, r+1) - F(x, r)
    const double nb = (double)x * (double)(N - x - 2 * r - 1) * invN3;
    return {fma(nb, bx, e2x), fma(nb, by, e2y)};
  };
  // triangles U(x,b) and D(x,b) inside the macro (always, on interior tiles)
  auto in_u = [&](int b) { return INNER || (x >= 0 && b >= 0 && x + b <= N - 1); };
  auto in_d = [&](int b) { return INNER || (x >= 0 && b >= 0 && x + b <= N - 2); };
  Band bm = make_band(hv(y0 - 1), vv(y0 - 1), hv(y0), in_u(y0 - 1), in_d(y0 - 1));  // band y0-1
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
    if (!INNER && j >= nrows) break;  // interior tiles always have kBlH rows
    const Band bp = make_band(bm.h, vv(yy), hv(yy + 1), in_u(yy), in_d(yy));  // band y
    const double wh = bp.u_cr + bm.d_top;                                          // edge (x,y)-(x+1,y)
    const double acc = ((wh * (x0v - dn1(x0v)) + up1(wh) * (x0v - up1(x0v))) +
                        (bp.wv * (x0v - xp) + bm.wv * (x0v - xm))) +
                       (up1(bp.wd) * (x0v - up1(xp)) + bm.wd * (x0v - dn1(xm)));
    const bool inside = lane >= 1 && lane <= kTileW && x + yy <= N;
    if (inside) {
      const bool dir = !INNER && ((M.dir_mask >> support_mask(2, N, x, yy, 0)) & 1);
      Y[row_start(N, yy) + xc] = dir ? x0v : acc;
    }
    xm = x0v;
    x0v = xp;
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
  static_assert(kBlH == kTileH2F, "the walk runs on the FP32 tile list");
  const int nwg = (int)(L.tiles_f32.size() / kWavesPerWG);
  if (nwg > 0)
    hipLaunchKernelGGL(blended_kernel, dim3(wave::xcd_grid(nwg)), dim3(kWG), 0, s, L.dev.tiles_f32, nwg, L.dev.md,
                       m->geo2_dev, bubble, x, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return launch_exchange_apply(L, MF_F64, y, s);
}

}  // namespace mf
