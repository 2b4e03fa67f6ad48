// Fused constant-stencil kernels for CDNA4 (gfx950): interior rows of every
// macro (apply, weighted Jacobi, residual + norm partials) and the interface
// kernel that completes macro-boundary rows.
//
// The paper's vertex-to-vertex kernel (Performance Modeling section) walks
// one triangle row by row, x fastest, reading seven neighbours with constant
// weights; on a CPU its speed depends on whether three source rows plus the
// destination row fit in a cache level (the layer condition).  Here the same
// reuse is kept in registers: one 64-lane wavefront owns 64 consecutive
// columns and walks a strip of rows upward, holding rows y-1, y, y+1 (2D) or
// the five rows of slices z-1, z, z+1 (3D) and exchanging the x+-1
// neighbours through cross-lane shuffles, so every source value is read from
// memory once per tile.  Future rows are loaded U rows ahead to keep enough
// bytes in flight for HBM3E.  No matrix cores: the path is HBM-bound.

#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mf {

namespace {

template <typename T>
__device__ __forceinline__ T wgt(const MacroDev& M, int i);
template <>
__device__ __forceinline__ double wgt<double>(const MacroDev& M, int i) { return M.w[i]; }
template <>
__device__ __forceinline__ float wgt<float>(const MacroDev& M, int i) { return M.wf[i]; }

template <typename T>
__device__ __forceinline__ T kel(const MacroDev& M, int t, int i);
template <>
__device__ __forceinline__ double kel<double>(const MacroDev& M, int t, int i) { return M.K[t][i]; }
template <>
__device__ __forceinline__ float kel<float>(const MacroDev& M, int t, int i) { return M.Kf[t][i]; }

template <typename T>
__device__ __forceinline__ T invd(const MacroDev& M);
template <>
__device__ __forceinline__ double invd<double>(const MacroDev& M) { return M.inv_diag; }
template <>
__device__ __forceinline__ float invd<float>(const MacroDev& M) { return M.inv_diagf; }

template <typename T>
__device__ __forceinline__ T up1(T v) { return __shfl_up(v, 1, kWave); }      // value of lane - 1
template <typename T>
__device__ __forceinline__ T dn1(T v) { return __shfl_down(v, 1, kWave); }    // value of lane + 1

template <typename T>
__device__ __forceinline__ void st(T* p, T v) { __builtin_nontemporal_store(v, p); }

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

// Maps this block to its natural workgroup index so that each of the 8 XCDs
// (which receive blocks round-robin) works through one contiguous chunk of
// the natural order: neighbouring strips then share that XCD's L2.
__device__ __forceinline__ int xcd_wg(int nwg) {
  const int chunk = (nwg + kXCD - 1) / kXCD;
  const int k = blockIdx.x % kXCD, j = blockIdx.x / kXCD;
  if (j >= chunk) return -1;
  const int n = k * chunk + j;
  return n < nwg ? n : -1;
}

constexpr int kU2 = 8;  // rows loaded ahead (2D)
constexpr int kU3 = 4;  // rows loaded ahead per slice (3D)

// ------------------------------------------------------------------ 2D tile
template <typename T, int MODE>
__device__ __forceinline__ void tile2d(const Tile t, const MacroDev& M, const T* __restrict__ X,
                                       T* __restrict__ Y, const T* __restrict__ B, T omega, double& ss,
                                       double& mx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int x = t.x0 - 1 + lane;
  const int y0 = t.y0;
  const int y1 = min(y0 + kTileH2, N - t.x0);  // rows with x0 + y <= N - 1
  X += M.base;
  Y += M.base;
  if (MODE != kApply) B += M.base;
  const T wS = wgt<T>(M, 0), wSE = wgt<T>(M, 1), wW = wgt<T>(M, 2), wC = wgt<T>(M, 3);
  const T wE = wgt<T>(M, 4), wNW = wgt<T>(M, 5), wN = wgt<T>(M, 6);
  const T id = invd<T>(M);

  int r = y0 - 1;
  int rs = (int)row_start(N, r);
  T am = (x + r <= N) ? X[rs + x] : T(0);
  rs += N + 1 - r;
  ++r;
  T a0 = (x + r <= N) ? X[rs + x] : T(0);
  T am_r = dn1(am), a0_l = up1(a0), a0_r = dn1(a0);
  int rs_c = rs;                   // start of output row y
  int rp = r + 1;                  // next row to prefetch
  int rs_p = rs + N + 1 - r;       // its start
  T q[kU2];
  T qb[kU2];
#pragma unroll
  for (int k = 0; k < kU2; ++k) {
    q[k] = (rp <= y1 && x + rp <= N) ? X[rs_p + x] : T(0);
    if (MODE != kApply) qb[k] = (rp - 1 < y1 && x + rp - 1 <= N) ? B[rs_p - (N + 2 - rp) + x] : T(0);
    rs_p += N + 1 - rp;
    ++rp;
  }
  for (int y = y0; y < y1; y += kU2) {
#pragma unroll
    for (int k = 0; k < kU2; ++k) {
      const int yy = y + k;
      const T ap = q[k];
      const T bv = MODE != kApply ? qb[k] : T(0);
      q[k] = (rp <= y1 && x + rp <= N) ? X[rs_p + x] : T(0);
      if (MODE != kApply) qb[k] = (rp - 1 < y1 && x + rp - 1 <= N) ? B[rs_p - (N + 2 - rp) + x] : T(0);
      rs_p += N + 1 - rp;
      ++rp;
      if (yy < y1) {
        const T ap_l = up1(ap), ap_r = dn1(ap);
        T acc = wS * am;
        acc = fma(wSE, am_r, acc);
        acc = fma(wW, a0_l, acc);
        acc = fma(wC, a0, acc);
        acc = fma(wE, a0_r, acc);
        acc = fma(wNW, ap_l, acc);
        acc = fma(wN, ap, acc);
        const bool ok = lane >= 1 && lane <= kTileW && x + yy <= N - 1;
        if (ok) {
          const int o = rs_c + x;
          if (MODE == kApply) {
            st(Y + o, acc);
          } else if (MODE == kJacobi) {
            st(Y + o, fma(omega * id, bv - acc, a0));
          } else {
            const T rv = MODE == kNormB ? bv : bv - acc;
            if (MODE == kResidual) st(Y + o, rv);
            ss += (double)rv * (double)rv;
            mx = fmax(mx, fabs((double)rv));
          }
        }
        am = a0;
        am_r = a0_r;
        a0 = ap;
        a0_l = ap_l;
        a0_r = ap_r;
        rs_c += N + 1 - yy;
      }
    }
  }
}

// ------------------------------------------------------------------ 3D tile
// Slice z of a tetrahedral macro is a triangle of side M = N - z; the output
// row y of slice z reads rows y, y+1 of slice z-1, rows y-1..y+1 of slice z
// and rows y-1, y of slice z+1.
template <typename T, int MODE>
__device__ __forceinline__ void tile3d(const Tile t, const MacroDev& M, const T* __restrict__ X,
                                       T* __restrict__ Y, const T* __restrict__ B, T omega, double& ss,
                                       double& mx) {
  const int lane = threadIdx.x & (kWave - 1);
  const int N = M.N;
  const int z = t.z;
  const int S0 = N - z, Sm = S0 + 1, Sp = S0 - 1;
  const int x = t.x0 - 1 + lane;
  const int y0 = t.y0;
  const int y1 = min(y0 + kTileH3, S0 - t.x0);
  const T* Xm = X + M.base + slice_base(N, z - 1);
  const T* X0 = X + M.base + slice_base(N, z);
  const T* Xp = X + M.base + slice_base(N, z + 1);
  T* Y0 = Y + M.base + slice_base(N, z);
  const T* B0 = MODE != kApply ? B + M.base + slice_base(N, z) : nullptr;
  T w[15];
#pragma unroll
  for (int i = 0; i < 15; ++i) w[i] = wgt<T>(M, i);
  const T id = invd<T>(M);

  // preloads: slice z-1 row y0; slice z rows y0-1, y0; slice z+1 row y0-1
  int rsm = (int)row_start(Sm, y0);
  T dm0 = (x + y0 <= Sm) ? Xm[rsm + x] : T(0);
  rsm += Sm + 1 - y0;  // row y0+1 of slice z-1
  int rs0 = (int)row_start(S0, y0 - 1);
  T am = (x + y0 - 1 <= S0) ? X0[rs0 + x] : T(0);
  rs0 += S0 + 1 - (y0 - 1);
  T a0 = (x + y0 <= S0) ? X0[rs0 + x] : T(0);
  int rs_c = rs0;                 // output row y in slice z
  rs0 += S0 + 1 - y0;             // row y0+1 of slice z
  int rsp = (int)row_start(Sp, y0 - 1);
  T pm = (x + y0 - 1 <= Sp) ? Xp[rsp + x] : T(0);
  rsp += Sp + 1 - (y0 - 1);       // row y0 of slice z+1
  T dm0_r = dn1(dm0), am_r = dn1(am), a0_l = up1(a0), a0_r = dn1(a0), pm_r = dn1(pm);

  // prefetch rings: slice z-1 row y+1, slice z row y+1, slice z+1 row y, b row y
  T qm[kU3], q0[kU3], qp[kU3], qb[kU3];
  int rm_next = y0 + 1, r0_next = y0 + 1, rp_next = y0, rb_next = y0;
  int rsb = rs_c;
#pragma unroll
  for (int k = 0; k < kU3; ++k) {
    qm[k] = (rm_next <= y1 && x + rm_next <= Sm) ? Xm[rsm + x] : T(0);
    rsm += Sm + 1 - rm_next;
    ++rm_next;
    q0[k] = (r0_next <= y1 && x + r0_next <= S0) ? X0[rs0 + x] : T(0);
    rs0 += S0 + 1 - r0_next;
    ++r0_next;
    qp[k] = (rp_next < y1 && x + rp_next <= Sp) ? Xp[rsp + x] : T(0);
    rsp += Sp + 1 - rp_next;
    ++rp_next;
    if (MODE != kApply) qb[k] = (rb_next < y1 && x + rb_next <= S0) ? B0[rsb + x] : T(0);
    rsb += S0 + 1 - rb_next;
    ++rb_next;
  }
  for (int y = y0; y < y1; y += kU3) {
#pragma unroll
    for (int k = 0; k < kU3; ++k) {
      const int yy = y + k;
      const T dm1 = qm[k], ap = q0[k], p0 = qp[k];
      const T bv = MODE != kApply ? qb[k] : T(0);
      qm[k] = (rm_next <= y1 && x + rm_next <= Sm) ? Xm[rsm + x] : T(0);
      rsm += Sm + 1 - rm_next;
      ++rm_next;
      q0[k] = (r0_next <= y1 && x + r0_next <= S0) ? X0[rs0 + x] : T(0);
      rs0 += S0 + 1 - r0_next;
      ++r0_next;
      qp[k] = (rp_next < y1 && x + rp_next <= Sp) ? Xp[rsp + x] : T(0);
      rsp += Sp + 1 - rp_next;
      ++rp_next;
      if (MODE != kApply) qb[k] = (rb_next < y1 && x + rb_next <= S0) ? B0[rsb + x] : T(0);
      rsb += S0 + 1 - rb_next;
      ++rb_next;
      if (yy < y1) {
        const T dm1_l = up1(dm1), dm1_r = dn1(dm1);
        const T ap_l = up1(ap), ap_r = dn1(ap);
        const T p0_l = up1(p0), p0_r = dn1(p0);
        T acc = w[0] * dm0;
        acc = fma(w[1], dm0_r, acc);
        acc = fma(w[2], dm1, acc);
        acc = fma(w[3], dm1_l, acc);
        acc = fma(w[4], am, acc);
        acc = fma(w[5], am_r, acc);
        acc = fma(w[6], a0_l, acc);
        acc = fma(w[7], a0, acc);
        acc = fma(w[8], a0_r, acc);
        acc = fma(w[9], ap_l, acc);
        acc = fma(w[10], ap, acc);
        acc = fma(w[11], pm, acc);
        acc = fma(w[12], pm_r, acc);
        acc = fma(w[13], p0_l, acc);
        acc = fma(w[14], p0, acc);
        const bool ok = lane >= 1 && lane <= kTileW && x + yy <= S0 - 1;
        if (ok) {
          const int o = rs_c + x;
          if (MODE == kApply) {
            st(Y0 + o, acc);
          } else if (MODE == kJacobi) {
            st(Y0 + o, fma(omega * id, bv - acc, a0));
          } else {
            const T rv = MODE == kNormB ? bv : bv - acc;
            if (MODE == kResidual) st(Y0 + o, rv);
            ss += (double)rv * (double)rv;
            mx = fmax(mx, fabs((double)rv));
          }
        }
        dm0 = dm1;
        dm0_r = dm1_r;
        am = a0;
        am_r = a0_r;
        a0 = ap;
        a0_l = ap_l;
        a0_r = ap_r;
        pm = p0;
        pm_r = p0_r;
        rs_c += S0 + 1 - yy;
      }
    }
  }
}

template <typename T, int DIM>
__device__ __forceinline__ T partial_row(const MacroDev& M, const T* __restrict__ X, int x, int y, int z) {
  constexpr ElemTable ET = elem_table(DIM);
  const int N = M.N;
  T acc = T(0);
#pragma unroll
  for (int t = 0; t < ET.ntypes; ++t) {
#pragma unroll
    for (int v = 0; v < ET.nv; ++v) {
      const int ax = x - ET.off[t][v][0], ay = y - ET.off[t][v][1], az = DIM == 3 ? z - ET.off[t][v][2] : 0;
      if (ax >= 0 && ay >= 0 && az >= 0 && ax + ay + az <= N - ET.slack[t]) {
#pragma unroll
        for (int u = 0; u < ET.nv; ++u) {
          const int qx = ax + ET.off[t][u][0], qy = ay + ET.off[t][u][1], qz = az + ET.off[t][u][2];
          const int64_t qi = M.base + (DIM == 2 ? idx2(N, qx, qy) : idx3(N, qx, qy, qz));
          acc = fma(kel<T>(M, t, v * 4 + u), X[qi], acc);
        }
      }
    }
  }
  return acc;
}

template <typename T>
__device__ __forceinline__ T ginvd(const double* d, const float* f, int g);
template <>
__device__ __forceinline__ double ginvd<double>(const double* d, const float*, int g) { return d[g]; }
template <>
__device__ __forceinline__ float ginvd<float>(const double*, const float* f, int g) { return f[g]; }

// Arguments of one stencil launch (passed by value).
template <typename T>
struct StencilArgs {
  const Tile* tiles;
  int ntiles;
  int grid_int;  // blocks [0, grid_int) do interior tiles, the rest interface groups
  int ngroups;
  const int32_t* gptr;
  const Copy* copies;
  const uint8_t* gflag;
  const double* ginv;
  const float* ginvf;
  const MacroDev* md;
  const T* X;
  T* Y;
  const T* B;
  T omega;
  double* part;   // sums at [0, np), maxima at [np, 2 np); interface slots start at ntiles
  int np;
};

// One interface group (unique macro-boundary DoF): sum the partial rows of
// its copies in fixed macro order, finish the row for MODE, write all copies.
template <typename T, int DIM, int MODE>
__device__ __forceinline__ void iface_group(const StencilArgs<T>& a, int g, double& ss, double& mx) {
  const int c0 = a.gptr[g], c1 = a.gptr[g + 1];
  const bool dir = a.gflag[g] & 1;
  const Copy cp0 = a.copies[c0];
  const MacroDev& M0 = a.md[cp0.macro];
  const int64_t i0 = M0.base + (DIM == 2 ? idx2(M0.N, cp0.x, cp0.y) : idx3(M0.N, cp0.x, cp0.y, cp0.z));
  bool write = true;
  T out = T(0);
  if (MODE == kExchangeSum) {
    if (!dir) {
      for (int c = c0; c < c1; ++c) {
        const Copy cp = a.copies[c];
        const MacroDev& Mc = a.md[cp.macro];
        out += a.X[Mc.base + (DIM == 2 ? idx2(Mc.N, cp.x, cp.y) : idx3(Mc.N, cp.x, cp.y, cp.z))];
      }
    }
  } else if (MODE == kDirichletSet) {
    write = dir;
    if (dir) out = a.B[i0];
  } else if (MODE == kNormB) {
    write = false;
    out = a.B[i0];
  } else if (dir) {
    const T xv = a.X[i0];
    if (MODE == kApply || MODE == kJacobi) out = xv;
    else out = a.B[i0] - xv;
  } else {
    T acc = T(0);
    for (int c = c0; c < c1; ++c) {
      const Copy cp = a.copies[c];
      acc += partial_row<T, DIM>(a.md[cp.macro], a.X, cp.x, cp.y, cp.z);
    }
    if (MODE == kApply) out = acc;
    else if (MODE == kJacobi) out = fma(a.omega * ginvd<T>(a.ginv, a.ginvf, g), a.B[i0] - acc, a.X[i0]);
    else out = a.B[i0] - acc;
  }
  if (MODE == kResidual || MODE == kNormB) {
    ss = (double)out * (double)out;
    mx = fabs((double)out);
  }
  if (write) {
    for (int c = c0; c < c1; ++c) {
      const Copy cp = a.copies[c];
      const MacroDev& Mc = a.md[cp.macro];
      a.Y[Mc.base + (DIM == 2 ? idx2(Mc.N, cp.x, cp.y) : idx3(Mc.N, cp.x, cp.y, cp.z))] = out;
    }
  }
}

// The whole operator in one launch: interior wave tiles first (mapped to
// XCDs in contiguous chunks), then one thread per interface group.  The two
// parts write disjoint entries, so they need no ordering.
template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(kWG) void stencil_kernel(const StencilArgs<T> a) {
  constexpr bool kPart = MODE == kResidual || MODE == kNormB;
  double ss = 0.0, mx = 0.0;
  if ((int)blockIdx.x < a.grid_int) {
    const int nwg = a.ntiles / kWavesPerWG;
    const int n = xcd_wg(nwg);
    if (n < 0) return;
    const int ti = n * kWavesPerWG + (threadIdx.x >> 6);
    const Tile t = a.tiles[ti];
    if (t.macro >= 0) {
      const MacroDev& M = a.md[t.macro];
      if (DIM == 2)
        tile2d<T, MODE>(t, M, a.X, a.Y, a.B, a.omega, ss, mx);
      else
        tile3d<T, MODE>(t, M, a.X, a.Y, a.B, a.omega, ss, mx);
    }
    if (kPart && a.part != nullptr) {
      ss = wave_sum(ss);
      mx = wave_max(mx);
      if ((threadIdx.x & (kWave - 1)) == 0) {
        a.part[ti] = ss;
        a.part[a.np + ti] = mx;
      }
    }
    return;
  }
  const int ib = blockIdx.x - a.grid_int;
  const int g = ib * kWG + threadIdx.x;
  if (g < a.ngroups) iface_group<T, DIM, MODE>(a, g, ss, mx);
  if (kPart && a.part != nullptr) {
    __shared__ double s_ss[kWavesPerWG], s_mx[kWavesPerWG];
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
      for (int i = 0; i < kWavesPerWG; ++i) {
        p += s_ss[i];
        q = fmax(q, s_mx[i]);
      }
      a.part[a.ntiles + ib] = p;
      a.part[a.np + a.ntiles + ib] = q;
    }
  }
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ part, int64_t np,
                                                     double* __restrict__ result) {
  __shared__ double s[256], m[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 256) {
    a += part[i];
    b = fmax(b, part[np + i]);
  }
  s[threadIdx.x] = a;
  m[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s[threadIdx.x] += s[threadIdx.x + w];
      m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    result[0] = s[0];
    result[1] = m[0];
  }
}

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

// interior: include the interior tiles; iface: include the interface groups
template <typename T, int DIM, int MODE>
void run(const Level& L, bool interior, bool iface, const void* x, void* y, const void* b, double omega,
         double* part, int64_t np, hipStream_t s) {
  StencilArgs<T> a;
  a.tiles = L.dev.tiles;
  a.ntiles = interior ? (int)L.tiles.size() : 0;
  const int nwg = a.ntiles / kWavesPerWG;
  a.grid_int = interior ? kXCD * ((nwg + kXCD - 1) / kXCD) : 0;
  a.ngroups = iface ? (int)L.ngroups() : 0;
  a.gptr = L.dev.grp_ptr;
  a.copies = L.dev.copies;
  a.gflag = L.dev.grp_flag;
  a.ginv = L.dev.grp_invdiag;
  a.ginvf = L.dev.grp_invdiagf;
  a.md = L.dev.md;
  a.X = (const T*)x;
  a.Y = (T*)y;
  a.B = (const T*)b;
  a.omega = (T)omega;
  a.part = part;
  a.np = (int)np;
  const int grid_if = (a.ngroups + kWG - 1) / kWG;
  const int grid = a.grid_int + grid_if;
  if (grid == 0) return;
  hipLaunchKernelGGL((stencil_kernel<T, DIM, MODE>), dim3(grid), dim3(kWG), 0, s, a);
}

template <typename T, int DIM>
void dispatch(int mode, const Level& L, bool interior, bool iface, const void* x, void* y, const void* b,
              double omega, double* part, int64_t np, hipStream_t s) {
  switch (mode) {
    case kApply: run<T, DIM, kApply>(L, interior, iface, x, y, b, omega, part, np, s); break;
    case kJacobi: run<T, DIM, kJacobi>(L, interior, iface, x, y, b, omega, part, np, s); break;
    case kResidual: run<T, DIM, kResidual>(L, interior, iface, x, y, b, omega, part, np, s); break;
    case kNormB: run<T, DIM, kNormB>(L, interior, iface, x, y, b, omega, part, np, s); break;
    case kExchangeSum: run<T, DIM, kExchangeSum>(L, false, true, x, y, b, omega, part, np, s); break;
    default: run<T, DIM, kDirichletSet>(L, false, true, x, y, b, omega, part, np, s); break;
  }
}

int launch(const mf_mesh* m, const Level& L, int dtype, int mode, bool interior, bool iface, const void* x,
           void* y, const void* b, double omega, double* part, int64_t np, hipStream_t s) {
  if (dtype == MF_F64) {
    if (m->dim == 2) dispatch<double, 2>(mode, L, interior, iface, x, y, b, omega, part, np, s);
    else dispatch<double, 3>(mode, L, interior, iface, x, y, b, omega, part, np, s);
  } else {
    if (m->dim == 2) dispatch<float, 2>(mode, L, interior, iface, x, y, b, omega, part, np, s);
    else dispatch<float, 3>(mode, L, interior, iface, x, y, b, omega, part, np, s);
  }
  return check_launch();
}

}  // namespace

int launch_stencil(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                   double omega, double* part, hipStream_t s) {
  return launch(m, L, dtype, mode, true, true, x, y, b, omega, part, L.n_partials(), s);
}

int launch_iface(const mf_mesh* m, const Level& L, int dtype, int mode, const void* x, void* y, const void* b,
                 hipStream_t s) {
  return launch(m, L, dtype, mode, false, true, x, y, b, 0.0, nullptr, 0, s);
}

int launch_reduce(const double* part, int64_t np, double* result, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, part, np, result);
  return check_launch();
}

}  // namespace mf
