// Per-point kernels: keyed random fill, multigrid restriction and
// prolongation, the coarse direct solve, and plain vector operations.
//
// The paper names multigrid as the natural use of its refinement levels
// (Intro, "Hybrid Tetrahedral Grids") and smoothers and vector additions as
// further generated operations (Performance Modeling section) but gives no
// detail; the transfers here are the P1 interpolation between nested levels
// and its transpose.

#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace mf {

namespace {

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <int DIM>
__device__ __forceinline__ int64_t lidx(int N, int x, int y, int z) {
  return DIM == 2 ? idx2(N, x, y) : idx3(N, x, y, z);
}

// x = 2u - 1 with u from the hash chained over (seed, sorted key pairs).
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void fill_random_kernel(const Tile* __restrict__ segs, int nseg,
                                                          const MacroDev* __restrict__ md, uint64_t seed,
                                                          T* __restrict__ X) {
  const int si = blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
  if (si >= nseg) return;
  const Tile sg = segs[si];
  if (sg.macro < 0) return;
  const MacroDev& M = md[sg.macro];
  const int N = M.N;
  const int x = sg.x0 + (threadIdx.x & (kWave - 1));
  const int y = sg.y0, z = DIM == 3 ? sg.z : 0;
  if (x + y + z > N) return;
  int64_t v[4];
  int64_t w[4];
  const int64_t wt[4] = {N - x - y - z, x, y, z};
  int n = 0;
  for (int k = 0; k <= DIM; ++k)
    if (wt[k] != 0) {
      v[n] = M.vid[k];
      w[n] = wt[k];
      ++n;
    }
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && v[j] < v[j - 1]; --j) {
      const int64_t tv = v[j], tw = w[j];
      v[j] = v[j - 1];
      w[j] = w[j - 1];
      v[j - 1] = tv;
      w[j - 1] = tw;
    }
  uint64_t h = splitmix(seed);
  for (int i = 0; i < n; ++i) h = splitmix(h ^ (((uint64_t)v[i] << 24) | (uint64_t)w[i]));
  const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
  X[M.base + lidx<DIM>(N, x, y, z)] = (T)(2.0 * u - 1.0);
}

// Restriction r_c = P^T r_f on one macro: a coarse point P gathers the fine
// point 2P (weight 1) and the fine points 2P + d for the stencil offsets d
// (weight 1/2) — the fine points whose interpolation uses P — counting only
// fine points this macro owns, so that the later exchange sums each fine DoF
// once.  Dirichlet fine points are skipped.
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void restrict_kernel(const Tile* __restrict__ segs, int nseg,
                                                       const MacroDev* __restrict__ mdc,
                                                       const MacroDev* __restrict__ mdf, const T* __restrict__ Rf,
                                                       T* __restrict__ Bc) {
  constexpr StencilTable ST = stencil_table(DIM);
  constexpr int full = DIM == 2 ? 7 : 15;
  const int si = blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
  if (si >= nseg) return;
  const Tile sg = segs[si];
  if (sg.macro < 0) return;
  const MacroDev& C = mdc[sg.macro];
  const MacroDev& F = mdf[sg.macro];
  const int Nc = C.N, Nf = F.N;
  const int x = sg.x0 + (threadIdx.x & (kWave - 1));
  const int y = sg.y0, z = DIM == 3 ? sg.z : 0;
  if (x + y + z > Nc) return;
  T acc = T(0);
#pragma unroll
  for (int s = 0; s < ST.n; ++s) {
    const int fx = 2 * x + ST.off[s][0], fy = 2 * y + ST.off[s][1], fz = DIM == 3 ? 2 * z + ST.off[s][2] : 0;
    if (fx < 0 || fy < 0 || fz < 0 || fx + fy + fz > Nf) continue;
    const int mask = support_mask(DIM, Nf, fx, fy, fz);
    const bool owned = mask == full || ((F.own_mask >> mask) & 1);
    const bool dir = mask != full && ((F.dir_mask >> mask) & 1);
    if (owned && !dir) {
      const T r = Rf[F.base + lidx<DIM>(Nf, fx, fy, fz)];
      acc += (s == ST.centre) ? r : T(0.5) * r;
    }
  }
  Bc[C.base + lidx<DIM>(Nc, x, y, z)] = acc;
}

// x_f += P e_c: even fine points take the coarse value, the others the mean
// of the two coarse endpoints of the coarse micro-edge they bisect; the
// edge direction follows from the coordinate parities.  Dirichlet points are
// left unchanged.
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void prolong_add_kernel(const Tile* __restrict__ segs, int nseg,
                                                          const MacroDev* __restrict__ mdc,
                                                          const MacroDev* __restrict__ mdf,
                                                          const T* __restrict__ Ec, T* __restrict__ Xf) {
  constexpr int full = DIM == 2 ? 7 : 15;
  const int si = blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
  if (si >= nseg) return;
  const Tile sg = segs[si];
  if (sg.macro < 0) return;
  const MacroDev& C = mdc[sg.macro];
  const MacroDev& F = mdf[sg.macro];
  const int Nc = C.N, Nf = F.N;
  const int x = sg.x0 + (threadIdx.x & (kWave - 1));
  const int y = sg.y0, z = DIM == 3 ? sg.z : 0;
  if (x + y + z > Nf) return;
  const int mask = support_mask(DIM, Nf, x, y, z);
  if (mask != full && ((F.dir_mask >> mask) & 1)) return;
  const int px = x & 1, py = y & 1, pz = z & 1;
  T e;
  if (!(px | py | pz)) {
    e = Ec[C.base + lidx<DIM>(Nc, x >> 1, y >> 1, z >> 1)];
  } else {
    // direction s of the bisected coarse edge: equal to the parity pattern,
    // except that of two or three odd coordinates the middle ones flip sign
    int sx = px, sy = py, sz = pz;
    if (px && py && !pz) sy = -1;        // (1,1,0) -> e1 - e2
    else if (px && !py && pz) sz = -1;   // (1,0,1) -> e1 - e3
    else if (!px && py && pz) sz = -1;   // (0,1,1) -> e2 - e3
    else if (px && py && pz) sy = -1;    // (1,1,1) -> e1 - e2 + e3
    const T a = Ec[C.base + lidx<DIM>(Nc, (x - sx) >> 1, (y - sy) >> 1, (z - sz) >> 1)];
    const T b = Ec[C.base + lidx<DIM>(Nc, (x + sx) >> 1, (y + sy) >> 1, (z + sz) >> 1)];
    e = T(0.5) * (a + b);
  }
  Xf[F.base + lidx<DIM>(Nf, x, y, z)] += e;
}

// Coarse direct solve: x(copies of unknown i) = sum_j Ainv[i][j] b(first copy of j).
// One wavefront per unknown; x must be zero elsewhere beforehand.
template <typename T>
__global__ __launch_bounds__(kWG) void coarse_solve_kernel(int n, const T* __restrict__ Ainv,
                                                           const int32_t* __restrict__ first,
                                                           const int32_t* __restrict__ cptr,
                                                           const int64_t* __restrict__ cidx,
                                                           const T* __restrict__ B, T* __restrict__ X) {
  const int i = blockIdx.x * kWavesPerWG + (threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  if (i >= n) return;
  T acc = T(0);
  for (int j = lane; j < n; j += kWave) acc = fma(Ainv[(int64_t)i * n + j], B[first[j]], acc);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  for (int c = cptr[i] + lane; c < cptr[i + 1]; c += kWave) X[cidx[c]] = acc;
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ x, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}
template <typename T>
__global__ void copy_kernel(T* __restrict__ d, const T* __restrict__ s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
template <typename T>
__global__ void axpy_kernel(T* __restrict__ y, const T* __restrict__ x, T a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fma(a, x[i], y[i]);
}
__global__ void scale_to_f32_kernel(const double* __restrict__ r, float* __restrict__ b, double s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (float)(s * r[i]);
}
__global__ void axpy_f32_kernel(double* __restrict__ x, const float* __restrict__ e, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = fma(a, (double)e[i], x[i]);
}

inline int blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

int launch_fill_random(const mf_mesh* m, const Level& L, int dtype, uint64_t seed, void* x, hipStream_t s) {
  const int nseg = (int)L.segs.size();
  const int grid = (nseg + kWavesPerWG - 1) / kWavesPerWG;
  if (grid == 0) return MF_OK;
  if (dtype == MF_F64) {
    if (m->dim == 2) hipLaunchKernelGGL((fill_random_kernel<double, 2>), dim3(grid), dim3(kWG), 0, s, L.dev.segs, nseg, L.dev.md, seed, (double*)x);
    else hipLaunchKernelGGL((fill_random_kernel<double, 3>), dim3(grid), dim3(kWG), 0, s, L.dev.segs, nseg, L.dev.md, seed, (double*)x);
  } else {
    if (m->dim == 2) hipLaunchKernelGGL((fill_random_kernel<float, 2>), dim3(grid), dim3(kWG), 0, s, L.dev.segs, nseg, L.dev.md, seed, (float*)x);
    else hipLaunchKernelGGL((fill_random_kernel<float, 3>), dim3(grid), dim3(kWG), 0, s, L.dev.segs, nseg, L.dev.md, seed, (float*)x);
  }
  return check_launch();
}

int launch_restrict(const mf_mesh* m, const Level& F, const Level& C, int dtype, const void* rf, void* bc,
                    hipStream_t s) {
  const int nseg = (int)C.segs.size();
  const int grid = (nseg + kWavesPerWG - 1) / kWavesPerWG;
  if (grid == 0) return MF_OK;
  if (dtype == MF_F64) {
    if (m->dim == 2) hipLaunchKernelGGL((restrict_kernel<double, 2>), dim3(grid), dim3(kWG), 0, s, C.dev.segs, nseg, C.dev.md, F.dev.md, (const double*)rf, (double*)bc);
    else hipLaunchKernelGGL((restrict_kernel<double, 3>), dim3(grid), dim3(kWG), 0, s, C.dev.segs, nseg, C.dev.md, F.dev.md, (const double*)rf, (double*)bc);
  } else {
    if (m->dim == 2) hipLaunchKernelGGL((restrict_kernel<float, 2>), dim3(grid), dim3(kWG), 0, s, C.dev.segs, nseg, C.dev.md, F.dev.md, (const float*)rf, (float*)bc);
    else hipLaunchKernelGGL((restrict_kernel<float, 3>), dim3(grid), dim3(kWG), 0, s, C.dev.segs, nseg, C.dev.md, F.dev.md, (const float*)rf, (float*)bc);
  }
  int rc = check_launch();
  if (rc) return rc;
  return launch_iface(m, C, dtype, kExchangeSum, bc, bc, nullptr, s);
}

int launch_prolong_add(const mf_mesh* m, const Level& F, const Level& C, int dtype, const void* ec, void* xf,
                       hipStream_t s) {
  const int nseg = (int)F.segs.size();
  const int grid = (nseg + kWavesPerWG - 1) / kWavesPerWG;
  if (grid == 0) return MF_OK;
  if (dtype == MF_F64) {
    if (m->dim == 2) hipLaunchKernelGGL((prolong_add_kernel<double, 2>), dim3(grid), dim3(kWG), 0, s, F.dev.segs, nseg, C.dev.md, F.dev.md, (const double*)ec, (double*)xf);
    else hipLaunchKernelGGL((prolong_add_kernel<double, 3>), dim3(grid), dim3(kWG), 0, s, F.dev.segs, nseg, C.dev.md, F.dev.md, (const double*)ec, (double*)xf);
  } else {
    if (m->dim == 2) hipLaunchKernelGGL((prolong_add_kernel<float, 2>), dim3(grid), dim3(kWG), 0, s, F.dev.segs, nseg, C.dev.md, F.dev.md, (const float*)ec, (float*)xf);
    else hipLaunchKernelGGL((prolong_add_kernel<float, 3>), dim3(grid), dim3(kWG), 0, s, F.dev.segs, nseg, C.dev.md, F.dev.md, (const float*)ec, (float*)xf);
  }
  return check_launch();
}

int launch_coarse_solve(const Level& L, int dtype, const void* b, void* x, hipStream_t s) {
  int rc = launch_fill(dtype, x, 0.0, L.storage, s);
  if (rc) return rc;
  const int n = (int)L.ncoarse;
  if (n == 0) return MF_OK;
  const int grid = (n + kWavesPerWG - 1) / kWavesPerWG;
  if (dtype == MF_F64)
    hipLaunchKernelGGL((coarse_solve_kernel<double>), dim3(grid), dim3(kWG), 0, s, n, L.dev.cinv, L.dev.cfirst,
                       L.dev.cptr, L.dev.cidx, (const double*)b, (double*)x);
  else
    hipLaunchKernelGGL((coarse_solve_kernel<float>), dim3(grid), dim3(kWG), 0, s, n, L.dev.cinvf, L.dev.cfirst,
                       L.dev.cptr, L.dev.cidx, (const float*)b, (float*)x);
  return check_launch();
}

int launch_fill(int dtype, void* x, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  if (dtype == MF_F64) hipLaunchKernelGGL((fill_kernel<double>), dim3(blocks_for(n)), dim3(256), 0, s, (double*)x, v, n);
  else hipLaunchKernelGGL((fill_kernel<float>), dim3(blocks_for(n)), dim3(256), 0, s, (float*)x, (float)v, n);
  return check_launch();
}

int launch_copy(int dtype, void* d, const void* src, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  if (dtype == MF_F64) hipLaunchKernelGGL((copy_kernel<double>), dim3(blocks_for(n)), dim3(256), 0, s, (double*)d, (const double*)src, n);
  else hipLaunchKernelGGL((copy_kernel<float>), dim3(blocks_for(n)), dim3(256), 0, s, (float*)d, (const float*)src, n);
  return check_launch();
}

int launch_axpy(int dtype, void* y, const void* x, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  if (dtype == MF_F64) hipLaunchKernelGGL((axpy_kernel<double>), dim3(blocks_for(n)), dim3(256), 0, s, (double*)y, (const double*)x, a, n);
  else hipLaunchKernelGGL((axpy_kernel<float>), dim3(blocks_for(n)), dim3(256), 0, s, (float*)y, (const float*)x, (float)a, n);
  return check_launch();
}

int launch_scale_to_f32(const double* r, float* b, double scale, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  hipLaunchKernelGGL(scale_to_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, s, r, b, scale, n);
  return check_launch();
}

int launch_axpy_f32(double* x, const float* e, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  hipLaunchKernelGGL(axpy_f32_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, e, a, n);
  return check_launch();
}

}  // namespace mf
