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
#include "rows.hpp"

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






// Each wave walks several tiles.  In 3D all loads of a step are issued
// before any store: the restriction's step takes kTransferU strided 64-point
// segments of coarse points, the prolongation's a run of slice segments of
// fine points (up to kTransferRun of one slice: one record, macro and
// slice-base lookup for all of them).  2D walks single segments.
constexpr int kTransferU = 4;

template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void restrict_kernel(const Launch<TransferArgs<T>> L) {
  TransferArgs<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int stride = a.nblk * kWavesPerWG;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if constexpr (DIM == 3) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int si = blk * kWavesPerWG + w; si < a.nseg; si += kTransferU * stride) {
      T acc[kTransferU];
      int64_t di[kTransferU];
      bool wr[kTransferU];
#pragma unroll
      for (int k = 0; k < kTransferU; ++k) {
        const int sk = si + k * stride;
        const Tile sg = sk < a.nseg ? load_seg(a.segs, sk) : Tile{-1, 0, 0, 0};
        wr[k] = false;
        if (sg.macro >= 0) acc[k] = restrict_seg3<T>(a, sg, sg.x0 + lane, true, di[k], wr[k]);
      }
#pragma unroll
      for (int k = 0; k < kTransferU; ++k)
        if (wr[k]) a.dst[di[k]] = acc[k];
    }
  } else {
    for (int si = blk * kWavesPerWG + w; si < a.nseg; si += stride) {
      const Tile sg = load_seg(a.segs, si);
      if (sg.macro >= 0) restrict_segment<T, DIM>(a, sg);
    }
  }
}


// x_f += P e_c.
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void prolong_add_kernel(const Launch<TransferArgs<T>> L) {
  TransferArgs<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int stride = a.nblk * kWavesPerWG;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if constexpr (DIM == 3) {
    const int lane = threadIdx.x & (kWave - 1);
    for (int si = blk * kWavesPerWG + w; si < a.nseg; si += stride) {
      const Tile run = load_seg(a.segs, si);
      if (run.macro < 0) continue;
      T u[kTransferRun], v[kTransferRun], xo[kTransferRun];
      int64_t di[kTransferRun];
      bool wr[kTransferRun];
#pragma unroll
      for (int k = 0; k < kTransferRun; ++k) {
        const int q = k * kWave + lane;
        wr[k] = false;
        if (k * kWave < run.y0) prolong_seg3<T>(a, run, run.x0 + q, q < run.y0, di[k], u[k], v[k], wr[k]);
      }
#pragma unroll
      for (int k = 0; k < kTransferRun; ++k)
        if (wr[k]) xo[k] = a.dst[di[k]];
#pragma unroll
      for (int k = 0; k < kTransferRun; ++k)
        if (wr[k]) a.dst[di[k]] = xo[k] + T(0.5) * (u[k] + v[k]);
    }
  } else {
    for (int si = blk * kWavesPerWG + w; si < a.nseg; si += stride) {
      const Tile sg = load_seg(a.segs, si);
      if (sg.macro >= 0) prolong_segment<T, DIM>(a, sg);
    }
  }
}



// First sweep from a zero iterate, pass 1: the interior row formula at every
// point of every macro (a plain stream over each macro's storage range).
template <typename T>
__global__ __launch_bounds__(kWG) void jacobi0_stream_kernel(const Launch<Jacobi0Args<T>> L) {
  Jacobi0Args<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int m = blk / a.bpm;
  const int64_t begin = (int64_t)(blk - m * a.bpm) * kJ0Points;
  const int64_t end = min(begin + (int64_t)kJ0Points, a.P);
  const MacroDev& M = a.md[m];
  const T c = a.omega * Prec<T>::invd(M);
  const T* __restrict__ B = a.B + M.base;
  T* __restrict__ Y = a.Y + M.base;
  // all of a thread's loads first, then the stores
  constexpr int kPer = kJ0Points / kWG;
  T v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = begin + threadIdx.x + (int64_t)k * kWG;
    v[k] = i < end ? B[i] : T(0);
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = begin + threadIdx.x + (int64_t)k * kWG;
    if (i < end) Y[i] = fma(c, v[k], T(0));
  }
}

// Pass 2: the macro-boundary DoFs, as jacobi0_point and jacobi0_group finish
// them (0 at Dirichlet DoFs, the partial stencil's centre at unshared ones,
// the assembled diagonal at shared ones).
template <typename T, int DIM>
__global__ __launch_bounds__(kWG) void jacobi0_fix_kernel(const Launch<Jacobi0Args<T>> L) {
  constexpr int full = DIM == 2 ? 7 : 15;
  constexpr int centre = stencil_table(DIM).centre;
  Jacobi0Args<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  if (blk < a.nblk_all) {
    const int g = blk * kWG + (int)threadIdx.x;
    if (g >= a.nall) return;
    const int c0 = a.aptr[g], c1 = a.aptr[g + 1];
    for (int c = c0; c < c1; ++c) {
      const Copy& k = a.acopies[c];
      const MacroDev& M = a.md[k.macro];
      const int mask = support_mask(DIM, M.N, k.x, k.y, k.z);
      const bool dir = mask != full && ((M.dir_mask >> mask) & 1);
      const bool shared = mask != full && !dir && ((M.shared_mask >> mask) & 1);
      if (shared) continue;  // the exchange part below
      const int64_t i = copy_index<DIM>(M, k);
      a.Y[i] = dir ? T(0) : fma(a.omega * centre_inv<T>(M, mask, full, centre), a.B[i], T(0));
    }
    return;
  }
  const int g = (blk - a.nblk_all) * kWG + (int)threadIdx.x;
  if (g < a.ngroups) jacobi0_group<T, DIM>(a, g);
}

// Coarse direct solve: x(copies of unknown i) = sum_j Ainv[i][j] b(first copy of j).
// One wavefront per unknown; x must be zero elsewhere beforehand.
template <typename T>
__global__ __launch_bounds__(kWG) void coarse_solve_kernel(const Launch<CoarseArgs<T>> L) {
  CoarseArgs<T> a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int i = blk * kWavesPerWG + (threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  if (i >= a.n) return;
  coarse_row<T>(a, i, lane);
}

// Plain vector kernels: grid-stride loops over each request's nblk blocks.
template <typename T, int KIND>
__global__ __launch_bounds__(256) void vector_kernel(const Launch<VecArgs> L) {
  VecArgs a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int64_t stride = (int64_t)a.nblk * 256;
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  if (KIND == kOpFill) {
    const T v = (T)a.a;
    for (; i < a.n; i += stride) ((T*)a.y)[i] = v;
  } else if (KIND == kOpCopy) {
    for (; i < a.n; i += stride) ((T*)a.y)[i] = ((const T*)a.x)[i];
  } else if (KIND == kOpAxpy) {
    const T c = (T)a.a;
    for (; i < a.n; i += stride) ((T*)a.y)[i] = fma(c, ((const T*)a.x)[i], ((T*)a.y)[i]);
  } else if (KIND == kOpScaleF32) {
    const double c = 1.0 / a.res[1];
    for (; i < a.n; i += stride) ((float*)a.y)[i] = (float)(c * ((const double*)a.x)[i]);
  } else {
    const double c = a.res[1];
    for (; i < a.n; i += stride) ((double*)a.y)[i] = fma(c, (double)((const float*)a.x)[i], ((double*)a.y)[i]);
  }
}

// ---------------------------------------------------------------- PCG
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// Grid-stride over the storage index, nblk blocks of 256 threads.  KIND
// kOpPcgZDot: z = s e with s = res[sslot] for FP32 e (the preconditioner
// solved for r / s) and 1 for FP64 e, partials of r . z.  KIND kOpPcgUpdate:
// alpha = res[2] / res[4], x += alpha p, r -= alpha q, partials of r . r and
// max |r|; with r32, also the next FP32 preconditioner input r / res[1]
// (res[1] = max |r| of the residual before this update) and *sout = res[1].
// Sums count each unique DoF once (owner bits); each block leaves one
// partial, its four waves summed in a fixed order.
constexpr int kPcgU = 4;

template <int KIND, typename TE>
__global__ __launch_bounds__(256) void pcg_lin_kernel(const Launch<PcgArgs> L) {
  PcgArgs a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int64_t stride = (int64_t)a.nblk * 256;
  double ss = 0.0, mx = 0.0;
  // kPcgU elements per thread and step, all loads issued before any use (the
  // owner-bit test selects instead of branching around the load), so each
  // thread keeps kPcgU independent loads in flight; the elements are still
  // taken in index order, so the sums are those of a one-element loop.
  const int64_t i0 = (int64_t)blk * 256 + threadIdx.x;
  if (KIND == kOpPcgZDot) {
    const double sc = sizeof(TE) == 4 ? a.res[a.sslot] : 1.0;
    const TE* e = (const TE*)a.e;
    const bool wz = a.z != nullptr && (const void*)a.z != a.e;
    for (int64_t i = i0; i < a.n; i += kPcgU * stride) {
      double zv[kPcgU], rv[kPcgU];
      uint32_t ow[kPcgU];
#pragma unroll
      for (int u = 0; u < kPcgU; ++u) {
        const int64_t j = i + u * stride, jj = j < a.n ? j : i;
        zv[u] = sc * (double)e[jj];
        rv[u] = a.r[jj];
        ow[u] = a.own[jj >> 5];
      }
#pragma unroll
      for (int u = 0; u < kPcgU; ++u) {
        const int64_t j = i + u * stride;
        if (j >= a.n) break;
        if (wz) a.z[j] = zv[u];
        if ((ow[u] >> (j & 31)) & 1u) ss = fma(rv[u], zv[u], ss);
      }
    }
  } else {
    const double alpha = a.res[2] / a.res[4];
    const double c32 = a.r32 ? 1.0 / a.res[1] : 0.0;  // as the scaled cast forms it
    if (a.r32 && blk == 0 && threadIdx.x == 0) *a.sout = a.res[1];
    for (int64_t i = i0; i < a.n; i += kPcgU * stride) {
      double xv[kPcgU], pv[kPcgU], qv[kPcgU], rv[kPcgU];
      uint32_t ow[kPcgU];
#pragma unroll
      for (int u = 0; u < kPcgU; ++u) {
        const int64_t j = i + u * stride, jj = j < a.n ? j : i;
        xv[u] = a.x[jj];
        pv[u] = a.p[jj];
        qv[u] = a.q[jj];
        rv[u] = a.r[jj];
        ow[u] = a.own[jj >> 5];
      }
#pragma unroll
      for (int u = 0; u < kPcgU; ++u) {
        const int64_t j = i + u * stride;
        if (j >= a.n) break;
        a.x[j] = fma(alpha, pv[u], xv[u]);
        const double rn = fma(-alpha, qv[u], rv[u]);
        a.r[j] = rn;
        if (a.r32) a.r32[j] = (float)(c32 * rn);
        if ((ow[u] >> (j & 31)) & 1u) ss = fma(rn, rn, ss);
        mx = fmax(mx, fabs(rn));
      }
    }
  }
  ss = wsum(ss);
  mx = wmax(mx);
  __shared__ double s_ss[4], s_mx[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_ss[w] = ss;
    s_mx[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a.part[blk] = (s_ss[0] + s_ss[1]) + (s_ss[2] + s_ss[3]);
    a.part[a.nblk + blk] = fmax(fmax(s_mx[0], s_mx[1]), fmax(s_mx[2], s_mx[3]));
  }
}

// p = z + beta p, beta = res[2] / res[3] (0 on the first iteration, res[3] == 0).
// p = z + beta p.  TZ = double: x is z; TZ = float: x is the FP32 V-cycle
// output e and z = res[1] e is formed here exactly as the r . z pass forms it
// (the mixed solver never stores z).
template <typename TZ>
__global__ __launch_bounds__(256) void pcg_dir_kernel(const Launch<VecArgs> L) {
  VecArgs a;
  const int blk = resolve(L, (int)blockIdx.x, a);
  const int64_t stride = (int64_t)a.nblk * 256;
  double* p = (double*)a.y;
  const TZ* zs = (const TZ*)a.x;
  const double sc = sizeof(TZ) == 4 ? a.res[a.sslot] : 1.0;
  auto z = [&](int64_t i) { return sizeof(TZ) == 4 ? sc * (double)zs[i] : (double)zs[i]; };
  if (a.res[3] == 0.0) {
    // first direction: p = z (p holds no earlier direction and is never read)
    for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < a.n; i += stride) p[i] = z(i);
    return;
  }
  const double beta = a.res[2] / a.res[3];
  for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < a.n; i += stride) p[i] = fma(beta, p[i], z(i));
}

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

template <int KIND>
int run_vector(int dtype, const Launch<VecArgs>& l, hipStream_t s) {
  if (l.nwg <= 0) return MF_OK;
  if (dtype == MF_F64) hipLaunchKernelGGL((vector_kernel<double, KIND>), dim3(l.nwg), dim3(256), 0, s, l);
  else hipLaunchKernelGGL((vector_kernel<float, KIND>), dim3(l.nwg), dim3(256), 0, s, l);
  return check_launch();
}

template <typename T>
void run_transfer(bool restrict_op, int dim, const Launch<TransferArgs<T>>& l, hipStream_t s) {
  if (restrict_op) {
    if (dim == 2) hipLaunchKernelGGL((restrict_kernel<T, 2>), dim3(l.nwg), dim3(kWG), 0, s, l);
    else hipLaunchKernelGGL((restrict_kernel<T, 3>), dim3(l.nwg), dim3(kWG), 0, s, l);
  } else {
    if (dim == 2) hipLaunchKernelGGL((prolong_add_kernel<T, 2>), dim3(l.nwg), dim3(kWG), 0, s, l);
    else hipLaunchKernelGGL((prolong_add_kernel<T, 3>), dim3(l.nwg), dim3(kWG), 0, s, l);
  }
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
  const int nwg = transfer_blocks((int)C.psegs.size());
  if (nwg == 0) return MF_OK;
  if (dtype == MF_F64) run_transfer<double>(true, m->dim, single(restrict_args<double>(F, C, rf, bc), nwg), s);
  else run_transfer<float>(true, m->dim, single(restrict_args<float>(F, C, rf, bc), nwg), s);
  int rc = check_launch();
  if (rc) return rc;
  return launch_iface(m, C, dtype, kExchangeSum, bc, bc, nullptr, s);
}

int launch_prolong_add(const mf_mesh* m, const Level& F, const Level& C, int dtype, const void* ec, void* xf,
                       hipStream_t s) {
  const int nwg = transfer_blocks((int)F.psegs.size());
  if (nwg == 0) return MF_OK;
  if (dtype == MF_F64) run_transfer<double>(false, m->dim, single(prolong_args<double>(F, C, ec, xf), nwg), s);
  else run_transfer<float>(false, m->dim, single(prolong_args<float>(F, C, ec, xf), nwg), s);
  return check_launch();
}

namespace {
template <typename T>
void run_jacobi0(int dim, int part, const Launch<Jacobi0Args<T>>& l, hipStream_t s) {
  if (part == 0) hipLaunchKernelGGL((jacobi0_stream_kernel<T>), dim3(l.nwg), dim3(kWG), 0, s, l);
  else if (dim == 2) hipLaunchKernelGGL((jacobi0_fix_kernel<T, 2>), dim3(l.nwg), dim3(kWG), 0, s, l);
  else hipLaunchKernelGGL((jacobi0_fix_kernel<T, 3>), dim3(l.nwg), dim3(kWG), 0, s, l);
}

template <typename T>
void jacobi0_both(int dim, const Jacobi0Args<T>& a, hipStream_t s) {
  if (const int n = jacobi0_stream_blocks(a)) run_jacobi0<T>(dim, 0, single(a, n), s);
  if (const int n = jacobi0_fix_blocks(a)) run_jacobi0<T>(dim, 1, single(a, n), s);
}
}  // namespace

int launch_jacobi0(const mf_mesh* m, const Level& L, int dtype, double omega, const void* b, void* y,
                   hipStream_t s) {
  if (dtype == MF_F64) jacobi0_both<double>(m->dim, jacobi0_args<double>(L, b, y, omega), s);
  else jacobi0_both<float>(m->dim, jacobi0_args<float>(L, b, y, omega), s);
  return check_launch();
}

int launch_coarse_solve(const Level& L, int dtype, const void* b, void* x, hipStream_t s) {
  int rc = launch_fill(dtype, x, 0.0, L.storage, s);
  if (rc) return rc;
  const int nwg = coarse_blocks(L);
  if (nwg == 0) return MF_OK;
  if (dtype == MF_F64)
    hipLaunchKernelGGL((coarse_solve_kernel<double>), dim3(nwg), dim3(kWG), 0, s,
                       single(coarse_args<double>(L, b, x), nwg));
  else
    hipLaunchKernelGGL((coarse_solve_kernel<float>), dim3(nwg), dim3(kWG), 0, s,
                       single(coarse_args<float>(L, b, x), nwg));
  return check_launch();
}

int launch_fill(int dtype, void* x, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const VecArgs a = vec_args(x, nullptr, nullptr, n, v);
  return run_vector<kOpFill>(dtype, single(a, a.nblk), s);
}

int launch_copy(int dtype, void* d, const void* src, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const VecArgs a = vec_args(d, src, nullptr, n, 0.0);
  return run_vector<kOpCopy>(dtype, single(a, a.nblk), s);
}

int launch_axpy(int dtype, void* y, const void* x, double c, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const VecArgs a = vec_args(y, x, nullptr, n, c);
  return run_vector<kOpAxpy>(dtype, single(a, a.nblk), s);
}

int launch_scale_to_f32(const double* r, float* b, const double* res, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const VecArgs a = vec_args(b, r, res, n, 0.0);
  return run_vector<kOpScaleF32>(MF_F64, single(a, a.nblk), s);
}

int launch_axpy_f32(double* x, const float* e, const double* res, int64_t n, hipStream_t s) {
  if (n <= 0) return MF_OK;
  const VecArgs a = vec_args(x, e, res, n, 0.0);
  return run_vector<kOpAxpyF32>(MF_F64, single(a, a.nblk), s);
}

namespace {
template <int KIND>
void run_pcg_point(int dim, int dtype, const Launch<PcgArgs>& l, hipStream_t s) {
  (void)dim;
  if (dtype == MF_F32) hipLaunchKernelGGL((pcg_lin_kernel<KIND, float>), dim3(l.nwg), dim3(256), 0, s, l);
  else hipLaunchKernelGGL((pcg_lin_kernel<KIND, double>), dim3(l.nwg), dim3(256), 0, s, l);
}
}  // namespace

int launch_pcg_zdot(const mf_mesh* m, const Level& L, int edtype, const double* r, const void* e, double* z,
                    const double* res, double* part, hipStream_t s, int sslot) {
  const int nwg = pcg_blocks(L);
  if (nwg == 0) return MF_OK;
  PcgArgs a = pcg_args(L, nullptr, (double*)r, nullptr, nullptr, e, z, res, part);
  a.sslot = sslot;
  run_pcg_point<kOpPcgZDot>(m->dim, edtype, single(a, nwg), s);
  return check_launch();
}

int launch_pcg_update(const mf_mesh* m, const Level& L, double* x, double* r, double* p, const double* q,
                      const double* res, double* part, hipStream_t s, float* r32, double* sout) {
  const int nwg = pcg_blocks(L);
  if (nwg == 0) return MF_OK;
  if ((r32 == nullptr) != (sout == nullptr)) return set_error(MF_EINVAL, "pcg update: r32 and sout go together");
  PcgArgs a = pcg_args(L, x, r, p, q, nullptr, nullptr, res, part);
  a.r32 = r32;
  a.sout = sout;
  run_pcg_point<kOpPcgUpdate>(m->dim, MF_F64, single(a, nwg), s);
  return check_launch();
}

namespace {
// MINRES's three-term recurrences: y = a y + b x1 + c x2 (x2 may be null),
// grid-stride; with part, each block leaves the maximum of |y| over its
// entries at part[nblk + block] and 0 at part[block] (the layout
// launch_reduce takes).
struct Lin3Args {
  double* y;
  const double* x1;
  const double* x2;
  double a, b, c;
  int64_t n;
  double* part;
  int nblk;
};

__global__ __launch_bounds__(256) void lin3_kernel(const Lin3Args a) {
  const int64_t stride = (int64_t)a.nblk * 256;
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < a.n; i += stride) {
    double v = a.b * a.x1[i];
    if (a.x2) v = fma(a.c, a.x2[i], v);
    v = fma(a.a, a.y[i], v);
    a.y[i] = v;
    mx = fmax(mx, fabs(v));
  }
  if (!a.part) return;
  mx = wmax(mx);
  __shared__ double s_mx[4];
  if ((threadIdx.x & (kWave - 1)) == 0) s_mx[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    a.part[blockIdx.x] = 0.0;
    a.part[a.nblk + blockIdx.x] = fmax(fmax(s_mx[0], s_mx[1]), fmax(s_mx[2], s_mx[3]));
  }
}
}  // namespace

int launch_lin3(double* y, const double* x1, const double* x2, double a, double b, double c, int64_t n, double* part,
                int nblk, hipStream_t s) {
  if (n <= 0) return MF_OK;
  if (nblk < 1) return set_error(MF_EINVAL, "lin3: no blocks");
  const Lin3Args la{y, x1, x2, a, b, c, n, part, nblk};
  hipLaunchKernelGGL(lin3_kernel, dim3(nblk), dim3(256), 0, s, la);
  return check_launch();
}

int launch_pcg_dir(double* p, const void* z, const double* res, int64_t n, hipStream_t s, int zdtype, int sslot) {
  if (n <= 0) return MF_OK;
  VecArgs a = vec_args(p, z, res, n, 0.0);
  a.sslot = sslot;
  if (zdtype == MF_F32) hipLaunchKernelGGL(pcg_dir_kernel<float>, dim3(a.nblk), dim3(256), 0, s, single(a, a.nblk));
  else hipLaunchKernelGGL(pcg_dir_kernel<double>, dim3(a.nblk), dim3(256), 0, s, single(a, a.nblk));
  return check_launch();
}

int launch_vector_batch(const BatchOp& op, const char* table, hipStream_t s) {
  if (op.nwg <= 0) return MF_OK;
  switch (op.kind) {
    case kOpRestrict:
    case kOpProlong:
      if (op.dtype == MF_F64) run_transfer<double>(op.kind == kOpRestrict, op.dim, batched<TransferArgs<double>>(op, table), s);
      else run_transfer<float>(op.kind == kOpRestrict, op.dim, batched<TransferArgs<float>>(op, table), s);
      return check_launch();
    case kOpCoarse:
      if (op.dtype == MF_F64)
        hipLaunchKernelGGL((coarse_solve_kernel<double>), dim3(op.nwg), dim3(kWG), 0, s,
                           batched<CoarseArgs<double>>(op, table));
      else
        hipLaunchKernelGGL((coarse_solve_kernel<float>), dim3(op.nwg), dim3(kWG), 0, s,
                           batched<CoarseArgs<float>>(op, table));
      return check_launch();
    case kOpFill: return run_vector<kOpFill>(op.dtype, batched<VecArgs>(op, table), s);
    case kOpCopy: return run_vector<kOpCopy>(op.dtype, batched<VecArgs>(op, table), s);
    case kOpAxpy: return run_vector<kOpAxpy>(op.dtype, batched<VecArgs>(op, table), s);
    case kOpScaleF32: return run_vector<kOpScaleF32>(MF_F64, batched<VecArgs>(op, table), s);
    case kOpAxpyF32: return run_vector<kOpAxpyF32>(MF_F64, batched<VecArgs>(op, table), s);
    case kOpPcgZDot: run_pcg_point<kOpPcgZDot>(op.dim, op.dtype, batched<PcgArgs>(op, table), s); return check_launch();
    case kOpPcgUpdate: run_pcg_point<kOpPcgUpdate>(op.dim, MF_F64, batched<PcgArgs>(op, table), s); return check_launch();
    case kOpPcgDir:
      if (op.dtype == MF_F32)
        hipLaunchKernelGGL(pcg_dir_kernel<float>, dim3(op.nwg), dim3(256), 0, s, batched<VecArgs>(op, table));
      else
        hipLaunchKernelGGL(pcg_dir_kernel<double>, dim3(op.nwg), dim3(256), 0, s, batched<VecArgs>(op, table));
      return check_launch();
    case kOpTail: return launch_tail_batch(op, table, s);
    case kOpJacobi0:
      if (op.dtype == MF_F64) run_jacobi0<double>(op.dim, op.mode, batched<Jacobi0Args<double>>(op, table), s);
      else run_jacobi0<float>(op.dim, op.mode, batched<Jacobi0Args<float>>(op, table), s);
      return check_launch();
    default: return set_error(MF_EINVAL, "unknown batch op");
  }
}

}  // namespace mf
