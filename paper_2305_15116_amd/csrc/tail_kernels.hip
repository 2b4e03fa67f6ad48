// The bottom of a V-cycle in one workgroup (gfx950).
//
// Below a few thousand points per level, every step of the cycle (stencil
// pass, exchange, transfer, fill, coarse solve) takes about the same time
// whatever its size: a chain of dependent loads plus the launch, about a
// dozen launches per level and cycle.  vcycle_tail_kernel runs the coarse
// solve and the levels just above it (kargs.hpp: kTailLevels,
// kTailMaxPoints) with one workgroup of 16 waves, a barrier between steps,
// and the data in that CU's caches.  The steps and their order are those of
// the multi-launch cycle (pre-smoothing from the zero iterate, residual,
// restriction and its exchange, recursion, prolongation, post-smoothing),
// and every point's arithmetic is the same as in the stencil, exchange and
// transfer kernels: stencil rows are the partial-stencil sum over the 7 / 15
// offsets in table order, which for interior points is the walk's FMA chain,
// so results match the multi-launch cycle up to the sign of zero sums.
//
// One workgroup per request: a batched launch gives each member its own.

#include <hip/hip_runtime.h>

#include "launch.hpp"
#include "rows.hpp"

namespace mf {

namespace {

constexpr int kTailWaves = kTailWG / kWave;

int check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

template <typename T>
__device__ __forceinline__ WTab<T> wtab_of(const MacroDev& M) {
  if constexpr (sizeof(T) == 8) return const_cast<WTab<T>>(M.wm);
  else return const_cast<WTab<T>>(M.wmf);
}

// Every storage point of a level, packed: thread t takes points t,
// t + kTailWG, ... and decodes each storage index into its macro and lattice
// point (all macros of a level have the same side N and point count).  The
// level's row segments would leave most lanes idle in 3D, where rows of
// small levels are a few points long.
template <int DIM, class Fn>
__device__ __forceinline__ void for_points(int N, int nmac, Fn&& fn) {
  const int P = (int)macro_points(DIM, N);
  const int n = P * nmac;
  for (int i = (int)threadIdx.x; i < n; i += kTailWG) {
    const int m = i / P;
    int r = i - m * P;
    int z = 0, S = N;
    if (DIM == 3) {
      // slice z holds (S + 1)(S + 2) / 2 points, S = N - z
      for (int sz = (S + 1) * (S + 2) / 2; r >= sz; sz = (S + 1) * (S + 2) / 2) {
        r -= sz;
        --S;
        ++z;
      }
    }
    int x, y = 0;
    if (DIM == 3) {
      slice_xy3(S, r, x, y);
    } else {
      for (int len = S + 1; r >= len; --len) {  // row y of the slice holds S + 1 - y points
        r -= len;
        ++y;
      }
      x = r;
    }
    fn(m, x, y, z);
  }
}

// One stencil pass of mode MODE over every point of the level: interior,
// Dirichlet and unshared rows finished, shared rows left as partial rows.
template <typename T, int DIM, int MODE>
__device__ __forceinline__ void tail_stencil(const TailLevel<T>& F, const T* X, T* Y, const T* B, T omega) {
  constexpr StencilTable ST = stencil_table(DIM);
  for_points<DIM>(F.N, F.nmac, [&](int m, int x, int y, int z) {
    const MacroDev& M = F.md[m];
    const int N = F.N;
    const int64_t i = M.base + lidx<DIM>(N, x, y, z);
    int off[15];
    if constexpr (DIM == 3) nbr_offsets3(N, y, z, off);
    T v[ST.n];
#pragma unroll
    for (int o = 0; o < ST.n; ++o) {
      const int nx = x + ST.off[o][0], ny = y + ST.off[o][1], nz = z + ST.off[o][2];
      const bool in = nx >= 0 && ny >= 0 && nz >= 0 && nx + ny + nz <= N;
      // neighbours outside the macro read the point itself (a valid index);
      // partial_sum drops them
      v[o] = X[in ? (DIM == 3 ? i + off[o] : M.base + lidx<DIM>(N, nx, ny, nz)) : i];
    }
    const int mask = support_mask(DIM, N, x, y, z);
    const WTab<T> W = wtab_of<T>(M);
    const T acc = partial_sum<T, DIM>(W, mask, N, x, y, z, v);
    double ss = 0.0, mx = 0.0;
    finish<T, DIM, MODE>(M, W, mask, acc, v[ST.centre], MODE != kApply ? B[i] : T(0), omega, Y + i, ss, mx);
  });
}

// The exchange of that pass: shared non-Dirichlet DoFs, one per thread.
template <typename T, int DIM, int MODE>
__device__ __forceinline__ void tail_exchange(const TailLevel<T>& F, const T* X, T* Y, const T* B, T omega) {
  GroupArgs<T> g{};
  g.ngroups = F.nx;
  g.gptr = F.xptr;
  g.copies = F.xcopies;
  g.cidx = F.xcidx;
  g.ginv = F.xinv;
  g.ginvf = F.xinvf;
  g.md = F.md;
  g.X = X;
  g.Y = Y;
  g.B = B;
  g.omega = omega;
  for (int k = (int)threadIdx.x; k < F.nx; k += kTailWG) {
    int64_t i0;
    exchange_row<T, DIM, MODE>(g, k, i0);
  }
}

template <typename T, int DIM, int MODE>
__device__ __forceinline__ void tail_pass(const TailLevel<T>& F, const T* X, T* Y, T omega) {
  tail_stencil<T, DIM, MODE>(F, X, Y, F.b, omega);
  __syncthreads();
  tail_exchange<T, DIM, MODE>(F, X, Y, F.b, omega);
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void tail_fill(T* x, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += kTailWG) x[i] = T(0);
}

// `sweeps` Jacobi sweeps ping-ponging x <-> t, as jacobi_sweeps does; from
// zero, as jacobi_sweeps_from_zero (first sweep omega D^-1 b into t).
template <typename T, int DIM>
__device__ __forceinline__ void tail_jacobi(const TailLevel<T>& F, int sweeps, T omega, bool from_zero) {
  if (from_zero && sweeps == 0) {
    tail_fill(F.x, F.storage);
    __syncthreads();
    return;
  }
  T* cur = F.x;
  T* oth = F.t;
  int i = 0;
  if (from_zero) {
    Jacobi0Args<T> ja{};
    ja.ngroups = F.nx;
    ja.gptr = F.xptr;
    ja.copies = F.xcopies;
    ja.gidx = F.xcidx;
    ja.ginv = F.xinv;
    ja.ginvf = F.xinvf;
    ja.md = F.md;
    ja.B = F.b;
    ja.Y = F.t;
    ja.omega = omega;
    for_points<DIM>(F.N, F.nmac, [&](int m, int x, int y, int z) { jacobi0_point<T, DIM>(ja, m, x, y, z); });
    for (int g = (int)threadIdx.x; g < F.nx; g += kTailWG) jacobi0_group<T, DIM>(ja, g);
    __syncthreads();
    cur = F.t;
    oth = F.x;
    i = 1;
  }
  for (; i < sweeps; ++i) {
    tail_pass<T, DIM, kJacobi>(F, cur, oth, omega);
    T* s = cur;
    cur = oth;
    oth = s;
  }
  if (cur != F.x) {
    for (int64_t k = threadIdx.x; k < F.storage; k += kTailWG) F.x[k] = cur[k];
    __syncthreads();
  }
}

// The request's record, read in place (constant address space: scalar
// loads) rather than copied, so that the per-level records indexed by a
// loop counter need no private memory.
template <class A>
__device__ __forceinline__ auto resolve_ref(const Launch<A>& L, int g) {
#if defined(__HIP_DEVICE_COMPILE__)
  if (L.nseg == 0) return as_const(&L.one);
  return as_const(L.many) + find_seg_c(L.wg0, L.nseg, g);
#else
  (void)g;
  return L.nseg == 0 ? &L.one : L.many;  // the host pass only type-checks device code
#endif
}

template <typename T, int DIM>
__global__ __launch_bounds__(kTailWG) void vcycle_tail_kernel(const Launch<TailArgs<T>> L) {
  extern __shared__ __align__(16) unsigned char tail_lds[];
  const auto* a = resolve_ref(L, (int)blockIdx.x);
  const int nlev = a->nlev, pre = a->pre, post = a->post;
  const T omega = a->omega;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int lane = (int)threadIdx.x & (kWave - 1);
  // Level k's record; with a->lds its b, x and t live in LDS (the kernel's
  // steps are chains of dependent loads, so their latency sets its time):
  // only the top level's b comes in from global memory and its x goes out.
  const bool lds = a->lds > 0;
  auto lvl = [&](int k) {
    TailLevel<T> v = a->lv[k];
    if (lds) {
      int64_t off = 0;
      for (int j = 0; j < k; ++j) off += 3 * tail_lds_vec(a->lv[j].storage, (int)sizeof(T));
      const int64_t sz = tail_lds_vec(v.storage, (int)sizeof(T));
      v.b = (T*)(tail_lds + off);
      v.x = (T*)(tail_lds + off + sz);
      v.t = (T*)(tail_lds + off + 2 * sz);
    }
    return v;
  };
  if (lds) {
    const TailLevel<T> G = a->lv[nlev - 1], S = lvl(nlev - 1);
    for (int64_t i = threadIdx.x; i < G.storage; i += kTailWG) S.b[i] = G.b[i];
    __syncthreads();
  }
  // descent: levels lc + nlev - 1 .. lc + 1 (restriction: one coarse point per thread)
  for (int k = nlev - 1; k >= 1; --k) {
    const TailLevel<T> F = lvl(k);
    const TailLevel<T> C = lvl(k - 1);
    tail_jacobi<T, DIM>(F, pre, omega, true);
    tail_pass<T, DIM, kResidual>(F, F.x, F.t, T(0));
    const TransferArgs<T> ta{nullptr, 0, 0, C.md, F.md, F.t, C.b};  // points come from for_points
    for_points<DIM>(C.N, C.nmac, [&](int m, int x, int y, int z) { restrict_point<T, DIM>(ta, m, x, y, z); });
    __syncthreads();
    GroupArgs<T> ga{};
    ga.ngroups = C.ng;
    ga.gptr = C.gptr;
    ga.copies = C.copies;
    ga.cidx = C.gcidx;
    ga.gflag = C.gflag;
    ga.md = C.md;
    ga.X = C.b;
    ga.Y = C.b;
    for (int g = (int)threadIdx.x; g < C.ng; g += kTailWG) iface_sum_row<T, DIM>(ga, g);
    __syncthreads();
  }
  // coarse level: x = 0, then the dense solve on its unknowns (a wave each)
  {
    CoarseArgs<T> cs = a->coarse;
    if (lds) {
      const TailLevel<T> C0 = lvl(0);
      cs.B = C0.b;
      cs.X = C0.x;
    }
    tail_fill(cs.X, a->lv[0].storage);
    __syncthreads();
    for (int i = wave; i < cs.n; i += kTailWaves) coarse_row<T>(cs, i, lane);
    __syncthreads();
  }
  // ascent: levels lc + 1 .. lc + nlev - 1
  for (int k = 1; k < nlev; ++k) {
    const TailLevel<T> F = lvl(k);
    const TailLevel<T> C = lvl(k - 1);
    const TransferArgs<T> ta{nullptr, 0, 0, C.md, F.md, C.x, F.x};
    for_points<DIM>(F.N, F.nmac, [&](int m, int x, int y, int z) { prolong_point<T, DIM>(ta, m, x, y, z); });
    __syncthreads();
    tail_jacobi<T, DIM>(F, post, omega, false);
  }
  if (lds) {
    const TailLevel<T> G = a->lv[nlev - 1], S = lvl(nlev - 1);
    for (int64_t i = threadIdx.x; i < G.storage; i += kTailWG) G.x[i] = S.x[i];
  }
}

template <typename T>
void run_tail(int dim, const Launch<TailArgs<T>>& l, int lds, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL((vcycle_tail_kernel<T, 2>), dim3(l.nwg), dim3(kTailWG), lds, s, l);
  else hipLaunchKernelGGL((vcycle_tail_kernel<T, 3>), dim3(l.nwg), dim3(kTailWG), lds, s, l);
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

}  // namespace

template <typename T>
TailArgs<T> tail_args(const mf_mesh* m, int lc, int nlev, int pre, int post, double omega,
                      const std::vector<void*>& b, const std::vector<void*>& x, const std::vector<void*>& t) {
  TailArgs<T> a{};
  a.nlev = nlev;
  a.pre = pre;
  a.post = post;
  a.omega = (T)omega;
  a.coarse = coarse_args<T>(m->levels[lc], b[lc], x[lc]);
  for (int k = 0; k < nlev; ++k) a.lv[k] = tail_level<T>(m->levels[lc + k], b[lc + k], x[lc + k], t[lc + k]);
  int64_t lds = 0;
  for (int k = 0; k < nlev; ++k) lds += 3 * tail_lds_vec(a.lv[k].storage, (int)sizeof(T));
  a.lds = lds <= kTailLdsMax ? (int)lds : 0;
  return a;
}
template TailArgs<double> tail_args<double>(const mf_mesh*, int, int, int, int, double, const std::vector<void*>&,
                                            const std::vector<void*>&, const std::vector<void*>&);
template TailArgs<float> tail_args<float>(const mf_mesh*, int, int, int, int, double, const std::vector<void*>&,
                                          const std::vector<void*>&, const std::vector<void*>&);

int launch_vcycle_tail(const mf_mesh* m, int lc, int nlev, int dtype, int pre, int post, double omega,
                       const std::vector<void*>& b, const std::vector<void*>& x, const std::vector<void*>& t,
                       hipStream_t s) {
  if (nlev < 1 || nlev > kTailLevels) return set_error(MF_EINVAL, "tail levels out of range");
  if (dtype == MF_F64) {
    const TailArgs<double> a = tail_args<double>(m, lc, nlev, pre, post, omega, b, x, t);
    run_tail<double>(m->dim, single(a, 1), a.lds, s);
  } else {
    const TailArgs<float> a = tail_args<float>(m, lc, nlev, pre, post, omega, b, x, t);
    run_tail<float>(m->dim, single(a, 1), a.lds, s);
  }
  return check_launch();
}

int launch_tail_batch(const BatchOp& op, const char* table, hipStream_t s) {
  if (op.nwg <= 0) return MF_OK;
  // op.variant: the largest LDS size of the members (each member's own record says whether it uses LDS)
  if (op.dtype == MF_F64) run_tail<double>(op.dim, batched<TailArgs<double>>(op, table), op.variant, s);
  else run_tail<float>(op.dim, batched<TailArgs<float>>(op, table), op.variant, s);
  return check_launch();
}

}  // namespace mf
