// Continuous batching of multigrid solves.
//
// A batch holds many independent solve requests (different meshes,
// dimensions and levels).  batch_step advances every member by one outer
// iteration of the solver of vcycle_solve — V-cycle correction, FP64
// residual and its norm — with each kernel of that iteration launched ONCE
// for all members that need it: the launch's workgroups are dealt out to the
// members (kargs.hpp), so small requests share launches instead of each
// paying its own launch latency.  The V-cycles of members of different depth
// are aligned at the coarse level: at every stage of the cycle, all members
// that take part are at the same distance from their coarse level (and, for
// the usual coarse level 2, at the same level).  Each member's arithmetic and
// its order are those of its own vcycle_solve, so results are bitwise equal
// to solving it alone.
//
// The launch sequence of a step (the plan) depends only on the members and
// their state; it is rebuilt when members join, leave or finish their first
// step, and its argument tables are uploaded to the device in one copy.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "launch.hpp"
#include "mesh.hpp"
#include "mf_stencil.h"
#include "solver.hpp"

using namespace mf;

namespace {

// kVerify (CG modes): the recurrence met rtol in the last step; this step
// recomputes the true FP64 residual b - A x and performs no iteration.
enum MemberState { kNew = 0, kRunning = 1, kVerify = 2 };

struct Member {
  int64_t tag = 0;
  const mf_mesh* m = nullptr;
  int level = 0, lc = 0;
  int tail = 0;  // levels lc .. lc + tail - 1 run in one workgroup launch (tail_levels)
  const double* b = nullptr;
  double* x = nullptr;
  Workspace w;
  double rtol = 0.0;
  int state = kNew;
  bool correct = false;  // this step starts with a V-cycle correction
  int iters = 0;
  double bnorm = 0.0, rel = 0.0;
  std::chrono::steady_clock::time_point t0;
};

// Host-side recorder of one plan: ops plus their argument tables.
struct PlanBuilder {
  std::vector<char> buf;
  std::vector<BatchOp> ops;

  void align(size_t a) {
    const size_t n = (buf.size() + a - 1) / a * a;
    buf.resize(n, 0);
  }
  // items: (argument record, workgroups); members with no workgroups are dropped.
  template <class A>
  void add(int kind, int dtype, int dim, int mode, const std::vector<std::pair<A, int>>& items, int variant = 0) {
    std::vector<const std::pair<A, int>*> live;
    for (const auto& it : items)
      if (it.second > 0) live.push_back(&it);
    if (live.empty()) return;
    BatchOp op{};
    op.kind = kind;
    op.dtype = dtype;
    op.dim = dim;
    op.mode = mode;
    op.variant = variant;
    op.nseg = (int)live.size();
    align(64);
    op.args_off = (int64_t)buf.size();
    buf.resize(buf.size() + sizeof(A) * live.size());
    for (size_t i = 0; i < live.size(); ++i) std::memcpy(buf.data() + op.args_off + i * sizeof(A), &live[i]->first, sizeof(A));
    align(16);
    op.wg0_off = (int64_t)buf.size();
    buf.resize(buf.size() + sizeof(int32_t) * (live.size() + 1));
    int32_t* wg0 = (int32_t*)(buf.data() + op.wg0_off);
    int64_t tot = 0;
    for (size_t i = 0; i < live.size(); ++i) {
      wg0[i] = (int32_t)tot;
      tot += live[i]->second;
    }
    wg0[live.size()] = (int32_t)tot;
    op.nwg = (int)tot;
    ops.push_back(op);
  }
};

}  // namespace

struct mf_batch {
  mf_solve_opts o{};
  int capacity = 0;
  int device = 0;
  std::vector<Member> mem;
  bool dirty = true;
  PlanBuilder plan;
  char* dtab = nullptr;  // device copy of the plan's tables
  size_t dcap = 0;
  char* htab = nullptr;  // pinned staging of the tables
  size_t hcap = 0;
  double* dres = nullptr;  // per member: residual (ss, max), b norm (ss, max)
  double* hres = nullptr;
};

namespace {

const Level& lev(const Member& M, int l) { return M.m->levels[l]; }

// Ops of one stencil pass (interior walk + exchange) over the selected
// members: sel(M) fills level / vectors / part and returns false to skip M.
struct Pass {
  int level;
  const void *x, *b;
  void* y;
  double* part;
};

template <typename T, class Sel>
void stencil_pass(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int dtype, int mode, double omega,
                  Sel sel) {
  // one stencil launch per tile shape (levels differ in it), then one exchange launch
  std::vector<std::pair<StencilArgs<T>, int>> sa[2];
  std::vector<std::pair<GroupArgs<T>, int>> ga;
  for (Member* M : ms) {
    if (M->m->dim != dim) continue;
    Pass p{};
    if (!sel(*M, p)) continue;
    const Level& L = lev(*M, p.level);
    const StencilArgs<T> a = stencil_args<T>(L, p.x, p.y, p.b, omega, p.part);
    sa[dim == 3 && L.pen_z == kPenSeg ? 1 : 0].push_back({a, a.nwg});
    if (!exchange_in_launch(L)) ga.push_back({exchange_args<T>(L, p.x, p.y, p.b, omega, p.part), exchange_blocks(L)});
  }
  P.add(kOpStencil, dtype, dim, mode, sa[0], kPenZ);
  P.add(kOpStencil, dtype, dim, mode, sa[1], kPenSeg);
  P.add(kOpExchange, dtype, dim, mode, ga);
}

template <class Sel>
void stencil_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int dtype, int mode, double omega, Sel sel) {
  if (dtype == MF_F64) stencil_pass<double>(P, ms, dim, dtype, mode, omega, sel);
  else stencil_pass<float>(P, ms, dim, dtype, mode, omega, sel);
}

// Vector op over the selected members: sel(M, args) returns false to skip.
template <class Sel>
void vector_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int kind, int dtype, Sel sel) {
  std::vector<std::pair<VecArgs, int>> va;
  for (Member* M : ms) {
    if (M->m->dim != dim) continue;
    VecArgs a{};
    if (!sel(*M, a)) continue;
    if (a.n <= 0) continue;
    va.push_back({a, a.nblk});
  }
  P.add(kind, dtype, dim, 0, va);
}

// First sweep from a zero iterate: t = omega D^-1 b, as jacobi_sweeps_from_zero.
template <typename T, class LevelOf>
void jacobi0_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, const mf_solve_opts& o, LevelOf lof) {
  std::vector<std::pair<Jacobi0Args<T>, int>> js, jf;
  for (Member* M : ms) {
    if (M->m->dim != dim) continue;
    const int l = lof(*M);
    if (l < 0) continue;
    const Jacobi0Args<T> a = jacobi0_args<T>(lev(*M, l), M->w.b[l], M->w.t[l], o.omega);
    js.push_back({a, jacobi0_stream_blocks(a)});
    jf.push_back({a, jacobi0_fix_blocks(a)});
  }
  P.add(kOpJacobi0, dtype_of<T>(), dim, 0, js);
  P.add(kOpJacobi0, dtype_of<T>(), dim, 1, jf);
}

// Jacobi sweeps at the members' cycle level (ping-pong x <-> t), as
// jacobi_sweeps does, or (from_zero) as jacobi_sweeps_from_zero.
template <class LevelOf>
void jacobi_stage(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int vdt, const mf_solve_opts& o,
                  int sweeps, LevelOf lof, bool from_zero = false) {
  if (from_zero && sweeps == 0) {
    vector_op(P, ms, dim, kOpFill, vdt, [&](const Member& M, VecArgs& a) {
      const int l = lof(M);
      if (l < 0) return false;
      a = vec_args(M.w.x[l], nullptr, nullptr, lev(M, l).storage, 0.0);
      return true;
    });
    return;
  }
  if (from_zero) {
    if (vdt == MF_F64) jacobi0_op<double>(P, ms, dim, o, lof);
    else jacobi0_op<float>(P, ms, dim, o, lof);
  }
  for (int i = from_zero ? 1 : 0; i < sweeps; ++i) {
    stencil_op(P, ms, dim, vdt, kJacobi, o.omega, [&](const Member& M, Pass& p) {
      const int l = lof(M);
      if (l < 0) return false;
      p.level = l;
      p.x = i % 2 == 0 ? M.w.x[l] : M.w.t[l];
      p.y = i % 2 == 0 ? M.w.t[l] : M.w.x[l];
      p.b = M.w.b[l];
      p.part = nullptr;
      return true;
    });
  }
  if (sweeps % 2 == 1)
    vector_op(P, ms, dim, kOpCopy, vdt, [&](const Member& M, VecArgs& a) {
      const int l = lof(M);
      if (l < 0) return false;
      a = vec_args(M.w.x[l], M.w.t[l], nullptr, lev(M, l).storage, 0.0);
      return true;
    });
}

template <typename T>
void transfer_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int dtype, bool restrict_op, int dl) {
  std::vector<std::pair<TransferArgs<T>, int>> ta;
  std::vector<std::pair<GroupArgs<T>, int>> ia;
  for (Member* M : ms) {
    if (M->m->dim != dim || M->level - M->lc < dl || dl < M->tail) continue;
    const int l = M->lc + dl;
    const Level& F = lev(*M, l);
    const Level& C = lev(*M, l - 1);
    if (restrict_op) {
      ta.push_back({restrict_args<T>(F, C, M->w.t[l], M->w.b[l - 1]), transfer_blocks((int)C.psegs.size())});
      ia.push_back({iface_args<T>(C, M->w.b[l - 1], M->w.b[l - 1], nullptr), iface_blocks(C)});
    } else {
      ta.push_back({prolong_args<T>(F, C, M->w.x[l - 1], M->w.x[l]), transfer_blocks((int)F.psegs.size())});
    }
  }
  P.add(restrict_op ? kOpRestrict : kOpProlong, dtype, dim, 0, ta);
  if (restrict_op) P.add(kOpIface, dtype, dim, kExchangeSum, ia);
}

template <typename T>
void coarse_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, int dtype) {
  std::vector<std::pair<CoarseArgs<T>, int>> ca;
  for (Member* M : ms) {
    if (M->m->dim != dim || M->tail > 0) continue;
    const Level& L = lev(*M, M->lc);
    ca.push_back({coarse_args<T>(L, M->w.b[M->lc], M->w.x[M->lc]), coarse_blocks(L)});
  }
  P.add(kOpCoarse, dtype, dim, 0, ca);
}

// The bottom of the cycle of members with a tail: one workgroup each.
template <typename T>
void tail_op(PlanBuilder& P, const std::vector<Member*>& ms, int dim, const mf_solve_opts& o) {
  std::vector<std::pair<TailArgs<T>, int>> ta;
  int lds = 0;  // dynamic LDS of the launch: the largest member's
  for (Member* M : ms) {
    if (M->m->dim != dim || M->tail == 0) continue;
    ta.push_back({tail_args<T>(M->m, M->lc, M->tail, o.pre, o.post, o.omega, M->w.b, M->w.x, M->w.t), 1});
    lds = std::max(lds, ta.back().first.lds);
  }
  P.add(kOpTail, dtype_of<T>(), dim, 0, ta, lds);
}

void reduce_op(PlanBuilder& P, const std::vector<std::pair<ReduceArgs, int>>& ra) { P.add(kOpReduce, MF_F64, 0, 0, ra); }

// The launch sequence of one step for the current members.
void build_plan(mf_batch* B) {
  PlanBuilder& P = B->plan;
  P.buf.clear();
  P.ops.clear();
  const mf_solve_opts& o = B->o;
  const bool f32 = mode_f32(o.mode), pcg = mode_pcg(o.mode);
  const int vdt = f32 ? MF_F32 : MF_F64;
  auto slot = [B](const Member& M) { return B->dres + 4 * (&M - B->mem.data()); };
  std::vector<Member*> all, corr, fresh, verify;
  for (size_t i = 0; i < B->mem.size(); ++i) {
    Member* M = &B->mem[i];
    all.push_back(M);
    if (M->correct) corr.push_back(M);
    if (M->state == kNew) fresh.push_back(M);
    if (M->state == kVerify) verify.push_back(M);
  }
  for (int dim = 2; dim <= 3; ++dim) {
    // ---- V-cycle correction (members with a residual that did not converge)
    bool any = false;
    int dmax = 0;
    for (Member* M : corr)
      if (M->m->dim == dim) {
        any = true;
        dmax = std::max(dmax, M->level - M->lc);
      }
    if (!any) continue;
    if (f32 && !pcg) {
      vector_op(P, corr, dim, kOpScaleF32, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.w.b[M.level], M.w.r64, M.w.result, lev(M, M.level).storage, 0.0);
        return true;
      });
    }
    // descent: stage dl works at level lc + dl of every member deep enough;
    // each level's iterate starts at zero (first sweep from zero)
    for (int dl = dmax; dl >= 1; --dl) {
      auto lof = [dl](const Member& M) { return M.level - M.lc >= dl && dl >= M.tail ? M.lc + dl : -1; };
      jacobi_stage(P, corr, dim, vdt, o, o.pre, lof, true);
      stencil_op(P, corr, dim, vdt, kResidual, 0.0, [&](const Member& M, Pass& p) {
        const int l = lof(M);
        if (l < 0) return false;
        p.level = l;
        p.x = M.w.x[l];
        p.y = M.w.t[l];
        p.b = M.w.b[l];
        p.part = nullptr;
        return true;
      });
      if (vdt == MF_F64) transfer_op<double>(P, corr, dim, vdt, true, dl);
      else transfer_op<float>(P, corr, dim, vdt, true, dl);
    }
    // coarse level, or the one-workgroup tail of members that have one
    vector_op(P, corr, dim, kOpFill, vdt, [](const Member& M, VecArgs& a) {
      if (M.tail > 0) return false;
      a = vec_args(M.w.x[M.lc], nullptr, nullptr, lev(M, M.lc).storage, 0.0);
      return true;
    });
    if (vdt == MF_F64) {
      coarse_op<double>(P, corr, dim, vdt);
      tail_op<double>(P, corr, dim, o);
    } else {
      coarse_op<float>(P, corr, dim, vdt);
      tail_op<float>(P, corr, dim, o);
    }
    // ascent
    for (int dl = 1; dl <= dmax; ++dl) {
      auto lof = [dl](const Member& M) { return M.level - M.lc >= dl && dl >= M.tail ? M.lc + dl : -1; };
      if (vdt == MF_F64) transfer_op<double>(P, corr, dim, vdt, false, dl);
      else transfer_op<float>(P, corr, dim, vdt, false, dl);
      jacobi_stage(P, corr, dim, vdt, o, o.post, lof);
    }
    if (pcg) continue;
    if (f32) {
      vector_op(P, corr, dim, kOpAxpyF32, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.x, M.w.x[M.level], M.w.result, lev(M, M.level).storage, 0.0);
        return true;
      });
    } else {
      vector_op(P, corr, dim, kOpAxpy, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.x, M.w.x[M.level], nullptr, lev(M, M.level).storage, 1.0);
        return true;
      });
    }
  }
  // ---- conjugate-gradient step around the V-cycle (scalars stay on the device)
  if (pcg && !corr.empty()) {
    auto pcg_op = [&](int kind, int dtype, auto make) {
      for (int dim = 2; dim <= 3; ++dim) {
        std::vector<std::pair<PcgArgs, int>> pa;
        for (Member* M : corr)
          if (M->m->dim == dim) pa.push_back({make(*M), pcg_blocks(lev(*M, M->level))});
        P.add(kind, dtype, dim, 0, pa);
      }
    };
    auto reduce_corr = [&](auto make) {
      std::vector<std::pair<ReduceArgs, int>> ra;
      for (Member* M : corr) ra.push_back({make(*M), 1});
      reduce_op(P, ra);
    };
    pcg_op(kOpPcgZDot, vdt, [](const Member& M) {
      PcgArgs a = pcg_args(lev(M, M.level), nullptr, M.w.r64, nullptr, nullptr, M.w.x[M.level], M.w.z64, M.w.result,
                           M.w.part);
      a.sslot = kSlotScale;
      return a;
    });
    reduce_corr([](const Member& M) {
      return ReduceArgs{M.w.part, lev(M, M.level).lin_blocks(), M.w.result + 2, nullptr, 1, 0};
    });
    for (int dim = 2; dim <= 3; ++dim)
      vector_op(P, corr, dim, kOpPcgDir, vdt, [f32](const Member& M, VecArgs& a) {
        a = vec_args(M.w.p64, f32 ? M.w.x[M.level] : (const void*)M.w.z64, M.w.result, lev(M, M.level).storage, 0.0);
        a.sslot = kSlotScale;
        return true;
      });
    for (int dim = 2; dim <= 3; ++dim)
      stencil_op(P, corr, dim, MF_F64, kApplyDot, 0.0, [](const Member& M, Pass& p) {
        p.level = M.level;
        p.x = M.w.p64;
        p.y = M.w.q64;
        p.b = nullptr;
        p.part = M.w.part;
        return true;
      });
    reduce_corr([](const Member& M) {
      return ReduceArgs{M.w.part, stencil_partials(lev(M, M.level), MF_F64), M.w.result + 4, nullptr, 0, 0};
    });
    pcg_op(kOpPcgUpdate, MF_F64, [f32](const Member& M) {
      PcgArgs a = pcg_args(lev(M, M.level), M.x, M.w.r64, M.w.p64, M.w.q64, nullptr, nullptr, M.w.result, M.w.part);
      if (f32) {
        // the next FP32 preconditioner input, as vcycle_solve forms it
        a.r32 = (float*)M.w.b[M.level];
        a.sout = M.w.result + kSlotScale;
      }
      return a;
    });
    reduce_corr([&](const Member& M) {
      return ReduceArgs{M.w.part, lev(M, M.level).lin_blocks(), M.w.result, slot(M), 0, 0};
    });
  }
  // ---- first step of new members: Dirichlet values of x, then ||b||
  for (int dim = 2; dim <= 3; ++dim) {
    std::vector<std::pair<GroupArgs<double>, int>> ia;
    for (Member* M : fresh)
      if (M->m->dim == dim) {
        const Level& L = lev(*M, M->level);
        ia.push_back({iface_args<double>(L, M->x, M->x, M->b), iface_blocks(L)});
      }
    P.add(kOpIface, MF_F64, dim, kDirichletSet, ia);
    stencil_op(P, fresh, dim, MF_F64, kNormB, 0.0, [](const Member& M, Pass& p) {
      p.level = M.level;
      p.x = M.b;
      p.y = nullptr;
      p.b = M.b;
      p.part = M.w.part;
      return true;
    });
  }
  {
    std::vector<std::pair<ReduceArgs, int>> ra;
    for (Member* M : fresh)
      ra.push_back({ReduceArgs{M->w.part, stencil_partials(lev(*M, M->level), MF_F64), M->w.result, slot(*M) + 2, 0, 0}, 1});
    reduce_op(P, ra);
  }
  // ---- FP64 residual and its norm: every member (refinement) or the new ones (PCG)
  const std::vector<Member*>& resid = pcg ? fresh : all;
  for (int dim = 2; dim <= 3; ++dim) {
    if (pcg)
      vector_op(P, fresh, dim, kOpFill, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.w.result + 2, nullptr, nullptr, 6, 0.0);
        return true;
      });
    stencil_op(P, resid, dim, MF_F64, kResidual, 0.0, [](const Member& M, Pass& p) {
      p.level = M.level;
      p.x = M.x;
      p.y = M.w.r64;
      p.b = M.b;
      p.part = M.w.part;
      return true;
    });
  }
  {
    std::vector<std::pair<ReduceArgs, int>> ra;
    for (Member* M : resid)
      ra.push_back({ReduceArgs{M->w.part, stencil_partials(lev(*M, M->level), MF_F64), M->w.result, slot(*M), 0, 0}, 1});
    reduce_op(P, ra);
  }
  // ---- mixed CG: the first FP32 preconditioner input of the new members and
  // its scale (the CG update forms the later ones)
  if (pcg && f32) {
    for (int dim = 2; dim <= 3; ++dim) {
      vector_op(P, fresh, dim, kOpScaleF32, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.w.b[M.level], M.w.r64, M.w.result, lev(M, M.level).storage, 0.0);
        return true;
      });
      vector_op(P, fresh, dim, kOpCopy, MF_F64, [](const Member& M, VecArgs& a) {
        a = vec_args(M.w.result + kSlotScale, M.w.result + 1, nullptr, 1, 0.0);
        return true;
      });
    }
  }
  // ---- CG members whose recurrence met rtol: the true residual, as vcycle_solve
  // recomputes it (into q and result[6..7], which no recurrence reads)
  if (verify.empty()) return;
  for (int dim = 2; dim <= 3; ++dim)
    stencil_op(P, verify, dim, MF_F64, kResidual, 0.0, [](const Member& M, Pass& p) {
      p.level = M.level;
      p.x = M.x;
      p.y = M.w.q64;
      p.b = M.b;
      p.part = M.w.part;
      return true;
    });
  std::vector<std::pair<ReduceArgs, int>> ra;
  for (Member* M : verify)
    ra.push_back(
        {ReduceArgs{M->w.part, stencil_partials(lev(*M, M->level), MF_F64), M->w.result + 6, slot(*M), 0, 0}, 1});
  reduce_op(P, ra);
}

int upload_plan(mf_batch* B, hipStream_t s) {
  const size_t n = B->plan.buf.size();
  if (n == 0) return MF_OK;
  hipError_t e = hipSuccess;
  if (n > B->dcap) {
    // the previous step ended with a stream synchronisation: no kernel reads the old table
    if (B->dtab) (void)hipFree(B->dtab);
    B->dtab = nullptr;
    B->dcap = 0;
    const size_t cap = std::max<size_t>(n * 2, 1 << 20);
    e = hipMalloc((void**)&B->dtab, cap);
    if (e != hipSuccess) return set_error(MF_ENOMEM, std::string("batch table: ") + hipGetErrorString(e));
    B->dcap = cap;
  }
  if (n > B->hcap) {
    if (B->htab) (void)hipHostFree(B->htab);
    B->htab = nullptr;
    B->hcap = 0;
    const size_t cap = std::max<size_t>(n * 2, 1 << 20);
    e = hipHostMalloc((void**)&B->htab, cap, hipHostMallocDefault);
    if (e != hipSuccess) return set_error(MF_ENOMEM, std::string("batch staging: ") + hipGetErrorString(e));
    B->hcap = cap;
  }
  std::memcpy(B->htab, B->plan.buf.data(), n);
  e = hipMemcpyAsync(B->dtab, B->htab, n, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

}  // namespace

extern "C" {

int batch_create(const mf_solve_opts* opts, int capacity, mf_batch** out) {
  if (!out) return set_error(MF_EINVAL, "out is NULL");
  *out = nullptr;
  if (capacity < 1 || capacity > 4096) return set_error(MF_EINVAL, "capacity must be in [1, 4096]");
  mf_solve_opts o = {1, 2, 2, -1, 50, 2.0 / 3.0, 1e-8};
  if (opts) o = *opts;
  if (o.mode < 0 || o.mode > 3) return set_error(MF_EINVAL, "batched solves take mode 0, 1, 2 or 3");
  if (mode_pcg(o.mode) && o.pre != o.post)
    return set_error(MF_EINVAL, "conjugate gradients need a symmetric V-cycle (pre == post)");
  if (o.pre < 0 || o.post < 0 || o.max_iter < 0) return set_error(MF_EINVAL, "bad solver options");
  mf_batch* B = nullptr;
  try {
    B = new mf_batch;
  } catch (const std::bad_alloc&) {
    return set_error(MF_ENOMEM, "host allocation failed");
  }
  B->o = o;
  B->capacity = capacity;
  (void)hipGetDevice(&B->device);
  hipError_t e = hipMalloc((void**)&B->dres, sizeof(double) * 4 * capacity);
  if (e == hipSuccess) e = hipHostMalloc((void**)&B->hres, sizeof(double) * 4 * capacity, hipHostMallocDefault);
  if (e != hipSuccess) {
    if (B->dres) (void)hipFree(B->dres);
    delete B;
    return set_error(MF_ENOMEM, std::string("batch buffers: ") + hipGetErrorString(e));
  }
  try {
    B->mem.reserve(capacity);
  } catch (const std::bad_alloc&) {
    (void)hipFree(B->dres);
    (void)hipHostFree(B->hres);
    delete B;
    return set_error(MF_ENOMEM, "host allocation failed");
  }
  *out = B;
  return MF_OK;
}

int batch_destroy(mf_batch* B) {
  if (!B) return MF_OK;
  if (B->dtab) (void)hipFree(B->dtab);
  if (B->htab) (void)hipHostFree(B->htab);
  if (B->dres) (void)hipFree(B->dres);
  if (B->hres) (void)hipHostFree(B->hres);
  delete B;
  return MF_OK;
}

int batch_size(const mf_batch* B, int* n) {
  if (!B || !n) return set_error(MF_EINVAL, "NULL argument");
  *n = (int)B->mem.size();
  return MF_OK;
}

int batch_add(mf_batch* B, const mf_mesh* m, int level, const double* b, double* x, void* workspace, double rtol,
              int64_t tag) {
  if (!B || !m) return set_error(MF_EINVAL, "NULL batch or mesh");
  if (level < 0 || level > m->max_level) return set_error(MF_EINVAL, "level outside [0, max_level]");
  if (m->host_only) return set_error(MF_ENOTSUP, "mesh was created host-only");
  if (!b || !x || !workspace) return set_error(MF_EINVAL, "NULL vector or workspace");
  if (!(rtol >= 0.0)) return set_error(MF_EINVAL, "rtol must be >= 0");
  if ((int)B->mem.size() >= B->capacity) return set_error(MF_ENOMEM, "batch is full");
  for (const Member& M : B->mem)
    if (M.tag == tag) return set_error(MF_EINVAL, "tag already in the batch");
  const int lc = (B->o.coarse_level >= 0 && B->o.coarse_level <= level) ? B->o.coarse_level : default_coarse(level);
  int rc;
  {
    std::lock_guard<std::mutex> lock(const_cast<mf_mesh*>(m)->norm_mutex);
    rc = build_coarse_solver(const_cast<mf_mesh*>(m), lc);
  }
  if (rc) return rc;
  Member M;
  M.tag = tag;
  M.m = m;
  M.level = level;
  M.lc = lc;
  M.tail = tail_levels(m, level, lc);
  M.b = b;
  M.x = x;
  M.w = carve(m, level, B->o.mode, 0, (char*)workspace);
  M.rtol = rtol;
  M.t0 = std::chrono::steady_clock::now();
  B->mem.push_back(std::move(M));
  B->dirty = true;
  return MF_OK;
}

int batch_step(mf_batch* B, void* stream, int64_t* done_tags, int* done_status, mf_solve_info* done_info,
               int* n_done) {
  if (!B || !n_done) return set_error(MF_EINVAL, "NULL batch or n_done");
  *n_done = 0;
  if (B->mem.empty()) return MF_OK;
  if (!done_tags || !done_status) return set_error(MF_EINVAL, "NULL output arrays");
  hipStream_t s = (hipStream_t)stream;
  for (Member& M : B->mem)
    if (M.correct) ++M.iters;
  if (B->dirty) {
    build_plan(B);
    int rc = upload_plan(B, s);
    if (rc) return rc;
    B->dirty = false;
  }
  for (const BatchOp& op : B->plan.ops) {
    const int rc = (op.kind <= kOpReduce) ? launch_stencil_batch(op, B->dtab, s) : launch_vector_batch(op, B->dtab, s);
    if (rc) return rc;
  }
  hipError_t e = hipMemcpyAsync(B->hres, B->dres, sizeof(double) * 4 * B->mem.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  // decide, per member, exactly as vcycle_solve does
  std::vector<Member> keep;
  keep.reserve(B->mem.size());
  bool changed = false;
  const auto now = std::chrono::steady_clock::now();
  for (size_t i = 0; i < B->mem.size(); ++i) {
    Member& M = B->mem[i];
    const double* r = B->hres + 4 * i;
    bool running = true;
    int status = MF_OK;
    if (M.state == kNew) {
      if (!std::isfinite(r[2])) {
        status = MF_ENUMERIC;
        running = false;
      }
      M.bnorm = std::sqrt(r[2]);
      M.state = kRunning;
      changed = true;
    }
    bool verify_next = false;
    if (running) {
      if (!std::isfinite(r[0]) || !std::isfinite(r[1])) {
        status = MF_ENUMERIC;
        running = false;
      } else {
        const bool verified = M.state == kVerify;  // r holds the true residual
        M.rel = M.bnorm > 0.0 ? std::sqrt(r[0]) / M.bnorm : std::sqrt(r[0]);
        if (M.rel <= M.rtol || r[1] == 0.0) {
          if (mode_pcg(B->o.mode) && M.iters > 0 && !verified) {
            verify_next = true;  // the recurrence says converged: confirm on b - A x first
          } else {
            status = MF_OK;
            running = false;
          }
        }
        if (running && !verify_next && M.iters >= B->o.max_iter) {
          status = MF_NOT_CONVERGED;
          running = false;
        }
        if (verified) {
          M.state = kRunning;
          changed = true;
        }
      }
    }
    if (running) {
      if (verify_next) {
        M.state = kVerify;
        M.correct = false;
        changed = true;
      } else {
        if (!M.correct) changed = true;
        M.correct = true;
      }
      keep.push_back(std::move(M));
      continue;
    }
    const int k = (*n_done)++;
    done_tags[k] = M.tag;
    done_status[k] = status;
    if (done_info) {
      done_info[k].iters = M.iters;
      done_info[k].rel_res = M.rel;
      done_info[k].seconds = std::chrono::duration<double>(now - M.t0).count();
    }
    changed = true;
  }
  B->mem.swap(keep);
  if (changed) B->dirty = true;
  return MF_OK;
}

}  // extern "C"
