// extern "C" entry points (include/mf_stencil.h) and the multigrid solver.
//
// apply_stencil is the paper's "apply" (an operator applied to a function,
// Performance Modeling section): the interior kernel covers every interior
// row of every macro with its constant stencil, then the interface kernel
// completes the rows of macro-boundary DoFs, which the paper leaves to
// interface primitives rather than to the macro kernels (same section,
// experiment description).  smooth and residual reuse the same kernels in
// their fused Jacobi and residual modes; vcycle_solve runs geometric
// multigrid over the refinement levels (Intro: the levels are a natural
// multigrid hierarchy) inside iterative refinement, conjugate gradients or
// MINRES.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "mf_stencil.h"
#include "launch.hpp"
#include "mesh.hpp"
#include "solver.hpp"

using namespace mf;

namespace {

int check_mesh(const mf_mesh* m, int level, bool device) {
  if (!m) return set_error(MF_EINVAL, "mesh is NULL");
  if (level < 0 || level > m->max_level)
    return set_error(MF_EINVAL, "level " + std::to_string(level) + " outside [0, " + std::to_string(m->max_level) + "]");
  if (device && m->host_only) return set_error(MF_ENOTSUP, "mesh was created host-only");
  return MF_OK;
}

int check_dtype(int dtype) {
  if (dtype != MF_F64 && dtype != MF_F32) return set_error(MF_EINVAL, "dtype must be MF_F64 or MF_F32");
  return MF_OK;
}

// Two doubles device -> host through a pinned buffer of the calling thread
// (a copy into pageable memory goes through the runtime's staging blit, about
// 20 us per solver iteration on MI355X).  The buffer lives until the process
// ends.
int sync_result(const double* result_dev, double out[2], hipStream_t s) {
  static thread_local double* pinned = nullptr;
  hipError_t e = hipSuccess;
  if (!pinned) e = hipHostMalloc((void**)&pinned, 2 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpyAsync(pinned, result_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  out[0] = pinned[0];
  out[1] = pinned[1];
  return MF_OK;
}

// r = b - A x with partials in `part`; reduces to result_dev and copies back.
int residual_norm(const mf_mesh* m, const Level& L, int dtype, const void* b, const void* x, void* r, double* part,
                  double* result_dev, double* ss, double* mx, hipStream_t s) {
  const int64_t np = stencil_partials(L, dtype);
  int rc = launch_stencil(m, L, dtype, kResidual, x, r, b, 0.0, part, s);
  if (!rc) rc = launch_reduce(part, np, result_dev, s);
  double out[2] = {0.0, 0.0};
  if (!rc) rc = sync_result(result_dev, out, s);
  if (rc) return rc;
  *ss = out[0];
  *mx = out[1];
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return set_error(MF_ENUMERIC, "residual norm is not finite");
  return MF_OK;
}

// sum of squares and max |.| of b over unique DoFs
int vector_norm(const mf_mesh* m, const Level& L, int dtype, const void* b, double* part, double* result_dev,
                double* ss, double* mx, hipStream_t s) {
  const int64_t np = stencil_partials(L, dtype);
  int rc = launch_stencil(m, L, dtype, kNormB, b, nullptr, b, 0.0, part, s);
  if (!rc) rc = launch_reduce(part, np, result_dev, s);
  double out[2] = {0.0, 0.0};
  if (!rc) rc = sync_result(result_dev, out, s);
  if (rc) return rc;
  *ss = out[0];
  *mx = out[1];
  if (!std::isfinite(out[0])) return set_error(MF_ENUMERIC, "norm of b is not finite");
  return MF_OK;
}

int jacobi_sweeps(const mf_mesh* m, const Level& L, int dtype, double omega, int sweeps, const void* b, void* x,
                  void* tmp, hipStream_t s) {
  void* cur = x;
  void* oth = tmp;
  for (int i = 0; i < sweeps; ++i) {
    const int rc = launch_stencil(m, L, dtype, kJacobi, cur, oth, b, omega, nullptr, s);
    if (rc) return rc;
    std::swap(cur, oth);
  }
  if (cur != x) return launch_copy(dtype, x, cur, L.storage, s);
  return MF_OK;
}

// Jacobi sweeps from a zero iterate: the first sweep is y = omega D^-1 b (one
// pass, no exchange), bitwise what a full sweep gives from x = 0; the rest as
// jacobi_sweeps.  x need not be initialised.
int jacobi_sweeps_from_zero(const mf_mesh* m, const Level& L, int dtype, double omega, int sweeps, const void* b,
                            void* x, void* tmp, hipStream_t s) {
  if (sweeps == 0) return launch_fill(dtype, x, 0.0, L.storage, s);
  int rc = launch_jacobi0(m, L, dtype, omega, b, tmp, s);
  void* cur = tmp;
  void* oth = x;
  for (int i = 1; i < sweeps && !rc; ++i) {
    rc = launch_stencil(m, L, dtype, kJacobi, cur, oth, b, omega, nullptr, s);
    std::swap(cur, oth);
  }
  if (!rc && cur != x) rc = launch_copy(dtype, x, cur, L.storage, s);
  return rc;
}

// One V-cycle on b[l] from the zero iterate; the correction lands in x[l].
// Levels lc .. lc + tail - 1 (tail = tail_levels(...), 0 for none) run in one
// workgroup launch.
int vcycle(const mf_mesh* m, int l, int lc, int tail, int dtype, const Workspace& w, const mf_solve_opts& o,
           hipStream_t s) {
  const Level& L = m->levels[l];
  if (tail > 0 && l == lc + tail - 1) return launch_vcycle_tail(m, lc, tail, dtype, o.pre, o.post, o.omega, w.b, w.x, w.t, s);
  if (l == lc) return launch_coarse_solve(L, dtype, w.b[l], w.x[l], s);
  int rc = jacobi_sweeps_from_zero(m, L, dtype, o.omega, o.pre, w.b[l], w.x[l], w.t[l], s);
  if (rc) return rc;
  rc = launch_stencil(m, L, dtype, kResidual, w.x[l], w.t[l], w.b[l], 0.0, nullptr, s);
  if (!rc) rc = launch_restrict(m, L, m->levels[l - 1], dtype, w.t[l], w.b[l - 1], s);
  if (!rc) rc = vcycle(m, l - 1, lc, tail, dtype, w, o, s);
  if (!rc) rc = launch_prolong_add(m, L, m->levels[l - 1], dtype, w.x[l - 1], w.x[l], s);
  if (!rc) rc = jacobi_sweeps(m, L, dtype, o.omega, o.post, w.b[l], w.x[l], w.t[l], s);
  return rc;
}

// z = M v: one V-cycle on v from the zero iterate, then partials of v . z
// (unique DoFs) reduced into result[2].  FP32 cycles take v scaled by
// 1 / result[1] (its max |.|, already on the device) and z = result[1] e is
// formed in FP64; FP64 cycles read v and write z in place of b and x of the
// top level.
int precondition(const mf_mesh* m, int level, int lc, int tail, bool f32, Workspace& w, const mf_solve_opts& o,
                 const double* v, double* z, hipStream_t s) {
  const Level& L = m->levels[level];
  int rc;
  if (f32) {
    rc = launch_scale_to_f32(v, (float*)w.b[level], w.result, L.storage, s);
    if (!rc) rc = vcycle(m, level, lc, tail, MF_F32, w, o, s);
    if (!rc) rc = launch_pcg_zdot(m, L, MF_F32, v, w.x[level], z, w.result, w.part, s);
  } else {
    w.b[level] = (void*)v;
    w.x[level] = z;
    rc = vcycle(m, level, lc, tail, MF_F64, w, o, s);
    if (!rc) rc = launch_pcg_zdot(m, L, MF_F64, v, z, z, w.result, w.part, s);
  }
  if (!rc) rc = launch_reduce(w.part, L.lin_blocks(), w.result + 2, s);
  return rc;
}

// Preconditioned MINRES (the outer solver of the paper's plume application,
// there around a block preconditioner; here around the symmetric V-cycle M,
// which is positive definite for this operator).  Lanczos in the inner
// product induced by M: the vectors v_j are kept unnormalised (gamma_j =
// sqrt(v_j . M v_j), z_j = M v_j / gamma_j), the tridiagonal is reduced by
// Givens rotations (c, s), and the directions w_j give x_j = x_{j-1} +
// c_{j+1} eta w_{j+1}; |eta| = sqrt(r . M r) for the current residual r,
// the norm MINRES minimises.  When |eta| falls to `trigger`
// times its first value (rtol at first) the FP64 residual b - A x is
// computed; the solve ends when it meets rtol, otherwise the trigger is
// tightened and the recurrence goes on.  On entry r64 holds b - A x and
// result[1] its max |.|.
int minres_iterate(const mf_mesh* m, int level, int lc, int tail, const double* b, double* x, Workspace& w,
                   const mf_solve_opts& o, double bnorm, double rel0, hipStream_t s, int* iters, double* rel_out,
                   bool* converged) {
  const Level& L = m->levels[level];
  const int64_t n = L.storage;
  const bool f32 = mode_f32(o.mode);
  const int nlin = (int)L.lin_blocks();
  double* v = w.r64;
  double* vo = w.v2;
  double* z = w.z64;
  double* zn = w.z2;
  double* wc = w.w1;
  double* wo = w.w2;
  int rc = launch_fill(MF_F64, vo, 0.0, n, s);
  if (!rc) rc = launch_fill(MF_F64, wc, 0.0, n, s);
  if (!rc) rc = launch_fill(MF_F64, wo, 0.0, n, s);
  if (!rc) rc = precondition(m, level, lc, tail, f32, w, o, v, z, s);
  double out[2] = {0.0, 0.0};
  if (!rc) rc = sync_result(w.result + 2, out, s);
  if (rc) return rc;
  auto true_rel = [&](double* rel) {
    double ts = 0.0, tm = 0.0;
    const int r = residual_norm(m, L, MF_F64, b, x, w.q64, w.part, w.result + 6, &ts, &tm, s);
    *rel = bnorm > 0.0 ? std::sqrt(ts) / bnorm : std::sqrt(ts);
    return r;
  };
  if (!std::isfinite(out[0]) || out[0] < 0.0)
    return set_error(MF_ENUMERIC, "preconditioner is not positive definite (v . M v < 0 or not finite)");
  double gamma = std::sqrt(out[0]), gamma_o = 1.0;
  double eta = gamma;
  const double eta0 = gamma;
  double c = 1.0, c_o = 1.0, sn = 0.0, sn_o = 0.0;
  double trigger = o.rtol, rel = rel0;
  int it = 0;
  *converged = false;
  for (;;) {
    if (gamma == 0.0 || std::fabs(eta) <= trigger * eta0) {
      // the M^-1-norm says converged (or v = 0): check the FP64 residual
      if (it > 0) {
        rc = true_rel(&rel);
        if (rc) return rc;
      }
      if (rel <= o.rtol || gamma == 0.0) {
        *converged = rel <= o.rtol;
        break;
      }
      trigger *= std::min(0.5, o.rtol / rel);
    }
    if (it >= o.max_iter) {
      if (it > 0) rc = true_rel(&rel);
      break;
    }
    // q = A z_u (z_u = gamma z_j) and z_u . q
    rc = launch_stencil(m, L, MF_F64, kApplyDot, z, w.q64, nullptr, 0.0, w.part, s);
    if (!rc) rc = launch_reduce(w.part, stencil_partials(L, MF_F64), w.result + 4, s);
    if (!rc) rc = sync_result(w.result + 4, out, s);
    if (rc) return rc;
    const double delta = out[0] / (gamma * gamma);  // z_j . A z_j
    // v_{j+1} = A z_j - (delta / gamma_j) v_j - (gamma_j / gamma_{j-1}) v_{j-1}, over v_{j-1}
    rc = launch_lin3(vo, w.q64, v, -gamma / gamma_o, 1.0 / gamma, -delta / gamma, n, f32 ? w.part : nullptr, nlin, s);
    if (!rc && f32) rc = launch_reduce(w.part, nlin, w.result, s);  // max |v_{j+1}| for the FP32 scaling
    std::swap(v, vo);
    if (!rc) rc = precondition(m, level, lc, tail, f32, w, o, v, zn, s);
    if (!rc) rc = sync_result(w.result + 2, out, s);
    if (rc) return rc;
    if (!std::isfinite(out[0]) || out[0] < 0.0)
      return set_error(MF_ENUMERIC, "preconditioner is not positive definite (v . M v < 0 or not finite)");
    const double gamma_n = std::sqrt(out[0]);
    // the new column of the tridiagonal, rotated by the last two rotations,
    // and the rotation that annihilates gamma_{j+1}
    const double a0 = c * delta - c_o * sn * gamma;
    const double a1 = std::hypot(a0, gamma_n);
    const double a2 = sn * delta + c_o * c * gamma;
    const double a3 = sn_o * gamma;
    if (!(a1 > 0.0) || !std::isfinite(a1)) return set_error(MF_ENUMERIC, "MINRES breakdown (zero rotation norm)");
    const double c_n = a0 / a1, sn_n = gamma_n / a1;
    // w_{j+1} = (z_j - a3 w_{j-1} - a2 w_j) / a1, over w_{j-1}; x += c_{j+1} eta w_{j+1}
    rc = launch_lin3(wo, z, wc, -a3 / a1, 1.0 / (a1 * gamma), -a2 / a1, n, nullptr, nlin, s);
    std::swap(wc, wo);
    if (!rc) rc = launch_axpy(MF_F64, x, wc, c_n * eta, n, s);
    if (rc) return rc;
    eta = -sn_n * eta;
    c_o = c;
    c = c_n;
    sn_o = sn;
    sn = sn_n;
    gamma_o = gamma;
    gamma = gamma_n;
    std::swap(z, zn);
    ++it;
  }
  *iters = it;
  *rel_out = rel;
  return rc;
}

}  // namespace

extern "C" {

const char* mf_last_error(void) { return mf::last_error(); }

int create_macro_mesh(int dim, int64_t n_vertices, const double* coords, int64_t n_cells, const int64_t* cells,
                      int max_level, int flags, mf_mesh** out) {
  if (!out) return set_error(MF_EINVAL, "out is NULL");
  *out = nullptr;
  if (dim != 2 && dim != 3) return set_error(MF_EINVAL, "dim must be 2 or 3");
  if (!coords || !cells || n_vertices <= 0 || n_cells <= 0) return set_error(MF_EINVAL, "empty or NULL mesh arrays");
  const int lmax = dim == 2 ? 15 : 11;
  if (max_level < 0 || max_level > lmax)
    return set_error(MF_EINVAL, "max_level must be in [0, " + std::to_string(lmax) + "]");
  if (n_cells > (int64_t)1 << 30) return set_error(MF_EINVAL, "too many cells");
  mf_mesh* m = nullptr;
  try {
    m = new mf_mesh;
    m->dim = dim;
    m->max_level = max_level;
    m->flags = flags;
    m->host_only = (flags & MF_FLAG_HOST_ONLY) != 0;
    m->nv = n_vertices;
    m->nc = n_cells;
    m->coords.assign(coords, coords + n_vertices * dim);
    m->cells.assign(cells, cells + n_cells * (dim + 1));
    const int rc = build_mesh(m);
    if (rc) {
      free_device(m);
      delete m;
      return rc;
    }
  } catch (const std::bad_alloc&) {
    if (m) {
      free_device(m);
      delete m;
    }
    return set_error(MF_ENOMEM, "host allocation failed");
  }
  *out = m;
  set_error(MF_OK, "");
  return MF_OK;
}

int destroy_macro_mesh(mf_mesh* m) {
  if (!m) return MF_OK;
  free_device(m);
  delete m;
  return MF_OK;
}

int mesh_info(const mf_mesh* m, int* dim, int64_t* n_macros, int* max_level) {
  if (!m) return set_error(MF_EINVAL, "mesh is NULL");
  if (dim) *dim = m->dim;
  if (n_macros) *n_macros = m->nc;
  if (max_level) *max_level = m->max_level;
  return MF_OK;
}

int mesh_num_dofs(const mf_mesh* m, int level, int64_t* storage, int64_t* unique) {
  int rc = check_mesh(m, level, false);
  if (rc) return rc;
  if (storage) *storage = m->levels[level].storage;
  if (unique) *unique = m->levels[level].unique;
  return MF_OK;
}

int mesh_dof_keys(const mf_mesh* m, int level, int64_t* vids, int32_t* weights) {
  int rc = check_mesh(m, level, false);
  if (rc) return rc;
  if (!vids || !weights) return set_error(MF_EINVAL, "NULL output");
  storage_keys(m, level, vids, weights);
  return MF_OK;
}

int mesh_dof_index(const mf_mesh* m, int level, int64_t n, const int64_t* ml, int64_t* index) {
  int rc = check_mesh(m, level, false);
  if (rc) return rc;
  if (n < 0 || (n > 0 && (!ml || !index))) return set_error(MF_EINVAL, "bad arrays");
  const int d1 = m->dim + 1;
  const Level& L = m->levels[level];
  for (int64_t i = 0; i < n; ++i) {
    const int64_t c = ml[i * d1], x = ml[i * d1 + 1], y = ml[i * d1 + 2], z = m->dim == 3 ? ml[i * d1 + 3] : 0;
    if (c < 0 || c >= m->nc || x < 0 || y < 0 || z < 0 || x + y + z > L.N)
      return set_error(MF_EINVAL, "point " + std::to_string(i) + " outside its macro");
    index[i] = L.base[c] + (m->dim == 2 ? idx2(L.N, (int)x, (int)y) : idx3(L.N, (int)x, (int)y, (int)z));
  }
  return MF_OK;
}

int mesh_stencil(const mf_mesh* m, int level, int64_t macro, double* w) {
  int rc = check_mesh(m, level, false);
  if (rc) return rc;
  if (macro < 0 || macro >= m->nc || !w) return set_error(MF_EINVAL, "bad macro or NULL output");
  const int n = m->dim == 2 ? 7 : 15;
  std::memcpy(w, m->levels[level].md[macro].wm[full_mask(m->dim)], sizeof(double) * n);
  return MF_OK;
}

int mesh_workspace_bytes(const mf_mesh* m, int level, int mode, int64_t* bytes) {
  int rc = check_mesh(m, level, false);
  if (rc) return rc;
  if (mode < 0 || mode >= kNumModes) return set_error(MF_EINVAL, "mode must be in 0..5");
  if (!bytes) return set_error(MF_EINVAL, "NULL output");
  *bytes = carve(m, level, mode, 0, nullptr).bytes;
  return MF_OK;
}

int mesh_fill_random(const mf_mesh* m, int level, int dtype, uint64_t seed, void* x, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!x) return set_error(MF_EINVAL, "x is NULL");
  return launch_fill_random(m, m->levels[level], dtype, seed, x, (hipStream_t)stream);
}

int mesh_set_dirichlet(const mf_mesh* m, int level, int dtype, const void* b, void* y, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!y) return set_error(MF_EINVAL, "y is NULL");
  return launch_iface(m, m->levels[level], dtype, kDirichletSet, y, y, b, (hipStream_t)stream);
}

int apply_stencil(const mf_mesh* m, int level, int dtype, const void* x, void* y, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!x || !y) return set_error(MF_EINVAL, "NULL vector");
  if (x == y) return set_error(MF_EINVAL, "y must not alias x");
  const Level& L = m->levels[level];
  hipStream_t s = (hipStream_t)stream;
  return launch_stencil(m, L, dtype, kApply, x, y, nullptr, 0.0, nullptr, s);
}

int apply_varcoef(const mf_mesh* m, int level, int dtype, const void* k, const void* x, void* y, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!k || !x || !y) return set_error(MF_EINVAL, "NULL vector");
  if (x == y || k == y) return set_error(MF_EINVAL, "y must not alias x or k");
  return launch_varcoef_apply(m, m->levels[level], dtype, k, x, y, (hipStream_t)stream);
}

int apply_blended(const mf_mesh* m, int level, const double* bubble, const double* x, double* y, void* stream) {
  int rc = check_mesh(m, level, true);
  if (rc) return rc;
  if (m->dim != 2) return set_error(MF_ENOTSUP, "blended macros are built for 2D meshes");
  if (!bubble || !x || !y) return set_error(MF_EINVAL, "NULL vector");
  if (x == y) return set_error(MF_EINVAL, "y must not alias x");
  return launch_blended_apply(m, m->levels[level], bubble, x, y, (hipStream_t)stream);
}

int apply_p2(const mf_mesh* m, int level, int dtype, const void* x, void* y, void* stream) {
  if (!m) return set_error(MF_EINVAL, "NULL mesh");
  if (m->dim != 2) return set_error(MF_ENOTSUP, "the P2 operator is built for 2D meshes");
  if (level < 0 || level + 1 > m->max_level)
    return set_error(MF_EINVAL, "P2 level must satisfy 0 <= level < max_level (it uses the lattice of level + 1)");
  int rc = check_mesh(m, level + 1, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!x || !y) return set_error(MF_EINVAL, "NULL vector");
  if (x == y) return set_error(MF_EINVAL, "y must not alias x");
  return launch_p2_apply(m, level, dtype, x, y, (hipStream_t)stream);
}

int smooth(const mf_mesh* m, int level, int dtype, double omega, int sweeps, const void* b, void* x, void* tmp,
           void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!b || !x || !tmp) return set_error(MF_EINVAL, "NULL vector");
  if (sweeps < 0) return set_error(MF_EINVAL, "sweeps < 0");
  if (x == tmp || b == x || b == tmp) return set_error(MF_EINVAL, "b, x and tmp must be distinct");
  return jacobi_sweeps(m, m->levels[level], dtype, omega, sweeps, b, x, tmp, (hipStream_t)stream);
}

int residual(const mf_mesh* m, int level, int dtype, const void* b, const void* x, void* r, double* norm2,
             void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (!b || !x || !r) return set_error(MF_EINVAL, "NULL vector");
  if (r == x || r == b) return set_error(MF_EINVAL, "r must not alias b or x");
  const Level& L = m->levels[level];
  hipStream_t s = (hipStream_t)stream;
  if (!norm2) {
    return launch_stencil(m, L, dtype, kResidual, x, r, b, 0.0, nullptr, s);
  }
  std::lock_guard<std::mutex> lock(const_cast<mf_mesh*>(m)->norm_mutex);
  double ss = 0.0, mx = 0.0;
  rc = residual_norm(m, L, dtype, b, x, r, L.dev.part, L.dev.result, &ss, &mx, s);
  *norm2 = std::sqrt(ss);
  return rc;
}

int restrict_residual(const mf_mesh* m, int level, int dtype, const void* rf, void* bc, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (level < 1) return set_error(MF_EINVAL, "restriction needs level >= 1");
  if (!rf || !bc || rf == bc) return set_error(MF_EINVAL, "NULL or aliased vectors");
  return launch_restrict(m, m->levels[level], m->levels[level - 1], dtype, rf, bc, (hipStream_t)stream);
}

int prolong_add(const mf_mesh* m, int level, int dtype, const void* ec, void* xf, void* stream) {
  int rc = check_mesh(m, level, true);
  if (!rc) rc = check_dtype(dtype);
  if (rc) return rc;
  if (level < 1) return set_error(MF_EINVAL, "prolongation needs level >= 1");
  if (!ec || !xf || ec == xf) return set_error(MF_EINVAL, "NULL or aliased vectors");
  return launch_prolong_add(m, m->levels[level], m->levels[level - 1], dtype, ec, xf, (hipStream_t)stream);
}

int vcycle_solve(const mf_mesh* m, int level, const double* b, double* x, void* workspace,
                 const mf_solve_opts* opts, mf_solve_info* info, void* stream) {
  int rc = check_mesh(m, level, true);
  if (rc) return rc;
  if (!b || !x || !workspace) return set_error(MF_EINVAL, "NULL vector or workspace");
  mf_solve_opts o = {0, 2, 2, default_coarse(level), 50, 2.0 / 3.0, 1e-10};
  if (opts) o = *opts;
  if (o.mode < 0 || o.mode >= kNumModes) return set_error(MF_EINVAL, "mode must be in 0..5");
  if (mode_krylov(o.mode) && o.pre != o.post)
    return set_error(MF_EINVAL, "conjugate gradients and MINRES need a symmetric V-cycle (pre == post)");
  if (o.pre < 0 || o.post < 0 || o.max_iter < 0 || !(o.rtol >= 0.0))
    return set_error(MF_EINVAL, "bad solver options");
  if (o.coarse_level < 0 || o.coarse_level > level) return set_error(MF_EINVAL, "coarse_level outside [0, level]");
  const int lc = o.coarse_level;
  {
    std::lock_guard<std::mutex> lock(const_cast<mf_mesh*>(m)->norm_mutex);
    rc = build_coarse_solver(const_cast<mf_mesh*>(m), lc);
  }
  if (rc) return rc;
  const int tail = tail_levels(m, level, lc);
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  const Level& L = m->levels[level];
  Workspace w = carve(m, level, o.mode, 0, (char*)workspace);
  const bool f32 = mode_f32(o.mode), pcg = mode_pcg(o.mode);
  const int vdt = f32 ? MF_F32 : MF_F64;
  // Dirichlet entries of x take b's values; the correction never changes them.
  rc = launch_iface(m, L, MF_F64, kDirichletSet, x, x, b, s);
  // ||b|| over unique DoFs
  double ss = 0.0, mx = 0.0;
  if (!rc) rc = vector_norm(m, L, MF_F64, b, w.part, w.result, &ss, &mx, s);
  if (rc) return rc;
  const double bnorm = std::sqrt(ss);
  // r = b - A x; PCG scalars start at zero (first direction p = z)
  rc = residual_norm(m, L, MF_F64, b, x, w.r64, w.part, w.result, &ss, &mx, s);
  if (!rc && pcg) rc = launch_fill(MF_F64, w.result + 2, 0.0, 6, s);
  if (!rc && pcg && f32) {
    // the first FP32 preconditioner input; the CG update forms the later ones
    rc = launch_scale_to_f32(w.r64, (float*)w.b[level], w.result, L.storage, s);
    if (!rc) rc = launch_copy(MF_F64, w.result + kSlotScale, w.result + 1, 1, s);
  }
  if (rc) return rc;
  if (mode_minres(o.mode)) {
    int it = 0;
    double rel = bnorm > 0.0 ? std::sqrt(ss) / bnorm : std::sqrt(ss);
    bool converged = false;
    if (rel <= o.rtol || mx == 0.0) {
      converged = true;
    } else {
      rc = minres_iterate(m, level, lc, tail, b, x, w, o, bnorm, rel, s, &it, &rel, &converged);
      if (rc) return rc;
    }
    if (info) {
      info->iters = it;
      info->rel_res = rel;
      info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? MF_OK : MF_NOT_CONVERGED;
  }
  const int64_t nlin = L.lin_blocks();
  int it = 0;
  double rel = 0.0;
  bool converged = false;
  for (;;) {
    rel = bnorm > 0.0 ? std::sqrt(ss) / bnorm : std::sqrt(ss);
    if (rel <= o.rtol || mx == 0.0) {
      if (pcg && it > 0) {
        // The CG recurrence says converged: confirm it on the true FP64
        // residual b - A x (into q, which the next iteration overwrites, and
        // result[6..7], which no recurrence reads), and report that value.
        // If it misses the tolerance the recurrence goes on unchanged.
        double ts = 0.0, tm = 0.0;
        rc = residual_norm(m, L, MF_F64, b, x, w.q64, w.part, w.result + 6, &ts, &tm, s);
        if (rc) return rc;
        rel = bnorm > 0.0 ? std::sqrt(ts) / bnorm : std::sqrt(ts);
        converged = rel <= o.rtol || tm == 0.0;
      } else {
        converged = true;
      }
      if (converged) break;
    }
    if (it >= o.max_iter) break;
    // preconditioner / correction: one V-cycle on r from zero
    if (f32 && !pcg) {
      // scale r by its max norm before the cast so FP32 keeps its relative precision
      rc = launch_scale_to_f32(w.r64, (float*)w.b[level], w.result, L.storage, s);
    }
    if (!rc) rc = vcycle(m, level, lc, tail, vdt, w, o, s);
    if (rc) return rc;
    if (!pcg) {
      // iterative refinement: x += e, then the new residual
      if (f32) rc = launch_axpy_f32(x, (const float*)w.x[level], w.result, L.storage, s);
      else rc = launch_axpy(MF_F64, x, w.x[level], 1.0, L.storage, s);
      if (!rc) rc = residual_norm(m, L, MF_F64, b, x, w.r64, w.part, w.result, &ss, &mx, s);
    } else {
      // conjugate gradients preconditioned by the V-cycle; scalars stay on the device
      // FP32 cycles: z = s e with s = the scale the input was formed with
      rc = launch_pcg_zdot(m, L, vdt, w.r64, w.x[level], w.z64, w.result, w.part, s, kSlotScale);
      if (!rc) rc = launch_reduce_shift(w.part, nlin, w.result + 2, s);                // r.z, previous r.z
      if (!rc)
        rc = launch_pcg_dir(w.p64, f32 ? w.x[level] : (const void*)w.z64, w.result, L.storage, s, vdt,
                            kSlotScale);  // p = z + beta p
      if (!rc) rc = launch_stencil(m, L, MF_F64, kApplyDot, w.p64, w.q64, nullptr, 0.0, w.part, s);
      if (!rc) rc = launch_reduce(w.part, stencil_partials(L, MF_F64), w.result + 4, s);       // p.Ap
      // x, r and, in mixed mode, the next FP32 preconditioner input
      if (!rc)
        rc = launch_pcg_update(m, L, x, w.r64, w.p64, w.q64, w.result, w.part, s,
                               f32 ? (float*)w.b[level] : nullptr, f32 ? w.result + kSlotScale : nullptr);
      if (!rc) rc = launch_reduce(w.part, nlin, w.result, s);                          // r.r, max|r|
      double out[2] = {0.0, 0.0};
      if (!rc) rc = sync_result(w.result, out, s);
      if (!rc) {
        ss = out[0];
        mx = out[1];
        if (!std::isfinite(ss) || !std::isfinite(mx)) rc = set_error(MF_ENUMERIC, "residual norm is not finite");
      }
    }
    if (rc) return rc;
    ++it;
  }
  if (info) {
    info->iters = it;
    info->rel_res = rel;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return converged ? MF_OK : MF_NOT_CONVERGED;
}

}  // extern "C"
