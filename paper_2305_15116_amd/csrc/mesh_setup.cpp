// Host set-up of a macro mesh: topology, per-level stencils and element
// matrices, interface groups, tile lists, coarse direct solver, device upload.
//
// The macro mesh is the unstructured coarse grid of the paper; each macro is
// refined uniformly, giving a structured index space per macro (Intro,
// "Hybrid Tetrahedral Grids").  Because all interior rows of a macro are the
// same, one stencil per macro and level is computed here (the paper's
// constant stencils, PETSc comparison section) from the element matrices of
// the few micro-element types; DoFs on macro boundaries are gathered into
// "groups" (one per unique DoF) that the interface kernel completes.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "mesh.hpp"

namespace mf {

namespace {
thread_local std::string t_err;
}

int set_error(int code, const std::string& msg) {
  t_err = msg;
  return code;
}
const char* last_error() { return t_err.c_str(); }

namespace {

// Element matrix of a simplex with edge matrix E (columns = edges from vertex
// 0) via the metric tensor: with G = E^{-T} the barycentric gradients of
// vertices 1..d are the columns of G, so g_i . g_j = ((E^T E)^{-1})_ij;
// vertex 0's gradient is minus their sum.  K = |T| (g_i . g_j).
bool metric_stiffness(int dim, const double E[3][3], double K[4][4]) {
  double Mt[3][3] = {{0}};
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) {
      double s = 0.0;
      for (int r = 0; r < dim; ++r) s += E[r][i] * E[r][j];
      Mt[i][j] = s;
    }
  double det, inv[3][3] = {{0}};
  if (dim == 2) {
    det = Mt[0][0] * Mt[1][1] - Mt[0][1] * Mt[1][0];
    if (!(det > 0.0)) return false;
    inv[0][0] = Mt[1][1] / det;
    inv[1][1] = Mt[0][0] / det;
    inv[0][1] = inv[1][0] = -Mt[0][1] / det;
  } else {
    const double a = Mt[0][0], b = Mt[0][1], c = Mt[0][2], d = Mt[1][1], e = Mt[1][2], f = Mt[2][2];
    const double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
    det = a * A + b * B + c * C;
    if (!(det > 0.0)) return false;
    inv[0][0] = A / det;
    inv[0][1] = inv[1][0] = B / det;
    inv[0][2] = inv[2][0] = C / det;
    inv[1][1] = (a * f - c * c) / det;
    inv[1][2] = inv[2][1] = (b * c - a * e) / det;
    inv[2][2] = (a * d - b * b) / det;
  }
  // |det E| = sqrt(det(E^T E))
  const double vol = std::sqrt(det) / (dim == 2 ? 2.0 : 6.0);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) K[i][j] = 0.0;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) K[i + 1][j + 1] = vol * inv[i][j];
  for (int j = 1; j <= dim; ++j) {
    double s = 0.0;
    for (int i = 1; i <= dim; ++i) s += K[i][j];
    K[0][j] = -s;
    K[j][0] = -s;
  }
  double s = 0.0;
  for (int i = 1; i <= dim; ++i)
    for (int j = 1; j <= dim; ++j) s += K[i][j];
  K[0][0] = s;
  return true;
}

struct PointKey {
  int64_t v[4];
  int32_t w[4];
  bool operator<(const PointKey& o) const {
    for (int k = 0; k < 4; ++k) {
      if (v[k] != o.v[k]) return v[k] < o.v[k];
      if (w[k] != o.w[k]) return w[k] < o.w[k];
    }
    return false;
  }
  bool operator==(const PointKey& o) const {
    for (int k = 0; k < 4; ++k)
      if (v[k] != o.v[k] || w[k] != o.w[k]) return false;
    return true;
  }
};

PointKey point_key(int dim, const int64_t* cellv, int N, int x, int y, int z) {
  const int64_t w[4] = {N - x - y - (dim == 3 ? z : 0), x, y, z};
  std::pair<int64_t, int64_t> pr[4];
  int n = 0;
  for (int k = 0; k <= dim; ++k)
    if (w[k] != 0) pr[n++] = {cellv[k], w[k]};
  // insertion sort by vertex id (at most 4 entries)
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && pr[j].first < pr[j - 1].first; --j) std::swap(pr[j], pr[j - 1]);
  PointKey k;
  for (int i = 0; i < 4; ++i) {
    k.v[i] = i < n ? pr[i].first : -1;
    k.w[i] = i < n ? (int32_t)pr[i].second : 0;
  }
  return k;
}

template <class F>
void for_each_boundary_point(int dim, int N, F&& fn) {
  if (dim == 2) {
    for (int y = 0; y <= N; ++y) {
      if (y == 0 || y == N) {
        for (int x = 0; x <= N - y; ++x) fn(x, y, 0);
      } else {
        fn(0, y, 0);
        fn(N - y, y, 0);
      }
    }
    return;
  }
  for (int z = 0; z <= N; ++z) {
    const int M = N - z;
    for (int y = 0; y <= M; ++y) {
      if (z == 0 || y == 0 || y == M) {
        for (int x = 0; x <= M - y; ++x) fn(x, y, z);
      } else {
        fn(0, y, z);
        fn(M - y, y, z);
      }
    }
  }
}

// Runs fn(i) for i in [0, n) on up to 16 host threads when `work` is large.
template <class F>
void parallel_for(size_t n, int64_t work, F&& fn) {
  unsigned nt = std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (work < (1 << 20) || n < 2) nt = 1;
  nt = (unsigned)std::min<size_t>(nt, n);
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&] {
      for (size_t i; (i = next.fetch_add(1)) < n;) fn(i);
    });
  for (auto& t : th) t.join();
}

}  // namespace

// ---------------------------------------------------------------- topology
static int build_topology(mf_mesh* m) {
  const int d1 = m->dim + 1;
  std::map<std::vector<int64_t>, int> facet_count;
  std::map<std::vector<int64_t>, int64_t> seen;
  for (int64_t c = 0; c < m->nc; ++c) {
    std::vector<int64_t> s(&m->cells[c * d1], &m->cells[c * d1] + d1);
    std::sort(s.begin(), s.end());
    for (int k = 0; k + 1 < d1; ++k)
      if (s[k] == s[k + 1]) return set_error(MF_EINVAL, "cell " + std::to_string(c) + " repeats a vertex");
    if (seen.count(s)) return set_error(MF_EINVAL, "cell " + std::to_string(c) + " repeats an earlier cell");
    seen[s] = c;
    for (int skip = 0; skip < d1; ++skip) {
      std::vector<int64_t> f;
      for (int k = 0; k < d1; ++k)
        if (k != skip) f.push_back(s[k]);
      if (++facet_count[f] > 2) return set_error(MF_EINVAL, "non-conforming mesh: a facet has more than two cells");
    }
  }
  // lowest macro containing each primitive (vertex subset of a cell), and how many contain it
  std::map<std::vector<int64_t>, int64_t> owner;
  std::map<std::vector<int64_t>, int> containing;
  for (int64_t c = 0; c < m->nc; ++c)
    for (int s = 1; s < (1 << d1); ++s) {
      std::vector<int64_t> prim;
      for (int k = 0; k < d1; ++k)
        if (s & (1 << k)) prim.push_back(m->cells[c * d1 + k]);
      std::sort(prim.begin(), prim.end());
      auto it = owner.find(prim);
      if (it == owner.end() || it->second > c) owner[prim] = c;
      containing[prim] += 1;
    }
  // primitives lying in a boundary facet
  std::map<std::vector<int64_t>, bool> on_boundary;
  for (auto& kv : facet_count) {
    if (kv.second != 1) continue;
    const auto& f = kv.first;
    const int n = (int)f.size();
    for (int s = 1; s < (1 << n); ++s) {
      std::vector<int64_t> prim;
      for (int k = 0; k < n; ++k)
        if (s & (1 << k)) prim.push_back(f[k]);
      on_boundary[prim] = true;
    }
  }
  const bool dirichlet = (m->flags & MF_FLAG_DIRICHLET) != 0;
  m->own_mask.assign(m->nc, 0);
  m->dir_mask.assign(m->nc, 0);
  m->shared_mask.assign(m->nc, 0);
  for (int64_t c = 0; c < m->nc; ++c)
    for (int s = 1; s < (1 << d1); ++s) {
      std::vector<int64_t> prim;
      for (int k = 0; k < d1; ++k)
        if (s & (1 << k)) prim.push_back(m->cells[c * d1 + k]);
      std::sort(prim.begin(), prim.end());
      if (owner[prim] == c) m->own_mask[c] |= (uint16_t)(1u << s);
      if (containing[prim] >= 2) m->shared_mask[c] |= (uint16_t)(1u << s);
      if (dirichlet && on_boundary.count(prim)) m->dir_mask[c] |= (uint16_t)(1u << s);
    }
  // every proper vertex subset of a cell is a macro-boundary primitive
  m->prims.clear();
  std::map<std::vector<int64_t>, size_t> index;
  for (auto& kv : containing) {
    if ((int)kv.first.size() == d1) continue;
    index[kv.first] = m->prims.size();
    Prim P;
    P.v = kv.first;
    P.dirichlet = dirichlet && on_boundary.count(kv.first) > 0;
    m->prims.push_back(std::move(P));
  }
  for (int64_t c = 0; c < m->nc; ++c)
    for (int s = 1; s < (1 << d1) - 1; ++s) {
      std::vector<int64_t> prim;
      for (int k = 0; k < d1; ++k)
        if (s & (1 << k)) prim.push_back(m->cells[c * d1 + k]);
      std::sort(prim.begin(), prim.end());
      Prim& P = m->prims[index.at(prim)];
      std::array<int8_t, 3> loc{};
      for (size_t j = 0; j < P.v.size(); ++j)
        for (int k = 0; k < d1; ++k)
          if (m->cells[c * d1 + k] == P.v[j]) loc[j] = (int8_t)k;
      P.cell.push_back(c);  // cells are visited in increasing order
      P.local.push_back(loc);
    }
  return MF_OK;
}

// ---------------------------------------------------------------- per level
static int build_level(mf_mesh* m, int level, Level& L) {
  const int dim = m->dim, d1 = dim + 1;
  const int N = 1 << level;
  L.level = level;
  L.N = N;
  const ElemTable ET = elem_table(dim);
  const StencilTable ST = stencil_table(dim);

  // storage offsets and macro constants
  L.base.resize(m->nc);
  L.md.assign(m->nc, MacroDev{});
  int64_t off = 0;
  for (int64_t c = 0; c < m->nc; ++c) {
    L.base[c] = off;
    off += macro_points(dim, N);
    MacroDev& M = L.md[c];
    std::memset(&M, 0, sizeof(M));
    M.base = L.base[c];
    for (int k = 0; k < 4; ++k) M.vid[k] = k < d1 ? m->cells[c * d1 + k] : -1;
    M.N = N;
    M.own_mask = m->own_mask[c];
    M.dir_mask = m->dir_mask[c];
    M.shared_mask = m->shared_mask[c];
    // macro Jacobian columns P_k - P_0
    const double* P0 = &m->coords[m->cells[c * d1] * dim];
    double J[3][3] = {{0}};
    for (int k = 1; k <= dim; ++k) {
      const double* Pk = &m->coords[m->cells[c * d1 + k] * dim];
      for (int r = 0; r < dim; ++r) J[r][k - 1] = Pk[r] - P0[r];
    }
    for (int t = 0; t < ET.ntypes; ++t) {
      double E[3][3] = {{0}};
      for (int k = 1; k <= dim; ++k)
        for (int r = 0; r < dim; ++r) {
          double s = 0.0;
          for (int q = 0; q < dim; ++q) s += J[r][q] * (double)(ET.off[t][k][q] - ET.off[t][0][q]);
          E[r][k - 1] = s / (double)N;
        }
      double K[4][4];
      if (!metric_stiffness(dim, E, K)) return set_error(MF_EINVAL, "degenerate macro " + std::to_string(c));
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          M.K[t][i * 4 + j] = K[i][j];
          M.Kf[t][i * 4 + j] = (float)K[i][j];
        }
    }
    // Partial stencil of every support mask: sum, over the (type, local vertex v)
    // incidences of the micro-elements inside the macro that contain a point
    // with that support, of row v of K_t.  An incidence is present iff the
    // element's vertex offset o_v is zero in every coordinate that vanishes
    // at the point, and, on the far face (weight w0 = 0), iff o_v has the
    // largest coordinate sum of its type; the full mask gives the interior stencil.
    const int fm = full_mask(dim);
    for (int mask = 1; mask <= fm; ++mask) {
      for (int t = 0; t < ET.ntypes; ++t)
        for (int v = 0; v < ET.nv; ++v) {
          bool ok = true;
          int osum = 0;
          for (int k = 0; k < dim; ++k) {
            osum += ET.off[t][v][k];
            if (!((mask >> (k + 1)) & 1) && ET.off[t][v][k] != 0) ok = false;
          }
          if (!(mask & 1) && osum != ET.slack[t]) ok = false;
          if (!ok) continue;
          for (int u = 0; u < ET.nv; ++u) {
            int d[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k) d[k] = ET.off[t][u][k] - ET.off[t][v][k];
            int hit = -1;
            for (int q = 0; q < ST.n; ++q)
              if (ST.off[q][0] == d[0] && ST.off[q][1] == d[1] && ST.off[q][2] == d[2]) hit = q;
            if (hit < 0) return set_error(MF_EINVAL, "internal: stencil offset not found");
            M.wm[mask][hit] += M.K[t][v * 4 + u];
          }
        }
      for (int q = 0; q < ST.n; ++q) M.wmf[mask][q] = (float)M.wm[mask][q];
    }
    M.inv_diag = 1.0 / M.wm[fm][ST.centre];
    M.inv_diagf = (float)M.inv_diag;
  }
  L.storage = off;

  // interface groups: every macro-boundary DoF, primitive by primitive (the
  // points whose support is exactly that vertex / edge / face), with one copy
  // per containing macro in macro order.  Offsets are counted first, then the
  // primitives are filled in parallel.
  const size_t np = m->prims.size();
  std::vector<int64_t> g_off(np + 1, 0), c_off(np + 1, 0), x_off(np + 1, 0), xc_off(np + 1, 0);
  auto prim_points = [N](int p) -> int64_t {
    if (p == 1) return 1;
    if (p == 2) return std::max(N - 1, 0);
    return N >= 2 ? (int64_t)(N - 1) * (N - 2) / 2 : 0;
  };
  for (size_t i = 0; i < np; ++i) {
    const Prim& P = m->prims[i];
    const int64_t n = prim_points((int)P.v.size()), nc = (int64_t)P.cell.size();
    const bool xg = !P.dirichlet && nc >= 2;
    g_off[i + 1] = g_off[i] + n;
    c_off[i + 1] = c_off[i] + n * nc;
    x_off[i + 1] = x_off[i] + (xg ? n : 0);
    xc_off[i + 1] = xc_off[i] + (xg ? n * nc : 0);
  }
  if (c_off[np] > (int64_t)INT32_MAX) return set_error(MF_ENOMEM, "too many interface copies");
  L.grp_ptr.assign(g_off[np] + 1, 0);
  L.grp_flag.assign(g_off[np], 0);
  L.copies.assign(c_off[np], Copy{});
  L.xgrp_ptr.assign(x_off[np] + 1, 0);
  L.xcopies.assign(xc_off[np], Copy{});
  L.xgrp_invdiag.assign(x_off[np], 0.0);
  L.grp_ptr[g_off[np]] = (int32_t)c_off[np];
  L.xgrp_ptr[x_off[np]] = (int32_t)xc_off[np];
  auto fill = [&](size_t i) {
    const Prim& P = m->prims[i];
    const int p = (int)P.v.size();
    const size_t nc = P.cell.size();
    const bool xg = !P.dirichlet && nc >= 2;
    int64_t g = g_off[i], c = c_off[i], xi = x_off[i], xc = xc_off[i];
    auto emit = [&](const int* w) {
      L.grp_ptr[g] = (int32_t)c;
      L.grp_flag[g] = P.dirichlet ? 1 : 0;
      ++g;
      double diag = 0.0;
      if (xg) L.xgrp_ptr[xi] = (int32_t)xc;
      for (size_t k = 0; k < nc; ++k) {
        int wl[4] = {0, 0, 0, 0};
        for (int j = 0; j < p; ++j) wl[P.local[k][j]] = w[j];
        const Copy cp{(int32_t)P.cell[k], wl[1], wl[2], dim == 3 ? wl[3] : 0};
        L.copies[c++] = cp;
        if (xg) {
          L.xcopies[xc++] = cp;
          // the assembled diagonal is the sum of the copies' partial centre weights
          diag += L.md[cp.macro].wm[support_mask(dim, N, cp.x, cp.y, cp.z)][ST.centre];
        }
      }
      if (xg) L.xgrp_invdiag[xi++] = diag != 0.0 ? 1.0 / diag : 0.0;
    };
    int w[3];
    if (p == 1) {
      w[0] = N;
      emit(w);
    } else if (p == 2) {
      for (w[0] = 1; w[0] <= N - 1; ++w[0]) {
        w[1] = N - w[0];
        emit(w);
      }
    } else {
      for (w[0] = 1; w[0] <= N - 2; ++w[0])
        for (w[1] = 1; w[0] + w[1] <= N - 1; ++w[1]) {
          w[2] = N - w[0] - w[1];
          emit(w);
        }
    }
  };
  parallel_for(np, c_off[np], fill);
  const int64_t ngroups = L.ngroups();
  // unique DoFs: interior points of every macro + groups
  int64_t interior = 0;
  if (dim == 2) interior = N >= 3 ? tri_count(N - 2) : 0;
  else interior = N >= 4 ? tet_count(N - 3) : 0;
  L.unique = interior * m->nc + ngroups;

  // owner bits: bit i set iff storage DoF i is the copy that counts its
  // unique DoF in norms and dot products (interior points, and boundary
  // points whose primitive this macro owns)
  // (slices of every macro on several threads: a word whose bits come from
  // two rows is or-ed atomically, words inside one row are stored)
  std::vector<std::atomic<uint32_t>> bits((size_t)((L.storage + 31) / 32));
  for (auto& w : bits) w.store(0u, std::memory_order_relaxed);
  auto set_range = [&](int64_t lo, int64_t hi) {  // bits [lo, hi)
    for (int64_t i = lo; i < hi;) {
      if ((i & 31) == 0 && i + 32 <= hi) {
        bits[i >> 5].store(0xffffffffu, std::memory_order_relaxed);
        i += 32;
      } else {
        bits[i >> 5].fetch_or(1u << (i & 31), std::memory_order_relaxed);
        ++i;
      }
    }
  };
  const int nz = dim == 3 ? N + 1 : 1;
  parallel_for((size_t)(m->nc * nz), L.storage, [&](size_t job) {
    const int64_t c = (int64_t)job / nz;
    const int z = (int)((int64_t)job % nz);
    const uint16_t om = m->own_mask[c];
    const int S = N - z;
    for (int y = 0; y <= S; ++y) {
      const int64_t r0 = L.base[c] + (dim == 2 ? idx2(N, 0, y) : idx3(N, 0, y, z));
      const int len = S - y + 1;
      if (y >= 1 && z >= 1 - (dim == 2 ? 1 : 0) && len >= 3) {
        set_range(r0 + 1, r0 + len - 1);
        for (int x : {0, len - 1})
          if ((om >> support_mask(dim, N, x, y, z)) & 1) set_range(r0 + x, r0 + x + 1);
      } else {
        for (int x = 0; x < len; ++x) {
          const int mk = support_mask(dim, N, x, y, z);
          if (mk == full_mask(dim) || ((om >> mk) & 1)) set_range(r0 + x, r0 + x + 1);
        }
      }
    }
  });
  L.own_bits.resize(bits.size());
  for (size_t i = 0; i < bits.size(); ++i) L.own_bits[i] = bits[i].load(std::memory_order_relaxed);

  // storage indices of the copies, so that exchange kernels index directly
  auto storage_index = [&](const Copy& c) {
    return L.md[c.macro].base + (dim == 2 ? idx2(N, c.x, c.y) : idx3(N, c.x, c.y, c.z));
  };
  L.cpidx.resize(L.copies.size());
  L.xcpidx.resize(L.xcopies.size());
  constexpr size_t kChunk = 1 << 16;
  parallel_for((L.copies.size() + kChunk - 1) / kChunk, (int64_t)L.copies.size(), [&](size_t k) {
    for (size_t i = k * kChunk; i < std::min(L.copies.size(), (k + 1) * kChunk); ++i) L.cpidx[i] = storage_index(L.copies[i]);
  });
  parallel_for((L.xcopies.size() + kChunk - 1) / kChunk, (int64_t)L.xcopies.size(), [&](size_t k) {
    for (size_t i = k * kChunk; i < std::min(L.xcopies.size(), (k + 1) * kChunk); ++i)
      L.xcpidx[i] = storage_index(L.xcopies[i]);
  });

  // wave tiles over every point of every macro, natural order: macro,
  // (slice chunk,) strip, band; on small 3D levels runs of slice segments
  // (macro, slice, index)
  L.tiles.clear();
  L.pen_z = dim == 3 && N <= kSegUpToN ? kPenSeg : kPenZ;
  if (L.pen_z == kPenSeg)
    L.tiles.reserve((size_t)m->nc * (macro_points(dim, N) / (kWave * seg_run(N)) + N + 2) + 64);
  else
    L.tiles.reserve((size_t)m->nc * (macro_points(dim, N) / (kTileW * (dim == 2 ? kTileH2 : kPenR * L.pen_z)) * 2 + 64));
  for (int64_t c = 0; c < m->nc; ++c) {
    if (L.pen_z == kPenSeg) {
      for (int z = 0; z <= N; ++z) {
        const int64_t S = N - z, P = (S + 1) * (S + 2) / 2;
        const int64_t run = kWave * seg_run(N);
        for (int64_t r0 = 0; r0 < P; r0 += run)
          L.tiles.push_back({(int32_t)c, (int32_t)r0, (int32_t)std::min<int64_t>(run, P - r0), z});
      }
    } else if (dim == 2) {
      for (int y0 = 0; y0 <= N; y0 += kTileH2)
        for (int x0 = 0; x0 + y0 <= N; x0 += kTileW) L.tiles.push_back({(int32_t)c, x0, y0, 0});
    } else {
      for (int z0 = 0; z0 <= N; z0 += L.pen_z)
        for (int y0 = 0; y0 + z0 <= N; y0 += kPenR)
          for (int x0 = 0; x0 + y0 + z0 <= N; x0 += kTileW) L.tiles.push_back({(int32_t)c, x0, y0, z0});
    }
  }
  while (L.tiles.size() % kWavesPerWG) L.tiles.push_back({-1, 0, 0, 0});
  // (measured: on pencil levels the group work lengthens the launch more than
  // the exchange launch costs, cube level 8 FP64 apply 96 -> 109 us)
  L.xfused = L.pen_z == kPenSeg && dim == 3;
  if (L.xfused) {
    // group tiles: the shared DoFs, finished in the same launch.  Their
    // workgroups are spread evenly among the runs' (each XCD takes a
    // contiguous chunk of workgroups, so appended ones would all land on one)
    std::vector<Tile> grp;
    const int64_t ng = L.nxgroups();
    for (int64_t g0 = 0; g0 < ng; g0 += kWave)
      grp.push_back({kGroupTile, (int32_t)g0, (int32_t)std::min<int64_t>(kWave, ng - g0), 0});
    while (grp.size() % kWavesPerWG) grp.push_back({-1, 0, 0, 0});
    const size_t nr = L.tiles.size() / kWavesPerWG, ngw = grp.size() / kWavesPerWG;
    std::vector<Tile> all;
    all.reserve(L.tiles.size() + grp.size());
    size_t ir = 0, ig = 0;
    while (ir < nr || ig < ngw) {
      // next: a group workgroup while the groups lag the runs proportionally
      const bool take_g = ig < ngw && (ir == nr || ig * nr <= ir * ngw);
      const Tile* src = take_g ? &grp[ig++ * kWavesPerWG] : &L.tiles[ir++ * kWavesPerWG];
      all.insert(all.end(), src, src + kWavesPerWG);
    }
    L.tiles.swap(all);
  }
  L.tiles_f32.clear();
  if (dim == 2) {
    for (int64_t c = 0; c < m->nc; ++c)
      for (int y0 = 0; y0 <= N; y0 += kTileH2F)
        for (int x0 = 0; x0 + y0 <= N; x0 += kTileW) L.tiles_f32.push_back({(int32_t)c, x0, y0, 0});
    while (L.tiles_f32.size() % kWavesPerWG) L.tiles_f32.push_back({-1, 0, 0, 0});
  }

  // row segments of 64 points over every storage point
  L.segs.clear();
  L.segs.reserve((size_t)m->nc * (macro_points(dim, N) / kWave * 2 + 64));
  for (int64_t c = 0; c < m->nc; ++c) {
    const int zmax = dim == 3 ? N : 0;
    for (int z = 0; z <= zmax; ++z) {
      const int M = N - z;
      for (int y = 0; y <= M; ++y)
        for (int x0 = 0; x0 <= M - y; x0 += kWave) L.segs.push_back({(int32_t)c, x0, y, z});
    }
  }
  while (L.segs.size() % kWavesPerWG) L.segs.push_back({-1, 0, 0, 0});
  L.psegs.clear();
  L.psegs.reserve((size_t)m->nc * (macro_points(dim, N) / kWave + (dim == 3 ? N + 2 : 2)) + 64);
  for (int64_t c = 0; c < m->nc; ++c) {
    const int zmax = dim == 3 ? N : 0;
    for (int z = 0; z <= zmax; ++z) {
      const int64_t S = N - z, P = (S + 1) * (S + 2) / 2;
      for (int64_t r0 = 0; r0 < P; r0 += kWave) L.psegs.push_back({(int32_t)c, (int32_t)r0, 0, z});
    }
  }
  while (L.psegs.size() % kWavesPerWG) L.psegs.push_back({-1, 0, 0, 0});
  // runs of slice segments for the 3D prolongation: kTransferRun segments
  // from N = 256 on, single ones below (more waves in flight for the
  // smaller levels, measured faster there)
  L.pruns.clear();
  if (dim == 3) {
    for (int64_t c = 0; c < m->nc; ++c)
      for (int z = 0; z <= N; ++z) {
        const int64_t S = N - z, P = (S + 1) * (S + 2) / 2, run = kWave * (N >= 256 ? kTransferRun : 1);
        for (int64_t r0 = 0; r0 < P; r0 += run)
          L.pruns.push_back({(int32_t)c, (int32_t)r0, (int32_t)std::min<int64_t>(run, P - r0), z});
      }
    while (L.pruns.size() % kWavesPerWG) L.pruns.push_back({-1, 0, 0, 0});
  }
  L.sbase.assign(dim == 3 ? N + 2 : 1, 0);
  if (dim == 3)
    for (int z = 0; z <= N + 1; ++z) L.sbase[z] = (int32_t)slice_base(N, z);
  return MF_OK;
}

int upload_level(mf_mesh* m, Level& L) {
  LevelDev& D = L.dev;
  int rc;
  if ((rc = dev_upload(&D.md, L.md))) return rc;
  if ((rc = dev_upload(&D.tiles, L.tiles))) return rc;
  if ((rc = dev_upload(&D.tiles_f32, L.tiles_f32))) return rc;
  if ((rc = dev_upload(&D.segs, L.segs))) return rc;
  if ((rc = dev_upload(&D.psegs, L.psegs))) return rc;
  if ((rc = dev_upload(&D.sbase, L.sbase))) return rc;
  if ((rc = dev_upload(&D.pruns, L.pruns))) return rc;
  if ((rc = dev_upload(&D.grp_ptr, L.grp_ptr))) return rc;
  if ((rc = dev_upload(&D.copies, L.copies))) return rc;
  if ((rc = dev_upload(&D.grp_flag, L.grp_flag))) return rc;
  if ((rc = dev_upload(&D.xgrp_ptr, L.xgrp_ptr))) return rc;
  if ((rc = dev_upload(&D.xcopies, L.xcopies))) return rc;
  if ((rc = dev_upload(&D.cpidx, L.cpidx))) return rc;
  if ((rc = dev_upload(&D.xcpidx, L.xcpidx))) return rc;
  if ((rc = dev_upload(&D.xgrp_invdiag, L.xgrp_invdiag))) return rc;
  if ((rc = dev_upload(&D.own_bits, L.own_bits))) return rc;
  std::vector<float> f(L.xgrp_invdiag.begin(), L.xgrp_invdiag.end());
  if ((rc = dev_upload(&D.xgrp_invdiagf, f))) return rc;
  std::vector<double> zeros(2 * (L.n_partials() + 1), 0.0);
  if ((rc = dev_upload(&D.part, zeros))) return rc;
  std::vector<double> z2(2, 0.0);
  if ((rc = dev_upload(&D.result, z2))) return rc;
  hipError_t e = hipHostMalloc((void**)&D.host_result, 2 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) return set_error(MF_ENOMEM, hipGetErrorString(e));
  (void)m;
  return MF_OK;
}

// ---------------------------------------------------------------- coarse direct solve
// Dense inverse of the assembled interior block at a coarse level, summed
// from the same element matrices the kernels use.
int build_coarse_solver(mf_mesh* m, int level) {
  Level& L = m->levels[level];
  if (L.ncoarse > 0 || !L.cfirst.empty()) return MF_OK;
  const int dim = m->dim, d1 = dim + 1;
  const int N = L.N;
  const ElemTable ET = elem_table(dim);
  // unique ids of all storage points by key
  struct Ent {
    PointKey k;
    int64_t sidx;
    int32_t macro, x, y, z;
  };
  std::vector<Ent> ent;
  for (int64_t c = 0; c < m->nc; ++c) {
    const int zmax = dim == 3 ? N : 0;
    for (int z = 0; z <= zmax; ++z)
      for (int y = 0; y <= N - z; ++y)
        for (int x = 0; x <= N - z - y; ++x) {
          const int64_t s = L.base[c] + (dim == 2 ? idx2(N, x, y) : idx3(N, x, y, z));
          ent.push_back({point_key(dim, &m->cells[c * d1], N, x, y, z), s, (int32_t)c, x, y, z});
        }
  }
  std::sort(ent.begin(), ent.end(), [](const Ent& a, const Ent& b) {
    if (!(a.k == b.k)) return a.k < b.k;
    return a.sidx < b.sidx;
  });
  std::vector<int64_t> uid_of(L.storage, -1);
  std::vector<int64_t> unk_of_uid;  // -1 for Dirichlet
  int64_t nu = 0, nunk = 0;
  L.cfirst.clear();
  L.cptr.clear();
  L.cidx.clear();
  std::vector<std::vector<int64_t>> copies_of_unk;
  for (size_t i = 0; i < ent.size(); ++i) {
    if (i == 0 || !(ent[i].k == ent[i - 1].k)) {
      const int s = support_mask(dim, N, ent[i].x, ent[i].y, ent[i].z);
      const bool dir = (m->dir_mask[ent[i].macro] >> s) & 1;
      unk_of_uid.push_back(dir ? -1 : nunk);
      if (!dir) {
        copies_of_unk.emplace_back();
        ++nunk;
      }
      ++nu;
    }
    uid_of[ent[i].sidx] = nu - 1;
    const int64_t k = unk_of_uid[nu - 1];
    if (k >= 0) copies_of_unk[k].push_back(ent[i].sidx);
  }
  if (nunk > 4096) return set_error(MF_ENOTSUP, "coarse level has more than 4096 unknowns; choose a coarser level");
  std::vector<double> A((size_t)nunk * nunk, 0.0);
  for (int64_t c = 0; c < m->nc; ++c) {
    const MacroDev& M = L.md[c];
    const int zmax = dim == 3 ? N : 0;
    for (int az = 0; az <= zmax; ++az)
      for (int ay = 0; ay <= N; ++ay)
        for (int ax = 0; ax <= N; ++ax)
          for (int t = 0; t < ET.ntypes; ++t) {
            if (ax + ay + az > N - ET.slack[t]) continue;
            int64_t ids[4];
            for (int v = 0; v < ET.nv; ++v) {
              const int x = ax + ET.off[t][v][0], y = ay + ET.off[t][v][1], z = az + ET.off[t][v][2];
              const int64_t s = L.base[c] + (dim == 2 ? idx2(N, x, y) : idx3(N, x, y, z));
              ids[v] = unk_of_uid[uid_of[s]];
            }
            for (int v = 0; v < ET.nv; ++v)
              for (int u = 0; u < ET.nv; ++u)
                if (ids[v] >= 0 && ids[u] >= 0) A[ids[v] * nunk + ids[u]] += M.K[t][v * 4 + u];
          }
  }
  // Cholesky A = C C^T, then A^{-1} = C^{-T} C^{-1}
  const int64_t n = nunk;
  std::vector<double> C(A);
  for (int64_t j = 0; j < n; ++j) {
    double d = C[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= C[j * n + k] * C[j * n + k];
    if (!(d > 0.0)) return set_error(MF_ENUMERIC, "coarse operator is not positive definite");
    d = std::sqrt(d);
    C[j * n + j] = d;
    for (int64_t i = j + 1; i < n; ++i) {
      double s = C[i * n + j];
      for (int64_t k = 0; k < j; ++k) s -= C[i * n + k] * C[j * n + k];
      C[i * n + j] = s / d;
    }
  }
  std::vector<double> Ci((size_t)n * n, 0.0);  // C^{-1}, lower triangular
  for (int64_t col = 0; col < n; ++col)
    for (int64_t i = col; i < n; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int64_t k = col; k < i; ++k) s -= C[i * n + k] * Ci[k * n + col];
      Ci[i * n + col] = s / C[i * n + i];
    }
  L.cinv.assign((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      double s = 0.0;
      for (int64_t k = std::max(i, j); k < n; ++k) s += Ci[k * n + i] * Ci[k * n + j];
      L.cinv[i * n + j] = s;
    }
  L.cptr.push_back(0);
  for (int64_t k = 0; k < n; ++k) {
    L.cfirst.push_back((int32_t)copies_of_unk[k][0]);
    for (int64_t s : copies_of_unk[k]) L.cidx.push_back(s);
    L.cptr.push_back((int32_t)L.cidx.size());
  }
  L.ncoarse = n;
  if (m->host_only) return MF_OK;
  int rc;
  if ((rc = dev_upload(&L.dev.cinv, L.cinv))) return rc;
  std::vector<float> f(L.cinv.begin(), L.cinv.end());
  if ((rc = dev_upload(&L.dev.cinvf, f))) return rc;
  if ((rc = dev_upload(&L.dev.cfirst, L.cfirst))) return rc;
  if ((rc = dev_upload(&L.dev.cptr, L.cptr))) return rc;
  if ((rc = dev_upload(&L.dev.cidx, L.cidx))) return rc;
  return MF_OK;
}

// ---------------------------------------------------------------- whole mesh
int build_mesh(mf_mesh* m) {
  const int dim = m->dim, d1 = dim + 1;
  for (int64_t i = 0; i < m->nc * d1; ++i)
    if (m->cells[i] < 0 || m->cells[i] >= m->nv) return set_error(MF_EINVAL, "cell vertex id out of range");
  for (int64_t c = 0; c < m->nc; ++c) {
    const double* P0 = &m->coords[m->cells[c * d1] * dim];
    double J[3][3] = {{0}}, scale = 0.0;
    for (int k = 1; k <= dim; ++k)
      for (int r = 0; r < dim; ++r) {
        J[r][k - 1] = m->coords[m->cells[c * d1 + k] * dim + r] - P0[r];
        scale = std::max(scale, std::fabs(J[r][k - 1]));
      }
    double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                          : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 1e-14 * std::pow(scale, dim)))
      return set_error(MF_EINVAL, "degenerate macro cell " + std::to_string(c));
  }
  int rc = build_topology(m);
  if (rc) return rc;
  m->levels.resize(m->max_level + 1);
  for (int l = 0; l <= m->max_level; ++l)
    if ((rc = build_level(m, l, m->levels[l]))) return rc;
  if (!m->host_only) {
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
    for (int l = 0; l <= m->max_level; ++l)
      if ((rc = upload_level(m, m->levels[l]))) return rc;
  }
  return build_2d_tables(m);
}

void free_device(mf_mesh* m) {
  for (auto& L : m->levels) {
    LevelDev& D = L.dev;
    void* ptrs[] = {D.md, D.tiles, D.tiles_f32, D.segs, D.psegs, D.sbase, D.pruns, D.grp_ptr, D.copies, D.grp_flag, D.xgrp_ptr, D.xcopies, D.cpidx, D.xcpidx, D.xgrp_invdiag,
                    D.xgrp_invdiagf,
                    D.part, D.result, D.cinv, D.cinvf, D.cfirst, D.cptr, D.cidx, D.own_bits, D.p2_tiles};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    if (D.host_result) (void)hipHostFree(D.host_result);
    D = LevelDev{};
  }
  if (m->p2_dev) (void)hipFree(m->p2_dev);
  m->p2_dev = nullptr;
  if (m->geo2_dev) (void)hipFree(m->geo2_dev);
  m->geo2_dev = nullptr;
}

void storage_keys(const mf_mesh* m, int level, int64_t* vids, int32_t* wts) {
  const Level& L = m->levels[level];
  const int dim = m->dim, d1 = dim + 1;
  const int N = L.N;
  for (int64_t c = 0; c < m->nc; ++c) {
    const int zmax = dim == 3 ? N : 0;
    for (int z = 0; z <= zmax; ++z)
      for (int y = 0; y <= N - z; ++y)
        for (int x = 0; x <= N - z - y; ++x) {
          const int64_t s = L.base[c] + (dim == 2 ? idx2(N, x, y) : idx3(N, x, y, z));
          const PointKey k = point_key(dim, &m->cells[c * d1], N, x, y, z);
          for (int i = 0; i < d1; ++i) {
            vids[s * d1 + i] = k.v[i];
            wts[s * d1 + i] = k.w[i];
          }
        }
  }
}

}  // namespace mf
