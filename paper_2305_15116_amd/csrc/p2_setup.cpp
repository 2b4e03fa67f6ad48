// Host set-up of the 2D-only operators: the P2 operator's per-macro element
// matrix, interior stencils and wave tiles, and the macro geometry the
// blended apply maps its lattice with.
//
// The paper's P2 discretisation (vertex and edge-midpoint DoFs) is applied in
// HyTeG by four kernels (vertex-to-vertex, edge-to-vertex, vertex-to-edge,
// edge-to-edge, Performance Modeling section), each reading its source array
// and updating its destination array; with one array holding both DoF kinds
// (p2.hpp) the four become one stencil per DoF class.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "mesh.hpp"

namespace mf {

namespace {

// Element stiffness of the quadratic triangle with edge vectors E[.][0] =
// P1 - P0 and E[.][1] = P2 - P0, local order v0 v1 v2 m01 m12 m02.  With
// barycentric gradients g_i, basis lambda_i (2 lambda_i - 1) at the vertices
// and 4 lambda_a lambda_b at the midpoints, and the exact integrals
// int lambda_a = |T|/3, int lambda_a lambda_b = |T| (1 + [a == b]) / 12:
//   vertex-vertex  K_ii = |T| g_i.g_i,  K_ik = -|T| g_i.g_k / 3
//   vertex-edge    K_i,ab = 4|T|/3 ([i == b] g_i.g_a + [i == a] g_i.g_b)
//   edge-edge      K_ab,cd = 4|T|/3 (g_a.g_c (1+[b==d]) + g_a.g_d (1+[b==c])
//                                    + g_b.g_c (1+[a==d]) + g_b.g_d (1+[a==c]))
bool p2_element_matrix(const double E[2][2], double K[6][6]) {
  const double det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
  if (det == 0.0) return false;
  double g[3][2];
  g[1][0] = E[1][1] / det;
  g[1][1] = -E[0][1] / det;
  g[2][0] = -E[1][0] / det;
  g[2][1] = E[0][0] / det;
  g[0][0] = -(g[1][0] + g[2][0]);
  g[0][1] = -(g[1][1] + g[2][1]);
  const double area = std::fabs(det) / 2.0;
  auto dot = [&](int i, int k) { return g[i][0] * g[k][0] + g[i][1] * g[k][1]; };
  const int ea[3] = {0, 1, 0}, eb[3] = {1, 2, 2};
  const double c43 = 4.0 * area / 3.0;
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) K[i][k] = i == k ? area * dot(i, i) : -area * dot(i, k) / 3.0;
  for (int i = 0; i < 3; ++i)
    for (int e = 0; e < 3; ++e) {
      const int a = ea[e], b = eb[e];
      const double v = c43 * ((i == b ? dot(i, a) : 0.0) + (i == a ? dot(i, b) : 0.0));
      K[i][3 + e] = v;
      K[3 + e][i] = v;
    }
  for (int e = 0; e < 3; ++e)
    for (int f = 0; f < 3; ++f) {
      const int a = ea[e], b = eb[e], c = ea[f], d = eb[f];
      K[3 + e][3 + f] = c43 * (dot(a, c) * (1 + (b == d)) + dot(a, d) * (1 + (b == c)) + dot(b, c) * (1 + (a == d)) +
                               dot(b, d) * (1 + (a == c)));
    }
  return true;
}

// Fine-lattice points of the up / down micro-triangle with coarse anchor
// (a, b), in the local order of the element matrix.
void tri_points(bool up, int a, int b, int px[6], int py[6]) {
  if (up) {
    px[0] = 2 * a;     py[0] = 2 * b;
    px[1] = 2 * a + 2; py[1] = 2 * b;
    px[2] = 2 * a;     py[2] = 2 * b + 2;
  } else {
    px[0] = 2 * a + 2; py[0] = 2 * b + 2;
    px[1] = 2 * a;     py[1] = 2 * b + 2;
    px[2] = 2 * a + 2; py[2] = 2 * b;
  }
  const int ea[3] = {0, 1, 0}, eb[3] = {1, 2, 2};
  for (int e = 0; e < 3; ++e) {
    px[3 + e] = (px[ea[e]] + px[eb[e]]) / 2;
    py[3 + e] = (py[ea[e]] + py[eb[e]]) / 2;
  }
}

// Interior stencil of DoF class (cx, cy) (parities of the fine coordinates):
// the sum of the element-matrix rows of every micro-triangle around a point
// of that class, keyed by neighbour offset.
std::map<std::pair<int, int>, double> class_stencil(const double K[6][6], int cx, int cy) {
  std::map<std::pair<int, int>, double> w;
  const int X = 8 + cx, Y = 8 + cy;
  for (int b = 0; b <= 8; ++b)
    for (int a = 0; a <= 8; ++a)
      for (int up = 1; up >= 0; --up) {
        int px[6], py[6];
        tri_points(up != 0, a, b, px, py);
        for (int lp = 0; lp < 6; ++lp)
          if (px[lp] == X && py[lp] == Y)
            for (int q = 0; q < 6; ++q) w[{px[q] - X, py[q] - Y}] += K[lp][q];
      }
  return w;
}

struct ClassLayout {
  int cx, cy, first, n;
  int d[5][2];  // representative offsets after the centre
};

// Weight slots of P2Macro::w (see p2.hpp).
const ClassLayout kVertexLayout = {0, 0, 0, 10, {{2, 0}, {0, 2}, {2, -2}, {1, 0}, {0, 1}}};
const int kVertexMore[4][2] = {{1, -1}, {1, 1}, {2, -1}, {1, -2}};
const ClassLayout kEdgeLayouts[3] = {
    {1, 0, 10, 5, {{1, 0}, {0, 1}, {-1, 1}, {-1, 2}, {0, 0}}},
    {0, 1, 15, 5, {{0, 1}, {2, -1}, {1, -1}, {1, 0}, {0, 0}}},
    {1, 1, 20, 5, {{1, 1}, {1, -1}, {0, 1}, {1, 0}, {0, 0}}},
};

// Fills w[first ..] of one class from its stencil map; every offset of the
// map must be the centre or one of the listed pairs, and opposite neighbours
// must carry the same weight (to rounding).
int fill_class(const std::map<std::pair<int, int>, double>& st, int first, int n, const int (*d)[2], double scale,
               double* w) {
  int used = 0;
  auto get = [&](int dx, int dy, double& v) {
    auto it = st.find({dx, dy});
    v = it == st.end() ? 0.0 : it->second;
    return it != st.end();
  };
  double c;
  used += get(0, 0, c);
  w[first] = c;
  for (int k = 1; k < n; ++k) {
    double p, q;
    const bool hp = get(d[k - 1][0], d[k - 1][1], p), hq = get(-d[k - 1][0], -d[k - 1][1], q);
    if (hp != hq || std::fabs(p - q) > 1e-12 * scale)
      return set_error(MF_ENUMERIC, "P2 stencil is not centrally symmetric");
    used += hp + hq;
    w[first + k] = p;
  }
  if (used != (int)st.size()) return set_error(MF_ENUMERIC, "P2 stencil has an unexpected neighbour");
  return MF_OK;
}

}  // namespace

int build_2d_tables(mf_mesh* m) {
  if (m->dim != 2) return MF_OK;
  m->geo2.assign(m->nc, Geo2{});
  for (int64_t c = 0; c < m->nc; ++c) {
    const double* P0 = &m->coords[m->cells[c * 3] * 2];
    const double* P1 = &m->coords[m->cells[c * 3 + 1] * 2];
    const double* P2 = &m->coords[m->cells[c * 3 + 2] * 2];
    for (int r = 0; r < 2; ++r) {
      m->geo2[c].p0[r] = P0[r];
      m->geo2[c].e1[r] = P1[r] - P0[r];
      m->geo2[c].e2[r] = P2[r] - P0[r];
    }
  }
  m->p2.assign(m->nc, P2Macro{});
  for (int64_t c = 0; c < m->nc; ++c) {
    const double* P0 = &m->coords[m->cells[c * 3] * 2];
    double E[2][2];
    for (int k = 1; k <= 2; ++k)
      for (int r = 0; r < 2; ++r) E[r][k - 1] = m->coords[m->cells[c * 3 + k] * 2 + r] - P0[r];
    double K[6][6];
    if (!p2_element_matrix(E, K)) return set_error(MF_EINVAL, "degenerate macro cell " + std::to_string(c));
    P2Macro& P = m->p2[c];
    double scale = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        P.K[i * 6 + j] = K[i][j];
        P.Kf[i * 6 + j] = (float)K[i][j];
        scale = std::max(scale, std::fabs(K[i][j]));
      }
    // vertex class: 10 slots, the first five pairs from the layout, the rest below
    int vd[9][2];
    for (int k = 0; k < 5; ++k) {
      vd[k][0] = kVertexLayout.d[k][0];
      vd[k][1] = kVertexLayout.d[k][1];
    }
    for (int k = 0; k < 4; ++k) {
      vd[5 + k][0] = kVertexMore[k][0];
      vd[5 + k][1] = kVertexMore[k][1];
    }
    int rc = fill_class(class_stencil(K, 0, 0), kVertexLayout.first, kVertexLayout.n, vd, scale, P.w);
    if (rc) return rc;
    for (const ClassLayout& L : kEdgeLayouts)
      if ((rc = fill_class(class_stencil(K, L.cx, L.cy), L.first, L.n, L.d, scale, P.w))) return rc;
    for (int k = 0; k < kP2Weights; ++k) P.wf[k] = (float)P.w[k];
  }
  // wave tiles: P2 of level l walks the lattice of level l + 1
  for (Level& L : m->levels) {
    L.p2_tiles.clear();
    if (L.level < 1) continue;
    const int M = L.N;
    for (int64_t c = 0; c < m->nc; ++c)
      for (int y0 = 0; y0 < M; y0 += kP2H)
        for (int x0 = 0; x0 + y0 < M; x0 += kP2TileW) L.p2_tiles.push_back({(int32_t)c, x0, y0, 0});
    while (L.p2_tiles.size() % kWavesPerWG) L.p2_tiles.push_back({-1, 0, 0, 0});
  }
  if (m->host_only) return MF_OK;
  int rc = dev_upload(&m->p2_dev, m->p2);
  if (!rc) rc = dev_upload(&m->geo2_dev, m->geo2);
  if (rc) return rc;
  for (Level& L : m->levels)
    if ((rc = dev_upload(&L.dev.p2_tiles, L.p2_tiles))) return rc;
  return MF_OK;
}

}  // namespace mf
