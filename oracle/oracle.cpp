// Oracle for the P1 (and 2D P2) matrix-free operators — TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously correct CPU FP64 code.  Only the test-suite, the
// smoke check and the CPU-baseline leg of the benchmark may load this library;
// the product path never does, and nothing here is shared with the HIP path.
//
// What it computes is the plain definition of the result: the assembled P1
// stiffness matrix of the uniformly refined macro mesh, stored in compressed
// row storage (Intro, "Sparse Matrices"; PETSc comparison section, where the
// sparse and matrix-free variants do the same flops on the same rows), times a
// vector.  The matrix-free method of the paper reaches the same rows because
// every interior row of a macro is the same stencil (Intro, "Hybrid
// Tetrahedral Grids").
//
// Steps, in the order they are written below:
//  1. Refinement by exact integer keys.  A lattice point of a macro with
//     vertices (v0..vd) and index-space coordinates p (p >= 0, sum p <= N,
//     N = 2^level) has barycentric integer weights (N - sum p, p1, .., pd).
//     Its key is the list of (global vertex id, weight) pairs with non-zero
//     weight, sorted by vertex id; the same point seen from any macro has the
//     same key, so keys identify unique DoFs with no floating point involved.
//  2. Micro-elements, enumerated in index space.  2D: "up" triangles
//     a+{0,e1,e2} and "down" triangles a+{e1,e1+e2,e2}.  3D: "up" tets
//     a+{0,e1,e2,e3}; an octahedron split into four tets around its
//     (0,1,0)-(1,0,1) diagonal; "down" tets a+{(1,1,0),(1,0,1),(0,1,1),(1,1,1)}.
//     This is Bey's tetrahedral refinement written in index space (the paper
//     is 2D only and leaves 3D to future work, Conclusion and Outlook).
//  3. Element stiffness K = |T| G^T G from the physical micro-element edge
//     vectors, G = barycentric gradients (solve with the edge vectors).
//  4. Assembly COO -> CSR, duplicates summed, explicit zeros kept.
//  5. Dirichlet boundary: DoFs on macro facets with exactly one adjacent cell
//     get identity rows; other rows keep their boundary columns.
//  6. y = A x as a row loop.
// Also: the 2D P2 stiffness matrix (vertex and edge DoFs) by the same steps
// with quadratic elements, the variable-coefficient P1 matrix, the P1 matrix
// of blended (non-affine) 2D macros, the same rows evaluated for a sample of points without a global
// build (for full-size checks), the P1 prolongation between two levels, the
// lumped mass vector, and the keyed SplitMix64 input generator.

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>
#include <omp.h>

namespace {

thread_local std::string g_err;

constexpr int MAXV = 4;

struct Key {
  int64_t v[MAXV];
  int32_t w[MAXV];
};

bool key_less(const Key& a, const Key& b) {
  for (int k = 0; k < MAXV; ++k) {
    if (a.v[k] != b.v[k]) return a.v[k] < b.v[k];
    if (a.w[k] != b.w[k]) return a.w[k] < b.w[k];
  }
  return false;
}

bool key_eq(const Key& a, const Key& b) {
  for (int k = 0; k < MAXV; ++k)
    if (a.v[k] != b.v[k] || a.w[k] != b.w[k]) return false;
  return true;
}

// Key of the point with barycentric weights wts (in the cell's vertex order).
Key make_key(int dim, const int64_t* cellv, const int64_t* wts) {
  std::array<std::pair<int64_t, int64_t>, MAXV> pr;
  int n = 0;
  for (int k = 0; k <= dim; ++k)
    if (wts[k] != 0) pr[n++] = {cellv[k], wts[k]};
  std::sort(pr.begin(), pr.begin() + n);
  Key key;
  for (int k = 0; k < MAXV; ++k) {
    key.v[k] = k < n ? pr[k].first : -1;
    key.w[k] = k < n ? (int32_t)pr[k].second : 0;
  }
  return key;
}

// Barycentric weights of index-space point p in a macro of N intervals.
void weights_of(int dim, int64_t N, const int64_t* p, int64_t* w) {
  int64_t s = 0;
  for (int k = 0; k < dim; ++k) { w[k + 1] = p[k]; s += p[k]; }
  w[0] = N - s;
}

// ---- SplitMix64 (Steele, Lea, Flood: "Fast splittable pseudorandom number
// generators", OOPSLA 2014), used as a counter-based hash of a point key.
uint64_t sm64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// x(key) = 2u - 1, u = top 53 bits of the chained hash, in [0, 1).
double keyed_value(uint64_t seed, const Key& k) {
  uint64_t h = sm64(seed);
  for (int i = 0; i < MAXV; ++i) {
    if (k.v[i] < 0) break;
    h = sm64(h ^ (((uint64_t)k.v[i] << 24) | (uint64_t)(uint32_t)k.w[i]));
  }
  double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u - 1.0;
}

// ---- Step 2: micro-element enumeration in index space.
// Calls fn(verts) for every micro-element whose anchor lies in the box
// [lo, hi] (inclusive, clipped to >= 0); verts holds dim+1 index-space points.
template <class F>
void for_each_element(int dim, int64_t N, const int64_t* lo, const int64_t* hi, F&& fn) {
  int64_t v[MAXV][3];
  if (dim == 2) {
    for (int64_t y = std::max<int64_t>(lo[1], 0); y <= hi[1]; ++y)
      for (int64_t x = std::max<int64_t>(lo[0], 0); x <= hi[0]; ++x) {
        if (x + y <= N - 1) {  // up triangle a, a+e1, a+e2
          int64_t t[3][3] = {{x, y, 0}, {x + 1, y, 0}, {x, y + 1, 0}};
          std::memcpy(v, t, sizeof(t));
          fn(v);
        }
        if (x + y <= N - 2) {  // down triangle a+e1, a+e1+e2, a+e2
          int64_t t[3][3] = {{x + 1, y, 0}, {x + 1, y + 1, 0}, {x, y + 1, 0}};
          std::memcpy(v, t, sizeof(t));
          fn(v);
        }
      }
    return;
  }
  for (int64_t z = std::max<int64_t>(lo[2], 0); z <= hi[2]; ++z)
    for (int64_t y = std::max<int64_t>(lo[1], 0); y <= hi[1]; ++y)
      for (int64_t x = std::max<int64_t>(lo[0], 0); x <= hi[0]; ++x) {
        const int64_t s = x + y + z;
        if (s <= N - 1) {  // up tet
          int64_t t[4][3] = {{x, y, z}, {x + 1, y, z}, {x, y + 1, z}, {x, y, z + 1}};
          std::memcpy(v, t, sizeof(t));
          fn(v);
        }
        if (s <= N - 2) {  // octahedron split around d0=(x,y+1,z) -- d1=(x+1,y,z+1)
          const int64_t d0[3] = {x, y + 1, z}, d1[3] = {x + 1, y, z + 1};
          const int64_t ring[4][3] = {{x + 1, y, z}, {x + 1, y + 1, z}, {x, y + 1, z + 1}, {x, y, z + 1}};
          for (int k = 0; k < 4; ++k) {
            const int64_t* a = ring[k];
            const int64_t* b = ring[(k + 1) % 4];
            int64_t t[4][3] = {{d0[0], d0[1], d0[2]}, {d1[0], d1[1], d1[2]},
                               {a[0], a[1], a[2]}, {b[0], b[1], b[2]}};
            std::memcpy(v, t, sizeof(t));
            fn(v);
          }
        }
        if (s <= N - 3) {  // down tet
          int64_t t[4][3] = {{x + 1, y + 1, z}, {x + 1, y, z + 1}, {x, y + 1, z + 1}, {x + 1, y + 1, z + 1}};
          std::memcpy(v, t, sizeof(t));
          fn(v);
        }
      }
}

// ---- Step 3: element stiffness from physical vertex coordinates.
// Edge vectors X_k - X_0 are formed from the exact integer differences of the
// vertices' barycentric weights, sum_j ((w_kj - w_0j) / N) P_j, so that they
// carry full relative precision at any level (subtracting two absolute
// coordinates would lose about log10(N) digits to cancellation).
void edge_matrix(int dim, const double* coords, const int64_t* cellv, int64_t N, int64_t (*v)[3],
                 double E[3][3]) {
  int64_t w0[MAXV];
  weights_of(dim, N, v[0], w0);
  for (int c = 0; c < 3; ++c)
    for (int r = 0; r < 3; ++r) E[r][c] = 0.0;
  for (int c = 0; c < dim; ++c) {
    int64_t wk[MAXV];
    weights_of(dim, N, v[c + 1], wk);
    for (int r = 0; r < dim; ++r) {
      double s = 0.0;
      for (int j = 0; j <= dim; ++j) s += ((double)(wk[j] - w0[j]) / (double)N) * coords[cellv[j] * dim + r];
      E[r][c] = s;
    }
  }
}

// Edge vectors of a micro-triangle of a blended 2D macro (map F = affine
// part + xi0 xi1 xi2 d, xi = lattice point / N): the affine part as in
// edge_matrix, plus d times the difference of the bubble between the two
// lattice points.  The bubble at (i, j) is n(i, j) / N^3 with the integer
// n(i, j) = (N - i - j) i j, so the difference is formed exactly in integers
// and divided once: no O(1) mapped coordinates are subtracted from each other.
void blended_edge_matrix(const double* coords, const int64_t* cellv, int64_t N, const double* d, int64_t (*v)[3],
                         double E[3][3]) {
  edge_matrix(2, coords, cellv, N, v, E);
  auto n = [N](const int64_t* p) { return (N - p[0] - p[1]) * p[0] * p[1]; };
  const double N3 = (double)N * (double)N * (double)N;
  for (int k = 0; k < 2; ++k) {
    const double db = (double)(n(v[k + 1]) - n(v[0])) / N3;
    for (int r = 0; r < 2; ++r) E[r][k] += db * d[r];
  }
}

// E = [X1-X0 | .. | Xd-X0]; lambda_{1..d} = E^{-1}(x - X0), so grad lambda_k
// is row k of E^{-1}; grad lambda_0 = -sum of the others; |T| = |det E| / d!.
// Returns false for a degenerate element.
bool element_stiffness(int dim, const double E[3][3], double K[MAXV][MAXV], double* vol) {
  double inv[3][3] = {{0}};
  double det;
  if (dim == 2) {
    det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
    if (det == 0.0) return false;
    inv[0][0] = E[1][1] / det;  inv[0][1] = -E[0][1] / det;
    inv[1][0] = -E[1][0] / det; inv[1][1] = E[0][0] / det;
  } else {
    const double c00 = E[1][1] * E[2][2] - E[1][2] * E[2][1];
    const double c01 = E[1][2] * E[2][0] - E[1][0] * E[2][2];
    const double c02 = E[1][0] * E[2][1] - E[1][1] * E[2][0];
    det = E[0][0] * c00 + E[0][1] * c01 + E[0][2] * c02;
    if (det == 0.0) return false;
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
    inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    inv[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
    inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    inv[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
    inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
  }
  double G[MAXV][3] = {{0}};
  for (int k = 0; k < dim; ++k)
    for (int r = 0; r < dim; ++r) G[k + 1][r] = inv[k][r];
  for (int r = 0; r < dim; ++r) {
    double s = 0.0;
    for (int k = 1; k <= dim; ++k) s += G[k][r];
    G[0][r] = -s;
  }
  const double v = std::fabs(det) / (dim == 2 ? 2.0 : 6.0);
  for (int i = 0; i <= dim; ++i)
    for (int j = 0; j <= dim; ++j) {
      double s = 0.0;
      for (int r = 0; r < dim; ++r) s += G[i][r] * G[j][r];
      K[i][j] = v * s;
    }
  *vol = v;
  return true;
}

// ---- Macro topology: facet counts and the boundary sub-simplices.
struct Topology {
  std::set<std::vector<int64_t>> boundary_subsets;  // every non-empty subset of a boundary facet
  std::map<std::vector<int64_t>, int64_t> cell_of_vertexset;
  bool ok = true;
};

Topology build_topology(int dim, int64_t nc, const int64_t* cells) {
  Topology t;
  std::map<std::vector<int64_t>, int> facet_count;
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t* cv = cells + c * (dim + 1);
    std::vector<int64_t> all(cv, cv + dim + 1);
    std::sort(all.begin(), all.end());
    for (int k = 0; k < dim; ++k)
      if (all[k] == all[k + 1]) { t.ok = false; g_err = "cell with repeated vertex"; return t; }
    if (t.cell_of_vertexset.count(all)) { t.ok = false; g_err = "duplicate cell"; return t; }
    t.cell_of_vertexset[all] = c;
    for (int skip = 0; skip <= dim; ++skip) {
      std::vector<int64_t> f;
      for (int k = 0; k <= dim; ++k) if (k != skip) f.push_back(all[k]);
      facet_count[f] += 1;
    }
  }
  for (auto& kv : facet_count) {
    if (kv.second > 2) { t.ok = false; g_err = "non-conforming: facet shared by more than two cells"; return t; }
    if (kv.second == 1) {
      const auto& f = kv.first;
      const int n = (int)f.size();
      for (int m = 1; m < (1 << n); ++m) {
        std::vector<int64_t> s;
        for (int k = 0; k < n; ++k) if (m & (1 << k)) s.push_back(f[k]);
        t.boundary_subsets.insert(s);
      }
    }
  }
  return t;
}

std::vector<int64_t> support_of(const Key& k) {
  std::vector<int64_t> s;
  for (int i = 0; i < MAXV; ++i) if (k.v[i] >= 0) s.push_back(k.v[i]);
  return s;
}

// Position of point p (index space) in a macro's dense (N+1)^dim lattice array.
inline int64_t lat_index(int dim, int64_t N, const int64_t* p) {
  const int64_t n1 = N + 1;
  return dim == 2 ? p[1] * n1 + p[0] : (p[2] * n1 + p[1]) * n1 + p[0];
}

}  // namespace

struct or_mesh {
  int dim = 0, level = 0;
  int64_t N = 0, nv = 0, nc = 0;
  std::vector<double> coords;
  std::vector<int64_t> cells;
  int64_t nu = 0;
  std::vector<Key> keys;          // sorted unique keys; uid = position
  std::vector<double> xyz;        // nu * dim
  std::vector<int8_t> bnd;        // Dirichlet (domain boundary) flag
  std::vector<int64_t> lat;       // per cell dense (N+1)^dim -> uid, -1 outside the simplex
  int64_t lat_stride = 0;
  // CSR (after or_assemble)
  int csr_dirichlet = -1;
  std::vector<int64_t> rowptr, cols;
  std::vector<double> vals;
};

namespace {

template <class F>
void for_each_cell_element(const or_mesh* m, int64_t c, F&& fn) {
  const int64_t lo[3] = {0, 0, 0};
  const int64_t hi[3] = {m->N, m->N, m->N};
  for_each_element(m->dim, m->N, lo, hi, fn);
  (void)c;
}

}  // namespace

extern "C" {

const char* or_last_error(void) { return g_err.c_str(); }

// The SplitMix64 output function on state z (exported so tests can pin it to
// the generator's published output sequence).
uint64_t or_splitmix64(uint64_t z) { return sm64(z); }

// Step 1 over the whole mesh: keys, unique ids, coordinates, Dirichlet flags.
or_mesh* or_build(int dim, int64_t nv, const double* coords, int64_t nc, const int64_t* cells, int level) {
  if (dim != 2 && dim != 3) { g_err = "dim must be 2 or 3"; return nullptr; }
  if (level < 0 || level > 14) { g_err = "level out of range"; return nullptr; }
  for (int64_t i = 0; i < nc * (dim + 1); ++i)
    if (cells[i] < 0 || cells[i] >= nv) { g_err = "cell vertex id out of range"; return nullptr; }
  Topology topo = build_topology(dim, nc, cells);
  if (!topo.ok) return nullptr;
  or_mesh* m = new or_mesh;
  m->dim = dim; m->level = level; m->N = int64_t(1) << level; m->nv = nv; m->nc = nc;
  m->coords.assign(coords, coords + nv * dim);
  m->cells.assign(cells, cells + nc * (dim + 1));
  const int64_t N = m->N, n1 = N + 1;
  m->lat_stride = dim == 2 ? n1 * n1 : n1 * n1 * n1;
  m->lat.assign((size_t)(m->lat_stride * nc), -1);

  struct Entry { Key k; int64_t slot; };
  std::vector<Entry> ent;
  for (int64_t c = 0; c < nc; ++c) {
    const int64_t* cv = &m->cells[c * (dim + 1)];
    int64_t p[3] = {0, 0, 0}, w[MAXV];
    const int64_t zmax = dim == 3 ? N : 0;
    for (p[2] = 0; p[2] <= zmax; ++p[2])
      for (p[1] = 0; p[1] + p[2] <= N; ++p[1])
        for (p[0] = 0; p[0] + p[1] + p[2] <= N; ++p[0]) {
          weights_of(dim, N, p, w);
          ent.push_back({make_key(dim, cv, w), c * m->lat_stride + lat_index(dim, N, p)});
        }
  }
  std::sort(ent.begin(), ent.end(), [](const Entry& a, const Entry& b) { return key_less(a.k, b.k); });
  int64_t uid = -1;
  for (size_t i = 0; i < ent.size(); ++i) {
    if (i == 0 || !key_eq(ent[i].k, ent[i - 1].k)) {
      ++uid;
      m->keys.push_back(ent[i].k);
    }
    m->lat[ent[i].slot] = uid;
  }
  m->nu = uid + 1;
  std::vector<Entry>().swap(ent);

  m->xyz.assign(m->nu * dim, 0.0);
  m->bnd.assign(m->nu, 0);
  for (int64_t u = 0; u < m->nu; ++u) {
    const Key& k = m->keys[u];
    for (int r = 0; r < dim; ++r) {
      double s = 0.0;
      for (int i = 0; i < MAXV; ++i)
        if (k.v[i] >= 0) s += ((double)k.w[i] / (double)N) * coords[k.v[i] * dim + r];
      m->xyz[u * dim + r] = s;
    }
    std::vector<int64_t> sup = support_of(k);
    if ((int)sup.size() <= dim && topo.boundary_subsets.count(sup)) m->bnd[u] = 1;
  }
  return m;
}

void or_free(or_mesh* m) { delete m; }
int64_t or_num_unique(const or_mesh* m) { return m->nu; }

void or_get_keys(const or_mesh* m, int64_t* vids, int32_t* wts) {
  const int d1 = m->dim + 1;
  for (int64_t u = 0; u < m->nu; ++u)
    for (int i = 0; i < d1; ++i) {
      vids[u * d1 + i] = m->keys[u].v[i];
      wts[u * d1 + i] = m->keys[u].w[i];
    }
}

void or_get_coords(const or_mesh* m, double* xyz) { std::memcpy(xyz, m->xyz.data(), sizeof(double) * m->xyz.size()); }
void or_get_boundary(const or_mesh* m, int8_t* flag) { std::memcpy(flag, m->bnd.data(), m->bnd.size()); }

void or_keyed_random(const or_mesh* m, uint64_t seed, double* x) {
  for (int64_t u = 0; u < m->nu; ++u) x[u] = keyed_value(seed, m->keys[u]);
}

// Micro-elements as unique-id tuples (ne x (dim+1)); returns ne.  Pass null to count.
int64_t or_elements(const or_mesh* m, int64_t* out) {
  int64_t ne = 0;
  const int d1 = m->dim + 1;
  for (int64_t c = 0; c < m->nc; ++c) {
    const int64_t* L = &m->lat[c * m->lat_stride];
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      if (out)
        for (int i = 0; i < d1; ++i) out[ne * d1 + i] = L[lat_index(m->dim, m->N, v[i])];
      ++ne;
    });
  }
  return ne;
}

namespace {
// Edge matrix of a micro-element and the unique ids of its vertices.
void element_data(const or_mesh* m, int64_t c, int64_t (*v)[3], double E[3][3], int64_t* ids) {
  const int64_t* cv = &m->cells[c * (m->dim + 1)];
  const int64_t* L = &m->lat[c * m->lat_stride];
  edge_matrix(m->dim, m->coords.data(), cv, m->N, v, E);
  for (int i = 0; i <= m->dim; ++i) ids[i] = L[lat_index(m->dim, m->N, v[i])];
}
}  // namespace

// Steps 3-5: CSR assembly.  dirichlet != 0 replaces boundary rows by identity rows.
// Returns nnz, or -1 on a degenerate element.
int64_t or_assemble(or_mesh* m, int dirichlet) {
  const int d1 = m->dim + 1;
  std::vector<int64_t> cnt(m->nu + 1, 0);
  for (int64_t c = 0; c < m->nc; ++c) {
    const int64_t* L = &m->lat[c * m->lat_stride];
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      for (int i = 0; i < d1; ++i) cnt[L[lat_index(m->dim, m->N, v[i])] + 1] += d1;
    });
  }
  for (int64_t u = 0; u < m->nu; ++u) cnt[u + 1] += cnt[u];
  std::vector<int64_t> ccol(cnt[m->nu]);
  std::vector<double> cval(cnt[m->nu]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      double E[3][3], K[MAXV][MAXV], vol;
      int64_t ids[MAXV];
      element_data(m, c, v, E, ids);
      if (!element_stiffness(m->dim, E, K, &vol)) { bad = true; return; }
      for (int i = 0; i < d1; ++i)
        for (int j = 0; j < d1; ++j) {
          const int64_t at = fill[ids[i]]++;
          ccol[at] = ids[j];
          cval[at] = K[i][j];
        }
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  m->rowptr.assign(m->nu + 1, 0);
  m->cols.clear();
  m->vals.clear();
  std::vector<std::pair<int64_t, double>> row;
  for (int64_t u = 0; u < m->nu; ++u) {
    if (dirichlet && m->bnd[u]) {
      m->cols.push_back(u);
      m->vals.push_back(1.0);
    } else {
      row.clear();
      for (int64_t k = cnt[u]; k < cnt[u + 1]; ++k) row.push_back({ccol[k], cval[k]});
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
      for (size_t k = 0; k < row.size(); ++k) {
        if (k > 0 && row[k].first == row[k - 1].first) m->vals.back() += row[k].second;
        else { m->cols.push_back(row[k].first); m->vals.push_back(row[k].second); }
      }
    }
    m->rowptr[u + 1] = (int64_t)m->cols.size();
  }
  m->csr_dirichlet = dirichlet ? 1 : 0;
  return (int64_t)m->cols.size();
}

// ---- Variable coefficient (the paper notes that varying weights can be
// computed on the fly, trading memory traffic for computation, comparison of
// matrix-free and sparse storage).  Operator: a(u, v) = integral of k grad u . grad v with k the P1
// interpolant of nodal values; grad u . grad v is constant on a P1 element,
// so the element matrix is exactly (mean of k over the element's vertices)
// times the constant-coefficient element matrix.  k is given per unique DoF.
// Same assembly as or_assemble otherwise.  Returns nnz, or -1.
int64_t or_assemble_varcoef(or_mesh* m, int dirichlet, const double* k) {
  const int d1 = m->dim + 1;
  std::vector<std::vector<std::pair<int64_t, double>>> rows(m->nu);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      double E[3][3], K[MAXV][MAXV], vol;
      int64_t ids[MAXV];
      element_data(m, c, v, E, ids);
      if (!element_stiffness(m->dim, E, K, &vol)) { bad = true; return; }
      double kt = 0.0;
      for (int i = 0; i < d1; ++i) kt += k[ids[i]];
      kt /= (double)d1;
      for (int i = 0; i < d1; ++i)
        for (int j = 0; j < d1; ++j) rows[ids[i]].push_back({ids[j], kt * K[i][j]});
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  m->rowptr.assign(m->nu + 1, 0);
  m->cols.clear();
  m->vals.clear();
  for (int64_t u = 0; u < m->nu; ++u) {
    if (dirichlet && m->bnd[u]) {
      m->cols.push_back(u);
      m->vals.push_back(1.0);
    } else {
      auto& row = rows[u];
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
      for (size_t q = 0; q < row.size(); ++q) {
        if (q > 0 && row[q].first == row[q - 1].first) m->vals.back() += row[q].second;
        else { m->cols.push_back(row[q].first); m->vals.push_back(row[q].second); }
      }
    }
    m->rowptr[u + 1] = (int64_t)m->cols.size();
  }
  m->csr_dirichlet = dirichlet ? 5 : 4;
  return (int64_t)m->cols.size();
}

// ---- Blended (non-affine) macros in 2D (the same remark of the paper on
// stencils computed on the fly: geometry that varies inside a macro, so no
// two rows share a stencil).
// Reading: macro c maps reference coordinates xi (lattice point / N) by
//   F(xi) = P0 + (P1 - P0) xi1 + (P2 - P0) xi2 + xi0 xi1 xi2 d_c,
// xi0 = 1 - xi1 - xi2, with a per-macro vector d_c.  The cubic bubble
// vanishes on the macro's edges, so neighbouring macros agree on every shared
// point.  Micro-triangles are the straight triangles on the mapped lattice
// points; the operator is the P1 stiffness matrix of that micro mesh.
// d holds nc x 2 values.  Returns nnz, or -1.
int64_t or_assemble_blended(or_mesh* m, int dirichlet, const double* d) {
  if (m->dim != 2) { g_err = "blended macros are 2D"; return -1; }
  const int64_t N = m->N;
  std::vector<std::vector<std::pair<int64_t, double>>> rows(m->nu);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    const int64_t* cv = &m->cells[c * 3];
    const int64_t* L = &m->lat[c * m->lat_stride];
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      double E[3][3];
      blended_edge_matrix(m->coords.data(), cv, N, &d[c * 2], v, E);
      double K[MAXV][MAXV], vol;
      if (!element_stiffness(2, E, K, &vol)) { bad = true; return; }
      int64_t ids[3];
      for (int i = 0; i < 3; ++i) ids[i] = L[lat_index(2, N, v[i])];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) rows[ids[i]].push_back({ids[j], K[i][j]});
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  m->rowptr.assign(m->nu + 1, 0);
  m->cols.clear();
  m->vals.clear();
  for (int64_t u = 0; u < m->nu; ++u) {
    if (dirichlet && m->bnd[u]) {
      m->cols.push_back(u);
      m->vals.push_back(1.0);
    } else {
      auto& row = rows[u];
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
      for (size_t q = 0; q < row.size(); ++q) {
        if (q > 0 && row[q].first == row[q - 1].first) m->vals.back() += row[q].second;
        else { m->cols.push_back(row[q].first); m->vals.push_back(row[q].second); }
      }
    }
    m->rowptr[u + 1] = (int64_t)m->cols.size();
  }
  m->csr_dirichlet = dirichlet ? 7 : 6;
  return (int64_t)m->cols.size();
}

// ---- P2 (quadratic) elements in 2D: the paper's own discretisation, with a
// DoF at every vertex and every edge midpoint of the micro-triangles (section
// comparing matrix-free and sparse storage: vertex and edge DoF counts, the
// 19-entry vertex stencil and the 9-entry edge stencils).  The micro-triangles
// of refinement level l have their vertices and edge midpoints exactly at the
// lattice points of level l+1, so the or_mesh built at level l+1 supplies the
// keys, unique ids and Dirichlet flags of the P2 DoFs.
//
// Element matrix K_ij = integral over T of grad phi_i . grad phi_j, local order
// (v0, v1, v2, m01, m12, m02), with phi = lambda_i (2 lambda_i - 1) at vertex i
// and 4 lambda_a lambda_b at the midpoint of edge ab.  Each integrand is a
// polynomial of degree 2, so the rule with weight |T|/3 at the three edge
// midpoints integrates it exactly.
namespace {
bool p2_element(const double E[3][3], double K[6][6]) {
  const double det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
  if (det == 0.0) return false;
  // grad lambda_1, grad lambda_2 = rows of E^{-1}; grad lambda_0 = -(sum)
  double G[3][2];
  G[1][0] = E[1][1] / det;  G[1][1] = -E[0][1] / det;
  G[2][0] = -E[1][0] / det; G[2][1] = E[0][0] / det;
  G[0][0] = -(G[1][0] + G[2][0]);
  G[0][1] = -(G[1][1] + G[2][1]);
  const double area = std::fabs(det) / 2.0;
  const int ea[3] = {0, 1, 0}, eb[3] = {1, 2, 2};  // edges m01, m12, m02
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) K[i][j] = 0.0;
  for (int q = 0; q < 3; ++q) {
    double lam[3] = {0.0, 0.0, 0.0};  // quadrature point: midpoint of edge q
    lam[ea[q]] = 0.5;
    lam[eb[q]] = 0.5;
    double g[6][2];
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r < 2; ++r) g[i][r] = (4.0 * lam[i] - 1.0) * G[i][r];
    for (int e = 0; e < 3; ++e)
      for (int r = 0; r < 2; ++r) g[3 + e][r] = 4.0 * (lam[eb[e]] * G[ea[e]][r] + lam[ea[e]] * G[eb[e]][r]);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) K[i][j] += (area / 3.0) * (g[i][0] * g[j][0] + g[i][1] * g[j][1]);
  }
  return true;
}
}  // namespace

// P2 stiffness matrix of level m->level - 1 on the DoFs of `m` (built at that
// level + 1), assembled like or_assemble: COO -> CSR with duplicates summed,
// identity rows at Dirichlet DoFs when dirichlet != 0.  Returns nnz, or -1.
int64_t or_assemble_p2(or_mesh* m, int dirichlet) {
  if (m->dim != 2 || m->level < 1) { g_err = "P2 needs a 2D mesh built at level >= 1"; return -1; }
  const int64_t Nc = m->N / 2;  // intervals of the P2 level per macro edge
  std::vector<std::vector<std::pair<int64_t, double>>> rows(m->nu);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    const int64_t* cv = &m->cells[c * 3];
    const int64_t* L = &m->lat[c * m->lat_stride];
    const int64_t lo[3] = {0, 0, 0}, hi[3] = {Nc, Nc, 0};
    for_each_element(2, Nc, lo, hi, [&](int64_t (*v)[3]) {
      // the six P2 points on the level-(l+1) lattice: doubled vertices, then midpoints
      int64_t f[6][3];
      for (int k = 0; k < 3; ++k)
        for (int r = 0; r < 3; ++r) f[k][r] = 2 * v[k][r];
      const int ea[3] = {0, 1, 0}, eb[3] = {1, 2, 2};
      for (int e = 0; e < 3; ++e)
        for (int r = 0; r < 3; ++r) f[3 + e][r] = v[ea[e]][r] + v[eb[e]][r];
      double E[3][3], K[6][6];
      edge_matrix(2, m->coords.data(), cv, m->N, f, E);
      if (!p2_element(E, K)) { bad = true; return; }
      int64_t ids[6];
      for (int k = 0; k < 6; ++k) ids[k] = L[lat_index(2, m->N, f[k])];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) rows[ids[i]].push_back({ids[j], K[i][j]});
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  m->rowptr.assign(m->nu + 1, 0);
  m->cols.clear();
  m->vals.clear();
  for (int64_t u = 0; u < m->nu; ++u) {
    if (dirichlet && m->bnd[u]) {
      m->cols.push_back(u);
      m->vals.push_back(1.0);
    } else {
      auto& row = rows[u];
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) { return a.first < b.first; });
      for (size_t k = 0; k < row.size(); ++k) {
        if (k > 0 && row[k].first == row[k - 1].first) m->vals.back() += row[k].second;
        else { m->cols.push_back(row[k].first); m->vals.push_back(row[k].second); }
      }
    }
    m->rowptr[u + 1] = (int64_t)m->cols.size();
  }
  m->csr_dirichlet = dirichlet ? 3 : 2;
  return (int64_t)m->cols.size();
}

void or_get_csr(const or_mesh* m, int64_t* rowptr, int64_t* cols, double* vals) {
  std::memcpy(rowptr, m->rowptr.data(), sizeof(int64_t) * m->rowptr.size());
  std::memcpy(cols, m->cols.data(), sizeof(int64_t) * m->cols.size());
  std::memcpy(vals, m->vals.data(), sizeof(double) * m->vals.size());
}

// Step 6: y = A x, one row at a time.
void or_spmv(const or_mesh* m, const double* x, double* y) {
  const int64_t* rp = m->rowptr.data();
  const int64_t* ci = m->cols.data();
  const double* va = m->vals.data();
#pragma omp parallel for schedule(static)
  for (int64_t u = 0; u < m->nu; ++u) {
    double s = 0.0;
    for (int64_t k = rp[u]; k < rp[u + 1]; ++k) s += va[k] * x[ci[k]];
    y[u] = s;
  }
}

// y = A x summed element by element, without forming the CSR (same definition,
// used where the CSR would not fit in host memory).
int or_apply_elementwise(const or_mesh* m, int dirichlet, const double* x, double* y) {
  const int d1 = m->dim + 1;
  std::fill(y, y + m->nu, 0.0);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      double E[3][3], K[MAXV][MAXV], vol;
      int64_t ids[MAXV];
      element_data(m, c, v, E, ids);
      if (!element_stiffness(m->dim, E, K, &vol)) { bad = true; return; }
      for (int i = 0; i < d1; ++i) {
        double s = 0.0;
        for (int j = 0; j < d1; ++j) s += K[i][j] * x[ids[j]];
        y[ids[i]] += s;
      }
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  if (dirichlet)
    for (int64_t u = 0; u < m->nu; ++u)
      if (m->bnd[u]) y[u] = x[u];
  return 0;
}

// Lumped mass: m_i = sum over micro-elements T containing i of |T| / (dim+1).
int or_lumped_mass(const or_mesh* m, double* mass) {
  const int d1 = m->dim + 1;
  std::fill(mass, mass + m->nu, 0.0);
  bool bad = false;
  for (int64_t c = 0; c < m->nc; ++c) {
    for_each_cell_element(m, c, [&](int64_t (*v)[3]) {
      double E[3][3], K[MAXV][MAXV], vol;
      int64_t ids[MAXV];
      element_data(m, c, v, E, ids);
      if (!element_stiffness(m->dim, E, K, &vol)) { bad = true; return; }
      for (int i = 0; i < d1; ++i) mass[ids[i]] += vol / d1;
    });
  }
  if (bad) { g_err = "degenerate micro-element"; return -1; }
  return 0;
}

// Rows of A (with identity Dirichlet rows when dirichlet != 0) at sampled
// lattice points, for x given by the keyed SplitMix64 generator with `seed`;
// needs no global build, so it runs at any level.  Sample s is the point
// sample_lat[s*dim ..] of cell sample_cell[s].  Returns 0, or -1 on bad input.
namespace {
// kcoef: evaluate the variable-coefficient operator of or_assemble_varcoef
// with nodal coefficient k = keyed value(kseed) + kshift.
struct KCoef {
  bool on;
  uint64_t seed;
  double shift;
};
int sample_rows_impl(int dim, int64_t nv, const double* coords, int64_t nc, const int64_t* cells, int level,
                     int dirichlet, uint64_t seed, int64_t ns, const int64_t* sample_cell, const int64_t* sample_lat,
                     const double* bubble, KCoef kcoef, double* y, int8_t* is_boundary) {
  if (dim != 2 && dim != 3) { g_err = "dim must be 2 or 3"; return -1; }
  Topology topo = build_topology(dim, nc, cells);
  if (!topo.ok) return -1;
  const int64_t N = int64_t(1) << level;
  const int d1 = dim + 1;
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t c = sample_cell[s];
    if (c < 0 || c >= nc) { g_err = "sample cell out of range"; return -1; }
    const int64_t* cv = cells + c * d1;
    int64_t p[3] = {0, 0, 0}, w[MAXV];
    int64_t sum = 0;
    bool neg = false;
    for (int k = 0; k < dim; ++k) { p[k] = sample_lat[s * dim + k]; sum += p[k]; neg = neg || p[k] < 0; }
    if (neg || sum > N) { g_err = "sample point outside its macro"; return -1; }
    weights_of(dim, N, p, w);
    const Key key = make_key(dim, cv, w);
    std::vector<int64_t> sup = support_of(key);
    const bool bnd = (int)sup.size() <= dim && topo.boundary_subsets.count(sup);
    if (is_boundary) is_boundary[s] = bnd ? 1 : 0;
    if (dirichlet && bnd) { y[s] = keyed_value(seed, key); continue; }
    double acc = 0.0;
    for (int64_t c2 = 0; c2 < nc; ++c2) {
      const int64_t* cv2 = cells + c2 * d1;
      // the point lies in cell c2 iff every vertex of its support is a vertex of c2
      int64_t w2[MAXV] = {0, 0, 0, 0};
      bool contains = true;
      for (int i = 0; i < MAXV && key.v[i] >= 0; ++i) {
        int pos = -1;
        for (int k = 0; k < d1; ++k) if (cv2[k] == key.v[i]) pos = k;
        if (pos < 0) { contains = false; break; }
        w2[pos] = key.w[i];
      }
      if (!contains) continue;
      int64_t p2[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      for (int k = 0; k < dim; ++k) { p2[k] = w2[k + 1]; lo[k] = p2[k] - 1; hi[k] = p2[k]; }
      for_each_element(dim, N, lo, hi, [&](int64_t (*v)[3]) {
        int me = -1;
        for (int i = 0; i < d1; ++i) {
          bool eq = true;
          for (int k = 0; k < dim; ++k) eq = eq && v[i][k] == p2[k];
          if (eq) me = i;
        }
        if (me < 0) return;
        double E[3][3], K[MAXV][MAXV], vol;
        double xv[MAXV];
        double kt = 0.0;
        for (int i = 0; i < d1; ++i) {
          int64_t wi[MAXV];
          weights_of(dim, N, v[i], wi);
          const Key ki = make_key(dim, cv2, wi);
          xv[i] = keyed_value(seed, ki);
          if (kcoef.on) kt += keyed_value(kcoef.seed, ki) + kcoef.shift;
        }
        if (bubble) blended_edge_matrix(coords, cv2, N, &bubble[c2 * 2], v, E);
        else edge_matrix(dim, coords, cv2, N, v, E);
        element_stiffness(dim, E, K, &vol);
        double r = 0.0;
        for (int j = 0; j < d1; ++j) r += K[me][j] * xv[j];
        acc += kcoef.on ? (kt / (double)d1) * r : r;
      });
    }
    y[s] = acc;
  }
  return 0;
}
}  // namespace

int or_sample_rows(int dim, int64_t nv, const double* coords, int64_t nc, const int64_t* cells, int level,
                   int dirichlet, uint64_t seed, int64_t ns, const int64_t* sample_cell,
                   const int64_t* sample_lat, double* y, int8_t* is_boundary) {
  return sample_rows_impl(dim, nv, coords, nc, cells, level, dirichlet, seed, ns, sample_cell, sample_lat, nullptr,
                          KCoef{false, 0, 0.0}, y, is_boundary);
}

// The same rows for the variable-coefficient operator of or_assemble_varcoef
// with k = keyed value(kseed) + kshift at every DoF.
int or_sample_rows_varcoef(int dim, int64_t nv, const double* coords, int64_t nc, const int64_t* cells, int level,
                           int dirichlet, uint64_t seed, uint64_t kseed, double kshift, int64_t ns,
                           const int64_t* sample_cell, const int64_t* sample_lat, double* y, int8_t* is_boundary) {
  return sample_rows_impl(dim, nv, coords, nc, cells, level, dirichlet, seed, ns, sample_cell, sample_lat, nullptr,
                          KCoef{true, kseed, kshift}, y, is_boundary);
}

// The same rows for the blended 2D operator of or_assemble_blended (bubble:
// nc x 2 values, one vector d per macro).
int or_sample_rows_blended(int64_t nv, const double* coords, int64_t nc, const int64_t* cells, int level,
                           int dirichlet, uint64_t seed, const double* bubble, int64_t ns,
                           const int64_t* sample_cell, const int64_t* sample_lat, double* y, int8_t* is_boundary) {
  return sample_rows_impl(2, nv, coords, nc, cells, level, dirichlet, seed, ns, sample_cell, sample_lat, bubble,
                          KCoef{false, 0, 0.0}, y, is_boundary);
}

// Keyed input values x(key) at (cell, lattice point) pairs, without a global build.
int or_keyed_points(int dim, int64_t nc, const int64_t* cells, int level, uint64_t seed, int64_t ns,
                    const int64_t* sample_cell, const int64_t* sample_lat, double* out) {
  const int64_t N = int64_t(1) << level;
  for (int64_t s = 0; s < ns; ++s) {
    const int64_t c = sample_cell[s];
    if (c < 0 || c >= nc) { g_err = "sample cell out of range"; return -1; }
    int64_t p[3] = {0, 0, 0}, w[MAXV];
    for (int k = 0; k < dim; ++k) p[k] = sample_lat[s * dim + k];
    weights_of(dim, N, p, w);
    for (int k = 0; k <= dim; ++k)
      if (w[k] < 0) { g_err = "sample point outside its macro"; return -1; }
    out[s] = keyed_value(seed, make_key(dim, cells + c * (dim + 1), w));
  }
  return 0;
}

// P1 prolongation from `coarse` (level l-1) to `fine` (level l) of the same
// mesh, as CSR (fine rows, coarse columns).  A fine point with all weights
// even is a coarse point; with exactly two odd weights i, j it is the
// midpoint of the coarse points (w +- (e_i - e_j)) / 2; with four odd weights
// (3D macro interior only) it is the midpoint of (w +- (-e0+e1-e2+e3)) / 2 in
// its macro's vertex order, the octahedron diagonal of the refinement.
// Returns nnz, or -1.
int64_t or_prolongation(const or_mesh* fine, const or_mesh* coarse, int64_t* rowptr, int64_t* cols, double* vals) {
  if (fine->dim != coarse->dim || fine->N != 2 * coarse->N || fine->nc != coarse->nc) {
    g_err = "prolongation needs the same mesh at consecutive levels";
    return -1;
  }
  const int dim = fine->dim, d1 = dim + 1;
  std::map<std::vector<int64_t>, int64_t> cell_of;
  for (int64_t c = 0; c < fine->nc; ++c) {
    std::vector<int64_t> s(&fine->cells[c * d1], &fine->cells[c * d1] + d1);
    std::sort(s.begin(), s.end());
    cell_of[s] = c;
  }
  auto find_coarse = [&](const int64_t* vids, const int64_t* w, int n) -> int64_t {
    const Key k = make_key(n - 1, vids, w);
    auto it = std::lower_bound(coarse->keys.begin(), coarse->keys.end(), k, key_less);
    if (it == coarse->keys.end() || !key_eq(*it, k)) return -1;
    return it - coarse->keys.begin();
  };
  int64_t nnz = 0;
  if (rowptr) rowptr[0] = 0;
  for (int64_t u = 0; u < fine->nu; ++u) {
    const Key& k = fine->keys[u];
    int n = 0;
    int64_t vids[MAXV], w[MAXV];
    for (int i = 0; i < MAXV && k.v[i] >= 0; ++i) { vids[i] = k.v[i]; w[i] = k.w[i]; ++n; }
    int odd[MAXV], no = 0;
    for (int i = 0; i < n; ++i) if (w[i] & 1) odd[no++] = i;
    std::vector<std::pair<int64_t, double>> ent;
    if (no == 0) {
      int64_t h[MAXV];
      for (int i = 0; i < n; ++i) h[i] = w[i] / 2;
      ent.push_back({find_coarse(vids, h, n), 1.0});
    } else if (no == 2) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int64_t h[MAXV];
        for (int i = 0; i < n; ++i) h[i] = w[i];
        h[odd[0]] += sgn;
        h[odd[1]] -= sgn;
        for (int i = 0; i < n; ++i) h[i] /= 2;
        ent.push_back({find_coarse(vids, h, n), 0.5});
      }
    } else if (no == 4 && dim == 3) {
      std::vector<int64_t> s(vids, vids + 4);
      const int64_t c = cell_of.at(s);
      const int64_t* cv = &fine->cells[c * d1];
      int64_t wc[MAXV] = {0, 0, 0, 0};
      for (int q = 0; q < 4; ++q)
        for (int i = 0; i < 4; ++i) if (vids[i] == cv[q]) wc[q] = w[i];
      const int64_t dg[4] = {-1, 1, -1, 1};
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int64_t h[MAXV];
        for (int q = 0; q < 4; ++q) h[q] = (wc[q] + sgn * dg[q]) / 2;
        ent.push_back({find_coarse(cv, h, 4), 0.5});
      }
    } else {
      g_err = "unexpected parity pattern";
      return -1;
    }
    for (auto& e : ent) {
      if (e.first < 0) { g_err = "parent not found"; return -1; }
      if (cols) { cols[nnz] = e.first; vals[nnz] = e.second; }
      ++nnz;
    }
    if (rowptr) rowptr[u + 1] = nnz;
  }
  return nnz;
}

// Wall time of `reps` CSR SpMVs with `nthreads` OpenMP threads after `warmup`
// untimed ones; per-rep seconds go to times[].  Returns the thread count used.
int or_time_spmv(const or_mesh* m, int nthreads, int warmup, int reps, double* times) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int used = 1;
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
  std::vector<double> x(m->nu), y(m->nu);
  for (int64_t u = 0; u < m->nu; ++u) x[u] = keyed_value(1, m->keys[u]);
  for (int r = 0; r < warmup; ++r) or_spmv(m, x.data(), y.data());
  for (int r = 0; r < reps; ++r) {
    auto t0 = std::chrono::steady_clock::now();
    or_spmv(m, x.data(), y.data());
    auto t1 = std::chrono::steady_clock::now();
    times[r] = std::chrono::duration<double>(t1 - t0).count();
  }
  return used;
}

}  // extern "C"
