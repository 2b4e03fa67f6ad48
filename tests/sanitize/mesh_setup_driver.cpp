// Host code of the library under a sanitizer (AddressSanitizer with leak
// detection, or ThreadSanitizer; build.sh): builds host-only meshes
// (MF_FLAG_HOST_ONLY: no device memory) of several 2D and 3D shapes and
// levels, queries their keys, lattice indices and stencils, and sets up
// three meshes concurrently from three threads, as the serving preparers
// do.  BIG=1 adds the 6-tet cube at level 8 (the multi-threaded set-up
// paths).
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <vector>
#include <random>
#include <algorithm>
#include <thread>
#include "mf_stencil.h"
static void ck(int rc, const char* what) { if (rc) { printf("FAIL %s: %d %s\n", what, rc, mf_last_error()); exit(1); } }
static void exercise(int dim, const std::vector<double>& co, const std::vector<int64_t>& ce, int maxl) {
  mf_mesh* m = nullptr;
  const int64_t nv = co.size() / dim, nc = ce.size() / (dim + 1);
  ck(create_macro_mesh(dim, nv, co.data(), nc, ce.data(), maxl, MF_FLAG_DIRICHLET | MF_FLAG_HOST_ONLY, &m), "create");
  for (int L = 0; L <= maxl; ++L) {
    int64_t s = 0, u = 0;
    ck(mesh_num_dofs(m, L, &s, &u), "num");
    std::vector<int64_t> vids(s * (dim + 1));
    std::vector<int32_t> w(s * (dim + 1));
    ck(mesh_dof_keys(m, L, vids.data(), w.data()), "keys");
    const int64_t n = 64;
    std::vector<int64_t> ml(n * (dim + 1)), idx(n);
    std::mt19937_64 g(L);
    const int64_t N = 1 << L;
    for (int64_t i = 0; i < n; ++i) {
      ml[i * (dim + 1)] = g() % nc;
      int64_t rem = N;
      for (int k = 0; k < dim; ++k) { int64_t c = rem ? g() % (rem + 1) : 0; ml[i * (dim + 1) + 1 + k] = c; rem -= c; }
    }
    ck(mesh_dof_index(m, L, n, ml.data(), idx.data()), "index");
    std::vector<double> st(dim == 2 ? 7 : 15);
    for (int64_t c = 0; c < nc; ++c) ck(mesh_stencil(m, L, c, st.data()), "stencil");
  }
  ck(destroy_macro_mesh(m), "destroy");
}
int main() {
  // unit triangle, two-triangle square, strip of triangles
  exercise(2, {0, 0, 1, 0, 0, 1}, {0, 1, 2}, 10);
  exercise(2, {0, 0, 1, 0, 1, 1, 0, 1}, {0, 1, 2, 0, 2, 3}, 9);
  {
    std::vector<double> co; std::vector<int64_t> ce; const int k = 8;
    for (int i = 0; i <= k; ++i) { co.push_back(i); co.push_back(0); co.push_back(i); co.push_back(1); }
    for (int i = 0; i < k; ++i) { ce.insert(ce.end(), {2 * i, 2 * i + 2, 2 * i + 1}); ce.insert(ce.end(), {2 * i + 1, 2 * i + 2, 2 * i + 3}); }
    exercise(2, co, ce, 7);
  }
  // Kuhn cube (6 tets), canonical and shuffled vertex orders
  std::vector<double> co;
  for (int v = 0; v < 8; ++v) { co.push_back(v & 1); co.push_back((v >> 1) & 1); co.push_back((v >> 2) & 1); }
  std::vector<int64_t> ce;
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (auto& p : perms) {
    int v = 0; ce.push_back(v);
    for (int k = 0; k < 3; ++k) { v |= 1 << p[k]; ce.push_back(v); }
  }
  exercise(3, co, ce, getenv("BIG") ? 8 : 6);
  std::mt19937 g(3);
  for (size_t c = 0; c < 6; ++c) std::shuffle(ce.begin() + 4 * c, ce.begin() + 4 * c + 4, g);
  exercise(3, co, ce, 6);
  // concurrent set-up from three threads (as the serving preparers do)
  {
    std::vector<std::thread> th;
    for (int t = 0; t < 3; ++t)
      th.emplace_back([&, t] {
        if (t == 0) exercise(3, co, ce, 6);
        else if (t == 1) exercise(2, {0, 0, 1, 0, 0, 1}, {0, 1, 2}, 9);
        else exercise(2, {0, 0, 1, 0, 1, 1, 0, 1}, {0, 1, 2, 0, 2, 3}, 8);
      });
    for (auto& x : th) x.join();
  }
  printf("sanitizer driver OK\n");
  return 0;
}
