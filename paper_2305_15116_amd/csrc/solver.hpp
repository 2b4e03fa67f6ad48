// Solver workspace layout shared by vcycle_solve and the batched solver.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

#include "mesh.hpp"

namespace mf {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Solver modes 0..5: bit 0 = FP32 V-cycles (else FP64); bit 1 = preconditioned
// conjugate gradients around the V-cycle; bit 2 = preconditioned MINRES
// around it (modes 4, 5); neither = iterative refinement.
constexpr int kNumModes = 6;
inline bool mode_f32(int mode) { return (mode & 1) != 0; }
inline bool mode_pcg(int mode) { return (mode & 2) != 0; }
inline bool mode_minres(int mode) { return (mode & 4) != 0; }
// Krylov modes need a symmetric (pre == post) V-cycle as the preconditioner.
inline bool mode_krylov(int mode) { return mode_pcg(mode) || mode_minres(mode); }

struct Workspace {
  std::vector<void*> b, x, t;  // per level
  double* r64 = nullptr;
  double* e64 = nullptr;
  double* t64 = nullptr;
  double* z64 = nullptr;  // PCG: preconditioned residual (== e64 in FP64 mode; in FP32 mode never
                          // stored: z = res[1] e is formed where it is read)
  double* p64 = nullptr;  // PCG: search direction
  double* q64 = nullptr;  // PCG: A p; MINRES: A z
  // MINRES: r64 and v2 hold the last two Lanczos vectors v, z64 and z2 the
  // preconditioned ones (FP64 z64 == e64), w1 and w2 the last two directions.
  double* v2 = nullptr;
  double* z2 = nullptr;
  double* w1 = nullptr;
  double* w2 = nullptr;
  double* part = nullptr;
  // 16 doubles: [0] r.r, [1] max|r|, [2] r.z, [3] previous r.z, [4] p.Ap,
  // [6..7] a recomputed residual's pair, [8] mixed CG: the scale of the FP32
  // preconditioner input in use (kSlotScale)
  double* result = nullptr;
  int64_t bytes = 0;
};

// Carves the workspace (base may be null to only measure it).  Per level l
// in [lc, level]: right-hand side b[l], iterate x[l] and ping-pong t[l] of the
// V-cycle (FP64 or FP32 by the mode); r64 = outer FP64 residual; the PCG
// vectors; part and result = norm / dot partials and their reductions.
inline Workspace carve(const mf_mesh* m, int level, int mode, int lc, char* base) {
  Workspace w;
  int64_t off = 0;
  auto take = [&](int64_t nbytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off += align_up(nbytes);
    return p;
  };
  const int64_t SL = m->levels[level].storage;
  w.b.assign(level + 1, nullptr);
  w.x.assign(level + 1, nullptr);
  w.t.assign(level + 1, nullptr);
  w.r64 = (double*)take(8 * SL);
  if (!mode_f32(mode)) {
    w.e64 = (double*)take(8 * SL);
    w.t64 = (double*)take(8 * SL);
    w.b[level] = w.r64;
    w.x[level] = w.e64;
    w.t[level] = w.t64;
    for (int l = lc; l < level; ++l) {
      const int64_t S = m->levels[l].storage;
      w.b[l] = take(8 * S);
      w.x[l] = take(8 * S);
      w.t[l] = take(8 * S);
    }
  } else {
    for (int l = lc; l <= level; ++l) {
      const int64_t S = m->levels[l].storage;
      w.b[l] = take(4 * S);
      w.x[l] = take(4 * S);
      w.t[l] = take(4 * S);
    }
  }
  if (mode_pcg(mode)) {
    w.z64 = mode_f32(mode) ? nullptr : w.e64;
    w.p64 = (double*)take(8 * SL);
    w.q64 = (double*)take(8 * SL);
  }
  if (mode_minres(mode)) {
    w.z64 = mode_f32(mode) ? (double*)take(8 * SL) : w.e64;
    w.q64 = (double*)take(8 * SL);
    w.v2 = (double*)take(8 * SL);
    w.z2 = (double*)take(8 * SL);
    w.w1 = (double*)take(8 * SL);
    w.w2 = (double*)take(8 * SL);
  }
  const Level& L = m->levels[level];
  const int64_t np = std::max<int64_t>(L.n_partials(), mode_krylov(mode) ? L.lin_blocks() : 0);
  w.part = (double*)take(8 * 2 * (np + 1));
  w.result = (double*)take(8 * 16);
  w.bytes = off;
  return w;
}

inline int default_coarse(int level) { return std::min(2, level); }

// Mixed CG keeps the scale of its FP32 preconditioner input here: the update
// forms the next input as r / max|r| of the residual before it, so when the
// preconditioner runs, result[1] already holds the next maximum.
constexpr int kSlotScale = 8;

}  // namespace mf
