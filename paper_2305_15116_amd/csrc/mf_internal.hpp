// Internal types of the matrix-free P1 stencil library, shared by the host
// set-up code and the HIP kernels (never by the oracle).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#define MF_HD __host__ __device__ __forceinline__

namespace mf {

// ---------------------------------------------------------------- tiling
// One wavefront (64 lanes) owns 64 consecutive columns of a macro row and
// produces the 62 inner ones (lanes 0 and 63 are the halo); it walks a strip
// of rows upward, keeping the three rows the 2D stencil reads in registers
// (the layout of the paper's generated kernel: x fastest, rows bottom-up,
// Performance Modeling, experiment description).  Four waves form a workgroup.
constexpr int kWave = 64;
constexpr int kTileW = 62;
// Short strips keep the rows written at any moment within a few MB, so the
// partial cache lines at wave boundaries are completed in L2 before write-back.
#ifndef MF_TILE_H2
#define MF_TILE_H2 8
#endif
constexpr int kTileH2 = MF_TILE_H2;   // rows per 2D wave tile (FP64)
// FP32 rows carry half the bytes: taller tiles with a deeper load ring keep
// as many bytes in flight per wave.
constexpr int kTileH2F = 16;
constexpr int kRingU2F = 8;
// 3D: a wave walks a "pencil" of kPenR rows upward through kPenZ slices,
// keeping the rows of slices z-1, z, z+1 in registers.
#ifndef MF_PEN_R
#define MF_PEN_R 4
#endif
#ifndef MF_PEN_Z
#define MF_PEN_Z 8
#endif
constexpr int kPenR = MF_PEN_R;
constexpr int kPenZ = MF_PEN_Z;
// Small 3D levels: instead of pencils, a wave takes a run of up to kSegRun
// slice segments (64 consecutive storage points of one slice each, across
// row ends), one point per lane, and gathers each point's 15 neighbours.
// A pencil's walk is a chain of dependent slice loads, and with few waves in
// flight that chain sets a small level's kernel time; a run has no chain, so
// a launch costs about one round of loads (measured on the 6-tet cube: 11-14
// us per FP64 apply at N = 16..64 against 18 us with pencils).  From N = 256
// on, the 15 gathered loads per point cost more than the walk (FP64 apply at
// N = 256: 169 us against 96).  kPenSeg marks a level whose tile list holds
// such runs.
constexpr int kPenSeg = 1;
#ifndef MF_SEG3D_UPTO_N
#define MF_SEG3D_UPTO_N 128
#endif
constexpr int kSegUpToN = MF_SEG3D_UPTO_N;  // runs of slice segments when N <= this
constexpr int kSegRun = 4;
// segments per run at side N: fewer on the smallest levels, for more waves
MF_HD constexpr int seg_run(int N) { return N >= 128 ? 4 : (N >= 64 ? 2 : 1); }
// On slice-run levels the stencil launch also finishes the shared DoFs: among
// the runs, the tile list holds group tiles (macro = kGroupTile,
// x0 = first exchange group, y0 = groups, at most 64), whose lanes compute
// each shared DoF's whole row from its copies' partial stencils, so no
// exchange launch follows.
constexpr int kGroupTile = -2;
// 3D prolongations walk runs of up to kTransferRun 64-point slice segments
// (single segments below N = 256).
constexpr int kTransferRun = 4;
#ifndef MF_WAVES_PER_WG
#define MF_WAVES_PER_WG 4
#endif
constexpr int kWavesPerWG = MF_WAVES_PER_WG;
constexpr int kWG = kWave * kWavesPerWG;
constexpr int kIfaceWG = 256;  // groups per interface workgroup
constexpr int kXCD = 8;        // MI355X: 8 accelerator complex dies, workgroups dealt round-robin

// A wave tile: columns [x0, x0+62) of rows [y0, y0+H) of `macro` (2D), or of
// rows [y0, y0+kPenR) in slices [z, z+kPenZ) (3D).  For per-point kernels the same record names a row segment
// of 64 points starting at x0 of row y0 in slice z; in the tile list of a kPenSeg level, y0 points of slice z
// from slice-local index x0 (a run of at most kSegRun segments), then group tiles (kGroupTile).  macro = -1:
// padding.
struct Tile {
  int32_t macro, x0, y0, z;
};

// A copy of a macro-boundary DoF: macro id and its index-space point.
struct Copy {
  int32_t macro, x, y, z;
};

// Per-macro, per-level constants.  wm[s] is the (partial) stencil of a point
// whose non-zero barycentric weights are the local vertices in mask s: the
// sum, over the micro-elements of this macro containing the point, of its
// rows of the element matrices.  s = full (7 in 2D, 15 in 3D) is the
// interior stencil; faces, edges and vertices of the macro get the rows of
// the elements on their side only, which copies of a shared DoF then sum.
// Element matrices K[t] are stored as 4x4 (2D uses the leading 3x3).
struct MacroDev {
  int64_t base;         // storage offset of the macro
  int64_t vid[4];       // global vertex ids in cell order (for keys)
  int32_t N;
  uint16_t own_mask;    // bit s: this macro owns the primitive spanned by local-vertex subset s
  uint16_t dir_mask;    // bit s: that primitive lies on the Dirichlet boundary
  uint16_t shared_mask; // bit s: that primitive belongs to more than one macro
  uint16_t pad0_;
  float inv_diagf;
  double inv_diag;      // 1 / interior centre weight
  double wm[16][16];
  float wmf[16][16];
  double K[6][16];      // element matrix of each micro-element type (row-major 4 x 4)
  float Kf[6][16];      // the same in FP32 (FP32 kernels read it without conversions)
};

// ---------------------------------------------------------------- layout
MF_HD int64_t tet_count(int64_t n) { return n * (n + 1) * (n + 2) / 6; }
MF_HD int64_t tri_count(int64_t n) { return n * (n + 1) / 2; }
// storage points of one macro
MF_HD int64_t macro_points(int dim, int64_t N) { return dim == 2 ? tri_count(N + 1) : tet_count(N + 1); }
// Tet(n) for 0 <= n < 2^16 with 32-bit divisions by constants only (device
// index math runs on the scalar unit, where 64-bit division is a long
// sequence): n(n+1)/2 is an integer, and one of n, n+1, n+2 is a multiple of 3.
MF_HD int64_t tet_count_small(int n) {
  const uint32_t t = (uint32_t)n * (uint32_t)(n + 1) / 2u;
  return (n % 3 == 1) ? (int64_t)t * (int64_t)((n + 2) / 3) : (int64_t)(t / 3u) * (int64_t)(n + 2);
}
// first index of slice z (3D, N <= 2048)
MF_HD int64_t slice_base(int N, int z) { return tet_count_small(N + 1) - tet_count_small(N + 1 - z); }
// start of row y in a triangle of side M (M < 2^15: fits 32 bits)
MF_HD int32_t row_start(int M, int y) { return y * (M + 2) - ((y * (y + 1)) >> 1); }
MF_HD int64_t idx2(int N, int x, int y) { return (int64_t)row_start(N, y) + x; }
MF_HD int64_t idx3(int N, int x, int y, int z) { return slice_base(N, z) + row_start(N - z, y) + x; }

// ---------------------------------------------------------------- micro-elements
// Index-space vertex offsets of the micro-element types (Bey's refinement in
// the lattice; 2D: the up and down triangles).  An element of type t with
// anchor a exists iff a >= 0 componentwise and sum(a) <= N - slack[t].
struct ElemTable {
  int ntypes;
  int nv;
  int8_t off[6][4][3];
  int8_t slack[6];
};

MF_HD constexpr ElemTable elem_table(int dim) {
  if (dim == 2)
    return ElemTable{2, 3,
                     {{{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 0}},
                      {{1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 0}},
                      {}, {}, {}, {}},
                     {1, 2, 0, 0, 0, 0}};
  // 3D: up tet; the octahedron around the (0,1,0)-(1,0,1) diagonal with ring
  // (1,0,0),(1,1,0),(0,1,1),(0,0,1); down tet.
  return ElemTable{6, 4,
                   {{{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
                    {{0, 1, 0}, {1, 0, 1}, {1, 0, 0}, {1, 1, 0}},
                    {{0, 1, 0}, {1, 0, 1}, {1, 1, 0}, {0, 1, 1}},
                    {{0, 1, 0}, {1, 0, 1}, {0, 1, 1}, {0, 0, 1}},
                    {{0, 1, 0}, {1, 0, 1}, {0, 0, 1}, {1, 0, 0}},
                    {{1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}}},
                   {1, 2, 2, 2, 2, 3}};
}

// Stencil offsets in weight order (see mf_stencil.h).
struct StencilTable {
  int n;
  int centre;
  int8_t off[15][3];
};

MF_HD constexpr StencilTable stencil_table(int dim) {
  if (dim == 2)
    return StencilTable{7, 3, {{0, -1, 0}, {1, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {-1, 1, 0}, {0, 1, 0}}};
  return StencilTable{15, 7,
                      {{0, 0, -1}, {1, 0, -1}, {0, 1, -1}, {-1, 1, -1},
                       {0, -1, 0}, {1, -1, 0}, {-1, 0, 0}, {0, 0, 0}, {1, 0, 0}, {-1, 1, 0}, {0, 1, 0},
                       {0, -1, 1}, {1, -1, 1}, {-1, 0, 1}, {0, 0, 1}}};
}

MF_HD constexpr int full_mask(int dim) { return dim == 2 ? 7 : 15; }

// Local-vertex support mask of point p of a macro: bit k set iff barycentric
// weight k is non-zero (weights (N - sum p, p1, .., pd)).
MF_HD int support_mask(int dim, int N, int x, int y, int z) {
  const int w0 = N - x - y - (dim == 3 ? z : 0);
  int m = (w0 != 0 ? 1 : 0) | (x != 0 ? 2 : 0) | (y != 0 ? 4 : 0);
  if (dim == 3) m |= (z != 0 ? 8 : 0);
  return m;
}

// Operation modes of the fused stencil kernels.
enum Mode : int {
  kApply = 0,     // y = A x
  kJacobi = 1,    // y = x + omega D^-1 (b - A x)
  kResidual = 2,  // y = b - A x  (+ sum of squares and max |.| partials)
  kNormB = 3,     // no output; partials of b only (||b|| over unique DoFs)
  kApplyDot = 4,  // y = A x  (+ partials of x . y over unique DoFs)
};

// Modes whose kernels leave (sum, max) partials.
MF_HD constexpr bool has_partials(int mode) { return mode == kResidual || mode == kNormB || mode == kApplyDot; }

// Interface-kernel-only modes.
enum IfaceMode : int {
  kExchangeSum = 10,   // y(all copies) = sum of the copies' values of x; Dirichlet -> 0
  kDirichletSet = 11,  // y = b at Dirichlet DoFs only
};

}  // namespace mf
