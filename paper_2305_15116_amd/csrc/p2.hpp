// P2 (quadratic) elements on 2D macro meshes: per-macro constants and tiles.
//
// A P2 field on the mesh refined l times has a DoF at every vertex and every
// edge midpoint of the level-l micro-triangles (the paper's vertex DoFs and
// its three edge orientations, matrix-free vs sparse comparison).  These are
// exactly the lattice points of level l+1, so a P2 vector of level l is laid
// out as the storage vector of level l+1 ("fine lattice", side M = 2^(l+1)):
// in fine coordinates (X, Y) a point is a vertex if X and Y are even, and the
// midpoint of a horizontal (X odd, Y even), vertical (X even, Y odd) or
// diagonal (both odd) micro-edge.  One array, one row walk and one pass cover
// what the paper splits into four kernels over four arrays.
#pragma once

#include <cstdint>

#include "mf_internal.hpp"

namespace mf {

// Interior P2 stencils of one macro in fine-lattice offsets.  The uniform
// refinement is invariant under a point reflection through any DoF, which
// maps every DoF class to itself, so each stencil is centrally symmetric:
// one weight per pair of opposite neighbours (d, -d), listed by d.
//   vertex      [0..9]:   C, (2,0), (0,2), (2,-2), (1,0), (0,1), (1,-1), (1,1), (2,-1), (1,-2)
//   horizontal  [10..14]: C, (1,0), (0,1), (-1,1), (-1,2)
//   vertical    [15..19]: C, (0,1), (2,-1), (1,-1), (1,0)
//   diagonal    [20..24]: C, (1,1), (1,-1), (0,1), (1,0)
// The vertex stencil has the paper's 19 entries (7 vertices, 12 edges) and
// each edge stencil its 9.
constexpr int kP2Weights = 25;

// Element matrix of every micro-triangle of a macro (the "down" triangles
// are point reflections of the "up" ones, which leaves a stiffness matrix
// unchanged), local order v0 v1 v2 m01 m12 m02.  Up triangle with coarse
// anchor (a, b): v0 (2a, 2b), v1 (2a+2, 2b), v2 (2a, 2b+2); down triangle:
// v0 (2a+2, 2b+2), v1 (2a, 2b+2), v2 (2a+2, 2b); m_ij the midpoint of v_i v_j.
struct P2Macro {
  double w[kP2Weights];
  double K[36];
  float wf[kP2Weights];
  float Kf[36];
};

// Wave tiles of the P2 walk: each lane owns two adjacent fine columns
// (an even one and the next), lanes 1..62 produce output, so a tile spans
// 124 fine columns and kP2H fine rows.
#ifndef MF_P2_H
#define MF_P2_H 8
#endif
constexpr int kP2H = MF_P2_H;
constexpr int kP2TileW = 2 * kTileW;
static_assert(kP2H % 2 == 0, "P2 tiles start on even rows");

}  // namespace mf
