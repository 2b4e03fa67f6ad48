// Host-side macro mesh and per-level metadata.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "mf_internal.hpp"
#include "mf_stencil.h"
#include "p2.hpp"

namespace mf {

// Device copies of one level's metadata.
struct LevelDev {
  MacroDev* md = nullptr;
  Tile* tiles = nullptr;       // interior wave tiles, padded to a multiple of kWavesPerWG
  Tile* tiles_f32 = nullptr;   // 2D FP32 wave tiles
  Tile* segs = nullptr;        // row segments of 64 points covering every storage point
  Tile* psegs = nullptr;       // slice segments: 64 consecutive storage points of one slice
  int32_t* sbase = nullptr;    // first macro-local index of each slice z = 0 .. N + 1 (3D)
  Tile* pruns = nullptr;       // 3D: runs of up to kTransferRun slice segments (prolongation)
  int32_t* grp_ptr = nullptr;  // ngroups + 1
  Copy* copies = nullptr;
  uint8_t* grp_flag = nullptr;  // bit0: Dirichlet
  int32_t* xgrp_ptr = nullptr;  // exchange groups: shared, non-Dirichlet DoFs
  Copy* xcopies = nullptr;
  int64_t* cpidx = nullptr;   // storage index of every copy (all-groups list)
  int64_t* xcpidx = nullptr;  // storage index of every copy (exchange list)
  double* xgrp_invdiag = nullptr;
  float* xgrp_invdiagf = nullptr;
  double* part = nullptr;       // norm partials: ntiles + iface blocks, then the same again for max
  double* result = nullptr;     // 2 doubles: sum of squares, max |.|
  double* host_result = nullptr;  // pinned host mirror of result
  // coarse direct solve (levels <= 2 only)
  double* cinv = nullptr;
  float* cinvf = nullptr;
  int32_t* cfirst = nullptr;   // storage index of each coarse unknown's first copy
  int32_t* cptr = nullptr;     // copies of each coarse unknown
  int64_t* cidx = nullptr;
  uint32_t* own_bits = nullptr;
  Tile* p2_tiles = nullptr;  // P2 walk tiles over this level's lattice (2D, level >= 1)
};

struct Level {
  int level = 0;
  int N = 0;
  int pen_z = 0;  // 3D tile shape: pencils of kPenZ slices, or runs of slice segments (kPenSeg)
  bool xfused = false;  // the stencil launch finishes shared DoFs (group tiles; slice-run levels): no exchange launch
  int64_t storage = 0, unique = 0;
  std::vector<int64_t> base;    // per macro storage offset
  std::vector<MacroDev> md;
  std::vector<Tile> tiles;      // interior wave tiles (natural order, padded)
  std::vector<Tile> tiles_f32;  // 2D FP32 wave tiles (kTileH2F rows); empty in 3D (same as tiles)
  std::vector<Tile> segs;       // per-point row segments
  // per-point slice segments {macro, first slice-local index, 0, z}: a
  // slice (the whole macro in 2D) is contiguous in storage, so its points
  // are cut into 64-point pieces across row ends (full lanes where rows are short)
  std::vector<Tile> psegs;
  std::vector<int32_t> sbase;  // slice bases, z = 0 .. N + 1 (3D; fits 32 bits up to N = 2048)
  std::vector<Tile> pruns;     // 3D: {macro, first slice-local index, points (<= kTransferRun * 64), z}
  std::vector<int32_t> grp_ptr;
  std::vector<Copy> copies;
  std::vector<uint8_t> grp_flag;
  // exchange groups: DoFs shared by several macros and not Dirichlet
  std::vector<int32_t> xgrp_ptr;
  std::vector<Copy> xcopies;
  std::vector<int64_t> cpidx, xcpidx;  // storage indices of copies / xcopies (kernels skip the macro lookup)
  std::vector<double> xgrp_invdiag;
  int64_t ngroups() const { return (int64_t)grp_ptr.size() - 1; }
  int64_t nxgroups() const { return (int64_t)xgrp_ptr.size() - 1; }
  int64_t iface_blocks() const { return (ngroups() + kIfaceWG - 1) / kIfaceWG; }
  int64_t xgroup_blocks() const { return (nxgroups() + kIfaceWG - 1) / kIfaceWG; }
  const std::vector<Tile>& tiles_for(int dtype) const {
    return dtype == MF_F32 && !tiles_f32.empty() ? tiles_f32 : tiles;
  }
  // norm / dot partials of one stencil pass: one per workgroup of tiles, then one per exchange block
  // (levels whose stencil launch finishes shared DoFs have no exchange partials)
  int64_t n_partials(int dtype) const {
    return (int64_t)tiles_for(dtype).size() / kWavesPerWG + (xfused ? 0 : xgroup_blocks());
  }
  int64_t n_partials() const { return std::max(n_partials(MF_F64), n_partials(MF_F32)); }  // buffer sizes
  // blocks of the linear (grid-stride) vector kernels with partials
  int64_t lin_blocks() const { return std::min<int64_t>(2048, std::max<int64_t>(1, (storage + 1023) / 1024)); }
  std::vector<uint32_t> own_bits;  // bit i: storage DoF i is its unique DoF's owner copy
  std::vector<Tile> p2_tiles;      // P2 of level - 1 on this lattice (2D): wave tiles, natural order, padded
  // coarse direct solve
  int64_t ncoarse = 0;          // unknowns (unique non-Dirichlet DoFs); 0 = not prepared
  std::vector<double> cinv;     // ncoarse^2 inverse of the interior block
  std::vector<int32_t> cfirst, cptr;
  std::vector<int64_t> cidx;
  LevelDev dev;
};

// A vertex, edge or (3D) face of the macro mesh: the support of the
// macro-boundary DoFs whose non-zero barycentric weights sit on exactly these
// vertices.  cells lists every macro containing it, in increasing order, with
// the local index (0..dim) of each of its vertices in that macro.
struct Prim {
  std::vector<int64_t> v;  // sorted global vertex ids
  std::vector<int64_t> cell;
  std::vector<std::array<int8_t, 3>> local;  // local[i][j]: local index of v[j] in cell[i]
  bool dirichlet = false;
};

// Geometry of a 2D macro: its first vertex and the edge vectors to the other two.
struct Geo2 {
  double p0[2];
  double e1[2];
  double e2[2];
};

}  // namespace mf

struct mf_mesh {
  int dim = 0;
  int max_level = 0;
  int flags = 0;
  bool host_only = false;
  int device = 0;
  int64_t nv = 0, nc = 0;
  std::vector<double> coords;
  std::vector<int64_t> cells;
  std::vector<uint16_t> own_mask, dir_mask, shared_mask;  // per macro
  std::vector<mf::Prim> prims;                            // macro-boundary primitives, sorted by vertex ids
  std::vector<mf::Level> levels;
  std::vector<mf::P2Macro> p2;       // 2D: P2 constants per macro (level-independent)
  mf::P2Macro* p2_dev = nullptr;
  std::vector<mf::Geo2> geo2;        // 2D: macro vertex and edge vectors (blended maps)
  mf::Geo2* geo2_dev = nullptr;
  std::mutex norm_mutex;  // serialises residual() calls that return a norm
};

namespace mf {

// Status helpers (thread-local message).
int set_error(int code, const std::string& msg);
const char* last_error();

// Device copy of a host vector (nullptr for an empty one).
template <class T>
int dev_upload(T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return MF_OK;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * src.size());
  if (e != hipSuccess) return set_error(e == hipErrorOutOfMemory ? MF_ENOMEM : MF_EDEVICE, hipGetErrorString(e));
  e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}

// Host set-up (mesh_setup.cpp).
int build_mesh(mf_mesh* m);
int build_coarse_solver(mf_mesh* m, int level);
void free_device(mf_mesh* m);
int upload_level(mf_mesh* m, Level& L);
// 2D tables (p2_setup.cpp): P2 constants and tiles, macro geometry; called by
// build_mesh after the levels.
int build_2d_tables(mf_mesh* m);

// Keys of every storage point of a level, (dim+1) pairs each.
void storage_keys(const mf_mesh* m, int level, int64_t* vids, int32_t* wts);

}  // namespace mf
