// Wavefront helpers shared by the stencil walks (device code, gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "mf_internal.hpp"

namespace mf {
namespace wave {

// Cross-lane neighbours through DPP wavefront shifts (a VALU op, no LDS
// traffic): wave_shr:1 gives each lane the value of lane - 1, wave_shl:1 that
// of lane + 1.  Lanes 0 and 63, which have no source, receive 0 (bound_ctrl);
// they are halo lanes whose results are never stored.  Without an `old`
// operand the move needs no register copy of its source.
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long l = __builtin_bit_cast(long long, v);
  const int lo = (int)(l & 0xffffffffLL), hi = (int)(l >> 32);
  const int rlo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  const int rhi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)rhi << 32) | (long long)(unsigned)rlo);
}
template <typename T>
__device__ __forceinline__ T up1(T v) { return dpp_move<kDppWaveShr1>(v); }  // value of lane - 1
template <typename T>
__device__ __forceinline__ T dn1(T v) { return dpp_move<kDppWaveShl1>(v); }  // value of lane + 1

// Maps this block to its natural workgroup index so that each of the 8 XCDs
// (which receive blocks round-robin) works through one contiguous chunk of
// the natural order: neighbouring strips then share that XCD's L2.
__device__ __forceinline__ int xcd_wg(int nwg) {
  const int chunk = (nwg + kXCD - 1) / kXCD;
  const int k = blockIdx.x % kXCD, j = blockIdx.x / kXCD;
  if (j >= chunk) return -1;
  const int n = k * chunk + j;
  return n < nwg ? n : -1;
}

// Grid of an XCD-mapped launch of nwg workgroups.
inline int xcd_grid(int nwg) { return kXCD * ((nwg + kXCD - 1) / kXCD); }

}  // namespace wave
}  // namespace mf
