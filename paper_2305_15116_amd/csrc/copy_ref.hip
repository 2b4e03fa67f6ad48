// device_copy: the measured streaming-copy bandwidth that the stencil
// kernels' rooflines are quoted against, next to the HBM3E peak.  The paper
// likewise measures the machine's load/store bandwidth with a streaming
// benchmark before modelling its kernels (Intro, hardware description).
//
// One 16-byte load and one non-temporal 16-byte store per lane, one block of
// 256 lanes per 4 KiB, no loop: among the shapes measured (loads per lane,
// grid-stride loops, 8- and 16-byte accesses, temporal and non-temporal
// loads and stores) this one moved the most bytes per second on MI355X.

#include <hip/hip_runtime.h>

#include <string>

#include "mesh.hpp"
#include "mf_stencil.h"

using namespace mf;

namespace {

typedef double v2d __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void stream_copy_kernel(const v2d* __restrict__ src, v2d* __restrict__ dst,
                                                          int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

}  // namespace

extern "C" int device_copy(void* dst, const void* src, int64_t n_bytes, void* stream) {
  if (!dst || !src) return set_error(MF_EINVAL, "NULL pointer");
  if (n_bytes < 0 || n_bytes % 16 != 0) return set_error(MF_EINVAL, "n_bytes must be a non-negative multiple of 16");
  if (((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return set_error(MF_EINVAL, "pointers must be 16-byte aligned");
  const int64_t n = n_bytes / 16;
  if (n == 0) return MF_OK;
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0x7fffffff) return set_error(MF_EINVAL, "copy too large for one launch");
  const char* d = (const char*)dst;
  const char* s = (const char*)src;
  if (d < s + n_bytes && s < d + n_bytes) return set_error(MF_EINVAL, "source and destination overlap");
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (const v2d*)src,
                     (v2d*)dst, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  return MF_OK;
}
