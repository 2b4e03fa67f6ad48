// residual_noalloc: the residual with its norm, for callers that cannot
// allocate device memory.
//
// residual() with a norm keeps its per-workgroup partials in buffers the
// mesh allocated at creation and serialises callers on a mutex.  This
// variant keeps them in one file-scope device array instead, so a call
// allocates nothing and takes no lock.  Each device that runs it holds its
// own copy of the array until the process ends; every call on a device
// shares that copy, so calls that overlap on one device race on it.

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "launch.hpp"
#include "mesh.hpp"
#include "mf_stencil.h"

using namespace mf;

namespace {

// 2 MiB: the (sum of squares, max) partial pairs of one residual pass plus
// the reduced pair.  Holds the 2D level-14 triangle and the 6-tet cube up to
// level 9.
constexpr int64_t kScratchDoubles = (2 << 20) / 8;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  The array's name is only a host-side
// stand-in: kernels and copies take this address.
int scratch_for_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(MF_ENOTSUP, "residual_noalloc: device id above 63");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return set_error(MF_EDEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return MF_OK;
}

}  // namespace

extern "C" int residual_noalloc(const mf_mesh* m, int level, int dtype, const void* b, const void* x, void* r,
                                double* norm2, void* stream) {
  if (!m) return set_error(MF_EINVAL, "mesh is NULL");
  if (level < 0 || level > m->max_level) return set_error(MF_EINVAL, "level outside [0, max_level]");
  if (m->host_only) return set_error(MF_ENOTSUP, "mesh was created host-only");
  if (dtype != MF_F64 && dtype != MF_F32) return set_error(MF_EINVAL, "dtype must be MF_F64 or MF_F32");
  if (!b || !x || !r || !norm2) return set_error(MF_EINVAL, "NULL vector or norm2");
  if (r == x || r == b) return set_error(MF_EINVAL, "r must not alias b or x");
  const Level& L = m->levels[level];
  // partials at [0, np) (sums) and [np, 2 np) (maxima), the reduced pair after them
  const int64_t np = stencil_partials(L, dtype);
  if (2 * np + 2 > kScratchDoubles)
    return set_error(MF_ENOMEM, "residual_noalloc: " + std::to_string(np) + " partial pairs need " +
                                    std::to_string((2 * np + 2) * 8) + " bytes of scratch, above its maximum of " +
                                    std::to_string(kScratchDoubles * 8) + " bytes");
  double* part = nullptr;
  int rc = scratch_for_current_device(&part);
  if (rc) return rc;
  double* result = part + 2 * np;
  hipStream_t s = (hipStream_t)stream;
  rc = launch_stencil(m, L, dtype, kResidual, x, r, b, 0.0, part, s);
  if (!rc) rc = launch_reduce(part, np, result, s);
  if (rc) return rc;
  double out[2] = {0.0, 0.0};
  hipError_t e = hipMemcpyAsync(out, result, sizeof(out), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, hipGetErrorString(e));
  *norm2 = std::sqrt(out[0]);
  if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return set_error(MF_ENUMERIC, "residual norm is not finite");
  return MF_OK;
}
