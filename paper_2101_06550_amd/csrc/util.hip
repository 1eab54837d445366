// util.hip -- a plain streaming copy, the reference for HBM measurements.
//
// Not part of the method: the benchmark times it to state the bandwidth a
// simple streaming kernel reaches on the device (next to the published
// peak), and the hardware byte counters of the benchmark are scaled by what
// they read for it.  One 16-byte non-temporal load and store per thread, the
// fastest of the copy shapes measured on gfx950 (6.5 TB/s).
#include <hip/hip_runtime.h>

#include "chx.h"
#include "common.hpp"

namespace chx {
namespace {

__global__ __launch_bounds__(256) void stream_copy_kernel(const double* __restrict__ src,
                                                          double* __restrict__ dst, size_t n) {
  const size_t base = (size_t)blockIdx.x * 512;
  const int t = threadIdx.x;
  if (base + 512 <= n) {
    const double2* s2 = reinterpret_cast<const double2*>(src + base);
    double2* d2 = reinterpret_cast<double2*>(dst + base);
    store_stream(d2 + t, load_stream(s2 + t));
  } else {
    for (size_t i = base + t; i < n; i += 256) dst[i] = src[i];
  }
}

}  // namespace
}  // namespace chx

extern "C" int chx_stream_copy(const double* src, double* dst, size_t n, chx_stream s) {
  if (n == 0) return CHX_OK;
  if (!src || !dst) return CHX_EINVAL;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) return CHX_EINVAL;
  const char* a = reinterpret_cast<const char*>(src);
  const char* b = reinterpret_cast<const char*>(dst);
  if (a < b + n * sizeof(double) && b < a + n * sizeof(double)) return CHX_EINVAL;
  const size_t blocks = (n + 511) / 512;
  if (blocks > 0x7fffffffu) return CHX_EINVAL;
  hipLaunchKernelGGL(chx::stream_copy_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(s), src, dst, n);
  return hipGetLastError() == hipSuccess ? CHX_OK : CHX_EHIP;
}
