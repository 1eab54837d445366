// stencil.hip -- cuSten-style 2D xy stencil (thesis Ch.3 "Software API",
// "Software Architecture"): blocks of the field plus their halos are staged in
// LDS, each thread writes its own outputs, input and output are separate
// buffers.  Weights of up to 9 x 9 arrive by value in the kernel arguments;
// premap 1 applies the stencil to v^3 - v (the non-linear Cahn-Hilliard term).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace chx {

constexpr int kMaxExt = 4;
constexpr int kTX = 64, kTY = 16;

struct StencilW {
  double w[(2 * kMaxExt + 1) * (2 * kMaxExt + 1)];
};

__global__ __launch_bounds__(256) void stencil2d_kernel(const double* __restrict__ in,
                                                        double* __restrict__ out, int nx, int ny,
                                                        long ld, StencilW W, int left, int right,
                                                        int top, int bottom, int periodic,
                                                        int premap) {
  __shared__ double tile[(kTY + 2 * kMaxExt) * (kTX + 2 * kMaxExt + 1)];
  const int t = threadIdx.x;
  const int i0 = blockIdx.x * kTX, j0 = blockIdx.y * kTY;
  const int hx = kTX + left + right, hy = kTY + top + bottom;
  const int pitch = kTX + 2 * kMaxExt + 1;
  for (int e = t; e < hx * hy; e += 256) {
    const int ly = e / hx, lx = e - ly * hx;
    int gj = j0 - top + ly, gi = i0 - left + lx;
    double v = 0.0;
    if (periodic) {
      gj = ((gj % ny) + ny) % ny;
      gi = ((gi % nx) + nx) % nx;
      v = in[(long)gj * ld + gi];
    } else if (gj >= 0 && gj < ny && gi >= 0 && gi < nx) {
      v = in[(long)gj * ld + gi];
    }
    if (premap == 1) v = v * v * v - v;
    tile[ly * pitch + lx] = v;
  }
  __syncthreads();
  const int tx = t & 63, ty0 = t >> 6;
  const int wx = left + right + 1;
  const int i = i0 + tx;
  if (i >= nx) return;
  for (int ty = ty0; ty < kTY; ty += 4) {
    const int j = j0 + ty;
    if (j >= ny) break;
    if (!periodic && (i - left < 0 || i + right >= nx || j - top < 0 || j + bottom >= ny))
      continue;
    double acc = 0.0;
    for (int q = 0; q < top + bottom + 1; ++q)
      for (int p = 0; p < wx; ++p) acc = fma(W.w[q * wx + p], tile[(ty + q) * pitch + tx + p], acc);
    out[(long)j * ld + i] = acc;
  }
}

hipError_t launch_stencil2d(const double* in, double* out, int nx, int ny, long ld,
                            const double* w, int left, int right, int top, int bottom,
                            int periodic, int premap, hipStream_t st) {
  StencilW W;
  const int n = (left + right + 1) * (top + bottom + 1);
  for (int k = 0; k < n; ++k) W.w[k] = w[k];
  for (int k = n; k < (2 * kMaxExt + 1) * (2 * kMaxExt + 1); ++k) W.w[k] = 0.0;
  dim3 grid((nx + kTX - 1) / kTX, (ny + kTY - 1) / kTY);
  hipLaunchKernelGGL(stencil2d_kernel, grid, dim3(256), 0, st, in, out, nx, ny, ld, W, left,
                     right, top, bottom, periodic, premap);
  return hipGetLastError();
}

}  // namespace chx
