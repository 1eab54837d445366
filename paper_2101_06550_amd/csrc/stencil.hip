// stencil.hip -- cuSten-style 2D xy stencil (thesis Ch.3 "Software API",
// "Software Architecture"): blocks of the field plus their halos are staged in
// LDS, each thread writes its own outputs, input and output are separate
// buffers.  Weights of up to 9 x 9 arrive by value in the kernel arguments;
// premap 1 applies the stencil to v^3 - v (the non-linear Cahn-Hilliard term).
// FP64 or FP32 arrays (the arithmetic in the arrays' type).
//
// One workgroup (4 waves) owns a 64-column x 32-row output tile.  The tile and
// its halo are loaded once into LDS (premap applied on the way in); lane l of
// wave w then computes the 8 outputs of column l in rows 8 w .. 8 w + 7,
// walking down the input rows and adding each row's values into all the
// outputs whose stencil that row falls in, so a value is read from LDS once
// per horizontal offset instead of once per weight.
// The extents are rounded up to a class (0, 1, 2 or 4 per direction), the
// weights padded with zeros; each class is its own instantiation with the
// loops fully unrolled.  Tiles are numbered so that the tiles one XCD runs
// (blocks go to the XCDs round robin) form a contiguous band of the field,
// so the halo rows two tiles share meet in one L2 (measured at 8192^2: the
// 5-point stencil 0.223 ms banded, 0.255 ms in plain order); the outputs
// are written with non-temporal stores (plain stores: 0.226 ms).
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "launch.hpp"

namespace chx {

namespace {

constexpr int kMaxExt = 4;
constexpr int kTX = 64;       // tile width (one wave across)
// outputs per thread (down a column): 8 (a 64 x 32 tile, 18 KB of LDS at
// extent 1, 8 workgroups per CU) measured faster than 16 (64 x 64, 35 KB, 4
// per CU) for every stencil of the benchmark, the 5-point one 0.223 against
// 0.238 ms and the 9 x 9 one 0.401 against 0.477 ms at 8192^2
constexpr int kRows = 8;
constexpr int kTY = 4 * kRows;

template <typename T>
struct StencilW {
  T w[(2 * kMaxExt + 1) * (2 * kMaxExt + 1)];
};

// Index of a periodic neighbour.  mode 1: one wrap (the caller guarantees
// n >= the extent), indices past the last one any stencil reads are clamped
// (their values are never used); mode 2: full modulo (tiny fields).
__device__ __forceinline__ int wrap_index(int g, int n, int mode) {
  if (mode == 2) {
    g %= n;
    return g < 0 ? g + n : g;
  }
  g = g < 0 ? g + n : g;
  g = g >= n ? g - n : g;
  return g < n ? g : n - 1;
}

template <int EX, int EY, typename T>
__global__ __launch_bounds__(256) void stencil2d_tiled(const T* __restrict__ in,
                                                       T* __restrict__ out, int nx, int ny,
                                                       long ld, StencilW<T> W, int ntx,
                                                       int per_xcd, int wrap, int premap,
                                                       int left, int right, int top,
                                                       int bottom) {
  constexpr int PX = kTX + 2 * EX, HY = kTY + 2 * EY, WX = 2 * EX + 1;
  __shared__ T tile[HY * PX];
  const int b = blockIdx.x;
  const int t = per_xcd ? (b & 7) * per_xcd + (b >> 3) : b;
  const int by = t / ntx, bx = t - by * ntx;
  const int i0 = bx * kTX, j0 = by * kTY;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // Halo load in three steps so that every load of the thread is in flight
  // at once: indices (wrapped, or clamped and flagged outside the field),
  // then the loads, all from in-bounds addresses, then the LDS writes.
  constexpr int NK = (HY + 3) / 4, NH = (PX + 63) / 64;
  long roff[NK];
  bool rok[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int gj = j0 - EY + wv + 4 * k;
    rok[k] = wrap || (gj >= 0 && gj < ny);
    const int jj = wrap ? wrap_index(gj, ny, wrap) : (gj < 0 ? 0 : (gj < ny ? gj : ny - 1));
    roff[k] = (long)jj * ld;
  }
  int cidx[NH];
  bool cok[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int gi = i0 - EX + lane + 64 * h;
    cok[h] = wrap || (gi >= 0 && gi < nx);
    cidx[h] = wrap ? wrap_index(gi, nx, wrap) : (gi < 0 ? 0 : (gi < nx ? gi : nx - 1));
  }
  T val[NK][NH];
#pragma unroll
  for (int k = 0; k < NK; ++k)
#pragma unroll
    for (int h = 0; h < NH; ++h) val[k][h] = in[roff[k] + cidx[h]];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int ly = wv + 4 * k;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int lx = lane + 64 * h;
      T v = (rok[k] && cok[h]) ? val[k][h] : T(0);
      if (premap) v = v * v * v - v;
      if (ly < HY && lx < PX) tile[ly * PX + lx] = v;
    }
  }
  __syncthreads();
  const int i = i0 + lane;
  if (i >= nx) return;
  if (!wrap && (i - left < 0 || i + right >= nx)) return;

  T acc[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = T(0);
  const T* col = tile + wv * kRows * PX + lane;
#pragma unroll
  for (int k = 0; k < kRows + 2 * EY; ++k) {
    T v[WX];
#pragma unroll
    for (int p = 0; p < WX; ++p) v[p] = col[k * PX + p];
#pragma unroll
    for (int q = 0; q <= 2 * EY; ++q) {
      const int r = k - q;
      if (r < 0 || r >= kRows) continue;
#pragma unroll
      for (int p = 0; p < WX; ++p) acc[r] = fma(W.w[q * WX + p], v[p], acc[r]);
    }
    // one input row at a time: the sums this row fed are complete before the
    // next row's values are read, so only one row's worth of values is live
#pragma unroll
    for (int q = 0; q <= 2 * EY; ++q) {
      const int r = k - q;
      if (r >= 0 && r < kRows) asm volatile("" : "+v"(acc[r])::"memory");
    }
  }

#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int j = j0 + wv * kRows + r;
    if (j >= ny) break;
    if (!wrap && (j - top < 0 || j + bottom >= ny)) continue;
    __builtin_nontemporal_store(acc[r], &out[(long)j * ld + i]);
  }
}

int ext_class(int e) { return e <= 2 ? e : kMaxExt; }

template <int EX, int EY, typename T>
void launch_class(dim3 grid, hipStream_t st, const T* in, T* out, int nx, int ny, long ld,
                  const StencilW<T>& W, int ntx, int per_xcd, int wrap, int premap, int left,
                  int right, int top, int bottom) {
  hipLaunchKernelGGL((stencil2d_tiled<EX, EY, T>), grid, dim3(256), 0, st, in, out, nx, ny, ld,
                     W, ntx, per_xcd, wrap, premap, left, right, top, bottom);
}

template <int EX, typename T>
void launch_ey(int ey, dim3 grid, hipStream_t st, const T* in, T* out, int nx, int ny, long ld,
               const StencilW<T>& W, int ntx, int per_xcd, int wrap, int premap, int left,
               int right, int top, int bottom) {
  switch (ey) {
    case 0: launch_class<EX, 0, T>(grid, st, in, out, nx, ny, ld, W, ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    case 1: launch_class<EX, 1, T>(grid, st, in, out, nx, ny, ld, W, ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    case 2: launch_class<EX, 2, T>(grid, st, in, out, nx, ny, ld, W, ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    default: launch_class<EX, 4, T>(grid, st, in, out, nx, ny, ld, W, ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
  }
}

template <typename T>
hipError_t launch_stencil2d_t(const T* in, T* out, int nx, int ny, long ld, const double* w,
                              int left, int right, int top, int bottom, int periodic, int premap,
                              hipStream_t st) {
  const int ex = ext_class(left > right ? left : right);
  const int ey = ext_class(top > bottom ? top : bottom);
  // the user's (top + bottom + 1) x (left + right + 1) weights placed in the
  // class's (2 ey + 1) x (2 ex + 1) rectangle, centre on centre (rounded to
  // the array type once, here)
  StencilW<T> W;
  for (T& v : W.w) v = T(0);
  const int uw = left + right + 1;
  for (int q = 0; q <= top + bottom; ++q)
    for (int p = 0; p < uw; ++p)
      W.w[(q - top + ey) * (2 * ex + 1) + (p - left + ex)] = (T)w[q * uw + p];
  const int wrap = !periodic ? 0 : (nx >= ex && ny >= ey ? 1 : 2);
  const long ntx = (nx + kTX - 1) / kTX, nty = (ny + kTY - 1) / kTY;
  const long ntiles = ntx * nty;
  if (ntiles > 0x7fffffffL) return hipErrorInvalidValue;
  const int per_xcd = ntiles % 8 == 0 ? (int)(ntiles / 8) : 0;
  const dim3 grid((unsigned)ntiles);
  switch (ex) {
    case 0: launch_ey<0, T>(ey, grid, st, in, out, nx, ny, ld, W, (int)ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    case 1: launch_ey<1, T>(ey, grid, st, in, out, nx, ny, ld, W, (int)ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    case 2: launch_ey<2, T>(ey, grid, st, in, out, nx, ny, ld, W, (int)ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
    default: launch_ey<4, T>(ey, grid, st, in, out, nx, ny, ld, W, (int)ntx, per_xcd, wrap, premap, left, right, top, bottom); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil2d(const double* in, double* out, int nx, int ny, long ld,
                            const double* w, int left, int right, int top, int bottom,
                            int periodic, int premap, hipStream_t st) {
  return launch_stencil2d_t<double>(in, out, nx, ny, ld, w, left, right, top, bottom, periodic,
                                    premap, st);
}

hipError_t launch_stencil2d_f32(const float* in, float* out, int nx, int ny, long ld,
                                const double* w, int left, int right, int top, int bottom,
                                int periodic, int premap, hipStream_t st) {
  return launch_stencil2d_t<float>(in, out, nx, ny, ld, w, left, right, top, bottom, periodic,
                                   premap, st);
}

}  // namespace chx
