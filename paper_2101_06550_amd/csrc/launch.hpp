// launch.hpp -- device-resident plan views and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace chx {

// Device copy of WholeTables (one-thread-per-system kernels).
struct DevWhole {
  int n = 0, P = 2, periodic = 1;
  double coef[5] = {};
  double minv[4] = {1, 0, 0, 1};
  const double* rec = nullptr;   // device, mi * 8
  const float* rec32 = nullptr;  // device, mi * 8
};

// Device copy of ChunkTables (chunked kernels, chunk length M).
struct DevChunk {
  int n = 0, P = 2, S = 0, dlo = 0, dcount = 0;
  int M = kChunk;                   // chunk length (32, or 16 for the step's small-grid plans)
  double coef[5] = {};
  const double* rec = nullptr;      // device, (M - P) * 8
  const double* blocks = nullptr;   // device, dcount * 4
  const float* rec32 = nullptr;
  const float* blocks32 = nullptr;
  int red_shape = 0;                // separator-kernel tile shape (index into the candidates)
};

// Number of candidate tile shapes of the separator kernel, and the LDS one
// launch of shape `shape` needs (elem = sizeof the sweep type; diag = the
// launch also finishes the diagnostics sum).
constexpr int kNumRedShapes = 15;
// LDS one workgroup may allocate on gfx950 (160 KB per CU)
constexpr size_t kMaxLdsBytes = 160 * 1024;
// (~0 when the shape cannot take S chunks)
size_t reduced_lds_bytes(int shape, int P, size_t elem, int S, int dcount, bool diag);
// Whether a shape is of the whole-column form (every separator part loaded
// once) rather than the windowed one.
bool reduced_shape_whole(int shape);

// Split row pass of the ADI step (penta, FP64, rows of 4096 or 8192 points):
// column separators fused with the interior rows, then the separator rows.
// kNumSplitShapes shapes of the fused kernel's separator part; split_fits
// says whether a shape's window fits the row tile's LDS.
constexpr int kNumSplitShapes = 3;
bool split_fits(const DevChunk& cy, const DevChunk& cx, int shape);
// Separator rows (sep) or interior rows of a step whose column chunks are Mc
// rows long, for a row plan of at most 256 chunks (16- or 32-point).
hipError_t launch_rows_subset(bool sep, double* x, int nx, int ny, int Mc, const DevChunk& cx,
                              hipStream_t st);
hipError_t launch_rows_split_fused(int shape, const DevChunk& cy, const double* rho, double* x,
                                   int nx, int ny, const DevChunk& cx, const double* dpart,
                                   long dnparts, double dscale, double* dout, hipStream_t st);
hipError_t launch_rows_sep(double* x, int nx, int ny, const DevChunk& cx, hipStream_t st);

// nsteps steps of a batched 1D periodic scheme (kind 0 Crank-Nicolson
// hyperdiffusion, 1 Crank-Nicolson diffusion, 2 1D Cahn-Hilliard) on the
// interleaved x (unknown i of system b at i ld + b).  Chunked lengths: the
// right-hand side is fused into the chunk sweep, the steps ping-pong between
// y0 and y1 (pitch batch) with the chunk correction deferred into the next
// sweep, and x is written once at the end; rho holds the separator parts.
// Other lengths: right-hand side into y0, whole sweeps, copy back, per step.
// The scheme's right-hand side alone, y = f(x), one thread per (system, unknown).
hipError_t launch_batch1d_rhs(int kind, const double* x, long ld, double* y, long ldy, int batch,
                              int n, double s, double al, hipStream_t st);
// Batches with one matrix per system (varband.hip): every band array set to a
// constant (nb arrays, entry i of system s at i * ld + s), and the fused
// factor-and-solve of periodic penta / tri systems in place on x (same ld for
// bands and x; ws of the rewrite mode, rows of ldw = batch rounded up to 32).
hipError_t vb_fill_bands(int nb, double* const* bands, const double* values, int n, int batch,
                         long ld, hipStream_t st);
hipError_t vb_penta_rewrite_periodic(int n, int batch, const double* const* bands, long ld,
                                     double* x, double* ws, hipStream_t st);
hipError_t vb_tri_rewrite_periodic(int n, int batch, const double* const* bands, long ld,
                                   double* x, double* ws, hipStream_t st);
size_t vb_rewrite_ws_bytes(int P, int n, int batch);
hipError_t launch_batch1d_steps(int kind, bool chunked, const DevChunk& c, const DevWhole& w,
                                double* x, long ld, int batch, int n, double s, double al,
                                int nsteps, double* y0, double* y1, double* rho,
                                hipStream_t st);

template <int P>
hipError_t launch_whole(const DevWhole& w, double* x, long ss, long es, int batch,
                        hipStream_t st);
// correct = false leaves the chunk interiors uncorrected (separator rows
// final): the caller applies x = y - Zl s_prev - Zr s_own later.
template <int P>
hipError_t launch_chunked_il(const DevChunk& c, double* x, long ld, int batch, double* rho,
                             hipStream_t st, bool correct = true);
template <int P>
hipError_t launch_reduced_il(const DevChunk& c, const double* rho, int batch, double* dst, long ld,
                             int drow_stride, int drow_off, hipStream_t st,
                             const double* dpart = nullptr, long dnparts = 0, double dscale = 0.0,
                             double* dout = nullptr);
template <int P>
// stream_in: the rows are read with non-temporal loads (standalone solves)
hipError_t launch_rows_lds(const DevChunk& c, double* x, long ld, int rows, hipStream_t st,
                           bool stream_in = false);

// FP32 sweeps with FP64 input/output (the refined path): the result is
// written to, or added into (acc), the FP64 output.
template <int P>
hipError_t launch_whole32(const DevWhole& w, double* work, long ss, long es, double* out, long oss,
                          long oes, int batch, bool acc, hipStream_t st);
template <int P>
hipError_t launch_chunked_il32(const DevChunk& c, const double* src, long lds, float* y32,
                               float* rho32, double* out, long ldo, int batch, bool acc,
                               hipStream_t st);
// FP32 rows of n = c.n (dense, ld = n) row-solved in FP32 into dst (FP32).
hipError_t launch_rows_lds_f32(const DevChunk& c, const float* src, float* dst, int rows,
                               hipStream_t st);
// FP32 separators of the chunked interleaved solve (batch systems, ld) from
// the FP32 parts rho into the separator rows of dst; with dout, block (0,0)
// also finishes the fixed-order sum of dnparts (mass, energy) partials.
hipError_t launch_reduced_il32(const DevChunk& c, const float* rho, int batch, float* dst,
                               long ld, hipStream_t st, const double* dpart = nullptr,
                               long dnparts = 0, double dscale = 0.0, double* dout = nullptr);
template <int P>
hipError_t launch_rows_lds32(const DevChunk& c, const double* src, long lds, double* dst, long ldd,
                             int rows, bool acc, hipStream_t st);
// r = f - A x along lines (FP64), strides (system, element) per array.
template <int P>
hipError_t launch_resid_lines(const double* coef, int periodic, int n, const double* f, long fss,
                              long fes, const double* x, long xss, long xes, double* r, long rss,
                              long res, int batch, bool sys_fast, hipStream_t st);

hipError_t launch_stencil2d(const double* in, double* out, int nx, int ny, long ld,
                            const double* w, int left, int right, int top, int bottom,
                            int periodic, int premap, hipStream_t st);
hipError_t launch_stencil2d_f32(const float* in, float* out, int nx, int ny, long ld,
                                const double* w, int left, int right, int top, int bottom,
                                int periodic, int premap, hipStream_t st);

}  // namespace chx
