// ens.hpp -- device descriptors of an uneven ensemble of Cahn-Hilliard runs.
// One launch per phase advances every run: each block reads a work item
// (run, tile coordinates) and runs the same kernel body as the single-field
// path on that run's buffers and that run's size class's plan tables.
#pragma once

#include <hip/hip_runtime.h>

#include "ch_launch.hpp"
#include "launch.hpp"

namespace chx {

constexpr int kEnsMaxClasses = 8;

struct EnsRun {
  double* c;               // the caller's field of this run (set per call)
  long ldc;                // its leading dimension
  long off_b0, off_b1;     // ping-pong buffers (byte offsets into the workspace)
  long off_rho, off_part;  // separator partials, diagnostic partials
  int nx, ny, cls;         // grid and size class
  int ncb, Sc;             // column-pass blocks per chunk row, column chunks
  long ncolblocks;         // column-pass blocks = ncb * Sc
  // Cahn-Hilliard-Cook forcing (set by ch_ensemble_set_noise): dt amp,
  // 1/dx, 1/dy, generator state mix(seed)
  double nscale, ninv_dx, ninv_dy;
  unsigned long long nseed;
  // FP32-refined runs: r (FP64), the FP32 column buffer and its separator
  // parts, the deferred FP32 solutions V_0 .. V_passes of a step, the refine
  // passes and the 64-column wave segments per row
  long off_r, off_y32, off_rho32, off_v[4];
  int passes, nseg;
};

struct EnsClass {
  DevChunk px, py;  // row (x) and column (y) plans
  ChCoef K;         // right-hand side and diagnostic coefficients
};

// Passed by value: kernel arguments live in the constant segment, so the
// plan-table pointers and the table reads stay scalar (uniform) loads.
struct EnsClasses {
  EnsClass c[kEnsMaxClasses];
};

// Work items are int4 {run, a, b, 0}.
// noise_step: NULL, or the device counter of a forced ensemble (step
// *noise_step + step is drawn inside the pass).
hipError_t launch_ens_column_pass(bool recon, bool diag, const unsigned long long* noise_step,
                                  const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                  int nitems, unsigned char* ws, int step, hipStream_t st);
// The forcing counter's advance by nsteps after a call.
hipError_t launch_ens_noise_advance(unsigned long long* noise_step, int nsteps, hipStream_t st);
hipError_t launch_ens_reduced(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                              int nitems, unsigned char* ws, int step, double* diag_out,
                              long diag_stride, size_t lds_bytes, hipStream_t st,
                              int shape = 0);
size_t ens_reduced_lds_bytes(int dcount, int shape = 0);
// Tile shapes of the FP64 ensemble's separator kernel (shape 0: 8 waves x 4
// chunks) and the chunks one block of a shape covers.
constexpr int kNumEnsRedShapes = 4;
int ens_red_chunks_per_block(int shape);
hipError_t launch_ens_rows(const EnsRun* runs, const EnsClasses& cls, const int4* items, int nitems,
                           unsigned char* ws, int step, hipStream_t st,
                           bool half = false);
// After the last step, over the column-pass items: every multi-kernel run's
// state into its field, and with diag_out its (mass, energy) at `index`.
hipError_t launch_ens_column_final(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                   int nitems, const int* big, int nbig, unsigned char* ws,
                                   int last_step, double* diag_out, long diag_stride, int index,
                                   hipStream_t st);
// Runs small enough for one workgroup's LDS: all nsteps in one launch,
// block b = run small[b]; threads / lds sized for the largest of them.
hipError_t launch_ens_small_steps(const EnsRun* runs, const EnsClasses& cls, const int* small,
                                  int nsmall, int threads, size_t lds, int nsteps,
                                  double* diag_out, long diag_stride,
                                  const unsigned long long* noise_step, hipStream_t st);

// FP32-refined ensembles (every run refined; work items ordered by refine
// passes, most first, so the items of the runs that make pass k are a prefix
// of each list).  Column items {run, segment block of 4 waves, chunk};
// separator items {run, bx, by}; row items {run, row group, 0}.
// pass 0: right-hand side (kept) swept in FP32, with (diag) the partials of
// the state; pass k >= 1: residual swept in FP32; both into the run's FP32
// column buffer and parts.
// from_v (pass 0 of every step after the first of a call): the state is
// rebuilt from the previous step's deferred FP32 solutions instead of read.
hipError_t launch_ens_rstep_column(int pass, bool diag, const EnsRun* runs, const EnsClasses& cls,
                                   const int4* items, int nitems, unsigned char* ws,
                                   hipStream_t st, bool from_v = false);
// FP32 separators into the column buffer; with diag_out, the state's (mass,
// energy) of step `step` (the pass-0 partials).
hipError_t launch_ens_reduced32(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                int nitems, unsigned char* ws, int step, double* diag_out,
                                long diag_stride, size_t lds_bytes, hipStream_t st,
                                int shape = 0);
// FP32 row solves of the column buffer into V_pass.
hipError_t launch_ens_rows32(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                             int nitems, unsigned char* ws, int pass, hipStream_t st);
// The state rebuilt from V_0 .. V_passes into every run's field; with
// diag_out its (mass, energy) at `index` (one block per run of big).
hipError_t launch_ens_rstep_final(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                  int nitems, const int* big, int nbig, unsigned char* ws,
                                  double* diag_out, long diag_stride, int index, hipStream_t st);
// Diagnostics of the final state of the runs big[0..nbig) from their partials
// (R.ncolblocks pairs at R.off_part).
hipError_t launch_ens_diag_final(const EnsRun* runs, const EnsClasses& cls, const int* big,
                                 int nbig, unsigned char* ws, double* diag_out, long diag_stride,
                                 int index, hipStream_t st);

}  // namespace chx
