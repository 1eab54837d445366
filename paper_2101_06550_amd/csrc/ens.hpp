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
  int ndbx, ndby;          // diagnostic-partial blocks (64 x 16 points each)
  long ncolblocks;         // column-pass blocks = ncb * Sc
  // Cahn-Hilliard-Cook forcing (set by ch_ensemble_set_noise): dt amp,
  // 1/dx, 1/dy, generator state mix(seed)
  double nscale, ninv_dx, ninv_dy;
  unsigned long long nseed;
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
                              long diag_stride, size_t lds_bytes, hipStream_t st);
size_t ens_reduced_lds_bytes(int dcount);
hipError_t launch_ens_rows(const EnsRun* runs, const EnsClasses& cls, const int4* items, int nitems,
                           unsigned char* ws, int step, hipStream_t st);
hipError_t launch_ens_finalize(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                               int nitems, unsigned char* ws, int last_step, hipStream_t st);
// Runs small enough for one workgroup's LDS: all nsteps in one launch,
// block b = run small[b]; threads / lds sized for the largest of them.
hipError_t launch_ens_small_steps(const EnsRun* runs, const EnsClasses& cls, const int* small,
                                  int nsmall, int threads, size_t lds, int nsteps,
                                  double* diag_out, long diag_stride,
                                  const unsigned long long* noise_step, hipStream_t st);
// Diagnostics of the final state of the runs big[0..nbig).
hipError_t launch_ens_diag(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                           int nitems, const int* big, int nbig, unsigned char* ws,
                           double* diag_out, long diag_stride, int index, hipStream_t st);

}  // namespace chx
