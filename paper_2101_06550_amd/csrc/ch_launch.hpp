// ch_launch.hpp -- Cahn-Hilliard kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace chx {

// Scalar coefficients of the explicit right-hand side and the diagnostics.
struct ChCoef {
  double cx, cy;        // D dt / dx^2, D dt / dy^2
  double ccross;        // 2 D gamma dt / (dx^2 dy^2)
  double inv_dx, inv_dy;
  double half_gamma;    // gamma / 2
  double dxdy;          // cell area (mass and energy scale)
};

// Coefficients of the thesis's delta-form scheme (Ch.3 eq. 3:ch_adi).
struct Ch2Coef {
  double a, b;                   // 2/3 D gamma dt, 2/3 D dt
  double inv_dx4, inv_dy4, inv_dx2dy2, inv_dx2, inv_dy2;
};
// Right-hand side r of the delta-form step from (C, Cp) (v == nullptr), or,
// with v, from (C_new, C) where C_new = 2C - Cp + v is also written to cnew
// (which must not alias c, cp, v or r).  recon != nullptr: v still needs the
// column-chunk correction of that plan (applied as v is read).  sweep !=
// nullptr (a chunked column plan, ny a multiple of 32): the kernel also runs
// the column chunk sweep, leaving the chunk interiors y in r and the
// separator parts in rho ([S][4][nx]) for the separator kernel.
hipError_t launch_ch2_rhs(const double* c, long ld, const double* cp, long ldp, const double* v,
                          long ldv, double* cnew, long ldn, double* r, long ldr, int nx, int ny,
                          const Ch2Coef& K, const DevChunk* recon, const DevChunk* sweep,
                          double* rho, hipStream_t st);
// out = 2C - Cp + v, out_prev = C, elementwise (outputs may alias inputs);
// recon as above.
hipError_t launch_ch2_update(const double* c, long ldc, const double* cp, long ldp,
                             const double* v, long ldv, double* out, double* out_prev, long ld,
                             int nx, int ny, const DevChunk* recon, hipStream_t st);

// q != nullptr: the Cahn-Hilliard-Cook increment (pitch nx) is added to the
// right-hand side.
// Cahn-Hilliard-Cook forcing drawn inside a kernel: generator state
// mix(seed), the counter step (of the call's first step for the
// single-workgroup kernel, of the pass otherwise), dt amp, 1/dx, 1/dy.
struct SmallNoise {
  unsigned long long seed_state, step0;
  double scale, inv_dx, inv_dy;
};

hipError_t launch_ch_column_pass(bool recon, bool diag, const double* src, long lds,
                                 double* ybuf, long ldy, int nx, int ny, const DevChunk& cy,
                                 double* rho, const ChCoef& K, double* part, hipStream_t st,
                                 const SmallNoise* nz = nullptr, int order = 0);
// Blocks of one column-pass launch (one (mass, energy) partial each).
long ch_column_pass_blocks(int nx, int Sc);
// After the last step: reconstruct the state into dst and, with diag_out,
// write its (mass, energy) there (partials in part, one per column-pass block).
hipError_t launch_ch_column_final(const double* src, long lds, double* dst, long ldd, int nx,
                                  int ny, const DevChunk& cy, const ChCoef& K, double* part,
                                  double* diag_out, hipStream_t st, int order = 0);
// FP32-refined step (refine.hip): (mass, energy) partial pairs of its column
// kernels; pass 0 (r = RHS(c) written, FP32 column chunk sweep, DIAG when
// part != nullptr); pass nb (residual of x rebuilt from the deferred FP32
// solutions v[0 .. nb-1], FP32 sweep); the state x rebuilt from v[0 .. nb-1]
// into c (and with diag_out its mass and energy there).
int rstep_segments(int nx);  // 64-column wave segments of a row of nx
long rstep_parts(int nx, int ny);
// vprev / nbprev: the previous step's deferred solutions (nbprev = its passes
// + 1), the state rebuilt from them; nbprev = 0 reads c.
hipError_t launch_rstep_first(const double* c, long ld, double* rbuf, float* y32, float* rho,
                              int nx, int ny, const DevChunk& cy, const ChCoef& K, double* part,
                              hipStream_t st, const float* const* vprev = nullptr,
                              int nbprev = 0);
hipError_t launch_rstep_resid(const double* rbuf, const float* const* v, int nb, float* y32,
                              float* rho, int nx, int ny, const DevChunk& cy, const double* cx5,
                              const double* cy5, hipStream_t st);
hipError_t launch_rstep_final(const float* const* v, int nb, double* c, long ld, int nx, int ny,
                              const DevChunk& cy, const ChCoef& K, double* part, double* diag_out,
                              hipStream_t st);
// beta = -(t / F) dF/dt per run and state from a stepping call's diagnostics.
hipError_t launch_ch_decay_rate(const double* diag, int nruns, int nstates, double t0, double dt,
                                double* beta, hipStream_t st);
long ch_diag_partial_blocks(int nx, int ny);
hipError_t launch_ch_diag(const double* c, long ld, int nx, int ny, const ChCoef& K, double* part,
                          double* out, hipStream_t st);
// out[0] = <C>, out[1] = <C^2> by Simpson's rule (part: ch_diag_partial_blocks pairs).
hipError_t launch_ch_simpson(const double* c, long ld, int nx, int ny, double* part, double* out,
                             hipStream_t st);
// out[0] = sum |C^|^2, out[1] = sum |k|^-1 |C^|^2 over the half spectrum of
// a real-to-complex transform (ny x (nx/2 + 1)); part: ch_k1_blocks pairs.
long ch_k1_blocks(int nx, int ny);
hipError_t launch_ch_k1(const double2* spec, int nx, int ny, double lx, double ly, double* part,
                        double* out, hipStream_t st);
hipError_t launch_ch_diag_final(const double* part, long nparts, double scale, double* out,
                                hipStream_t st);
hipError_t launch_ch_residual2d(const double* r, long ldr, const double* c, long ldc, double* R,
                                long ldR, int nx, int ny, const double* cx, const double* cy,
                                hipStream_t st);
// Small grids (one workgroup, field resident in LDS for all nsteps steps):
// at most kSmallMaxThreads tasks (nx ny / 32) and the LDS of ch_small_lds_bytes.
constexpr int kSmallMaxThreads = 512;
size_t ch_small_lds_bytes(int nx, int ny);
bool ch_small_fits(int nx, int ny, size_t max_lds);
hipError_t launch_ch_small_steps(double* c, long ldc, int nx, int ny, int nsteps,
                                 const DevChunk& cy, const DevChunk& cx, const ChCoef& K,
                                 double* diag, const SmallNoise* nz, hipStream_t st);
hipError_t launch_ch_rhs_plain(const double* c, long ld, double* r, long ldr, int nx, int ny,
                               const ChCoef& K, hipStream_t st);

}  // namespace chx
