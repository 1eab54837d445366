/*
 * chx.h -- C-ABI of the MI355X (gfx950) Cahn-Hilliard ADI library.
 *
 * The library implements the hot path of A. Gloster's thesis (arXiv
 * 2101.06550): batched constant-coefficient cyclic pentadiagonal and
 * tridiagonal solves (Ch.4 "cuPentBatch", Ch.5 single-LHS batched solvers),
 * cuSten-style 2D stencils (Ch.3 "Software API") and one semi-implicit ADI
 * time step of the periodic 2D Cahn-Hilliard equation (Ch.2 eq. 2:ch,
 * Ch.3 eq. 3:ch_adi), all on HIP kernels written for gfx950.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: CHX_OK (0) or a negative CHX_E*
 *    code.  No C++ exception crosses this boundary.
 *  - Pointers named "device" are HIP device pointers (for instance
 *    torch.Tensor.data_ptr() of a CUDA/HIP tensor); pointers named "host" are
 *    ordinary host memory.  The caller owns every field, right-hand side,
 *    workspace and output buffer.  The library owns only the opaque plan and
 *    handle objects and the small device tables inside them; *_destroy frees
 *    them.
 *  - Device work is enqueued asynchronously on the caller's stream
 *    (chx_stream = hipStream_t; 0 = the null stream).  Argument checks are
 *    synchronous and happen before anything is enqueued.  A failed kernel
 *    launch returns CHX_EHIP.
 *  - Plans and handles are immutable after creation, so one plan may be used
 *    from several streams and host threads at once; calls that share a
 *    workspace or an output buffer must not overlap.
 *  - Arrays are FP64 unless said otherwise.  2D fields are row-major with x
 *    (index i) fastest: element (i, j) at j*ld + i, ld >= nx.
 *  - There is no CPU fallback: without a usable gfx950 device the calls that
 *    launch work return CHX_EHIP.
 */
#ifndef CHX_H
#define CHX_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CHX_OK = 0,
  CHX_EINVAL = -1,          /* bad argument (null pointer, ld too small, ...)  */
  CHX_EUNSUPPORTED_N = -2,  /* system size below the minimum (5 penta, 3 tri)  */
  CHX_EPIVOT = -3,          /* zero, negative or non-finite pivot in a factor  */
  CHX_EHIP = -4,            /* a HIP runtime call or kernel launch failed      */
  CHX_ENONFINITE = -5,      /* a diagnostic sum is NaN or infinite             */
  CHX_ENOMEM = -6,          /* workspace too small / allocation failed         */
  CHX_EREFINE = -7,         /* iterative refinement did not reduce the error   */
  CHX_ESCRATCH = -8         /* needs more than the static scratch (see below)  */
};

enum chx_dtype {
  CHX_F64 = 0,              /* FP64 sweeps and storage                          */
  CHX_F32_REFINED = 1,      /* FP32 sweeps + FP64 residual refinement (FP64 I/O) */
  CHX_F32 = 2               /* FP32 arrays and arithmetic (stencil2d_apply)       */
};

enum chx_layout {
  CHX_INTERLEAVED = 0,      /* element i of system s at i*ld + s, ld >= batch    */
  CHX_CONTIGUOUS = 1        /* element i of system s at s*ld + i, ld >= n        */
};

typedef struct chx_penta_plan_s* chx_penta_plan;
typedef struct chx_tri_plan_s* chx_tri_plan;
typedef struct chx_ch_s* chx_ch;
typedef void* chx_stream;

/* Library version, e.g. 100 for 0.1.0. */
int chx_version(void);

/* chx_stream_copy: dst[i] = src[i], i < n (device FP64 arrays, 16-byte
 *   aligned, not overlapping), one streaming kernel, asynchronous on stream s.
 *   A measurement helper, not part of the method: its rate is the HBM
 *   bandwidth a plain streaming kernel reaches (the practical ceiling next to
 *   the published peak), and hardware byte counters are calibrated on it.
 *   CHX_EINVAL for NULL, misaligned or overlapping arrays. */
int chx_stream_copy(const double* src, double* dst, size_t n, chx_stream s);
/* Human-readable text for a status code (static storage). */
const char* chx_status_string(int status);

/* ------------------------------------------------------------------------
 * Pentadiagonal systems (Ch.4 "The pentadiagonal matrix system",
 * "Solution of the pentadiagonal system"; Ch.5 "Pentadiagonal Systems").
 * Row i of the n x n matrix is a x[i-2] + b x[i-1] + c x[i] + d x[i+1] +
 * e x[i+2]; periodic != 0 wraps the indices mod n (the corners of the
 * cyclic matrix, removed by Navon's bordering of the last two unknowns),
 * periodic == 0 drops the entries that fall outside the matrix.
 *
 * penta_factor: factor once (host, FP64 accumulated in extended precision)
 *   and upload the plan's tables -- the LR factors of the bordered block,
 *   the bordering (Schur-complement) vectors and their FP32 copies -- so that
 *   every later solve only sweeps.  n >= 5, else CHX_EUNSUPPORTED_N.  The
 *   factorisation does not pivot (as in the thesis): a pivot alpha_i <= 0 or
 *   not finite gives CHX_EPIVOT; the matrix should be symmetric positive
 *   definite or diagonally dominant.  The device that is current when this is
 *   called holds the tables; solves must run on that device.
 * penta_plan_destroy: frees the plan (NULL is accepted).
 */
int penta_factor(int n, double a, double b, double c, double d, double e,
                 int periodic, chx_penta_plan* out);
int penta_plan_destroy(chx_penta_plan p);

/* Bytes of device workspace that penta_solve_batch needs for (batch, layout,
 * dtype, refine_passes); 0 means no workspace is used (ws may be NULL). */
size_t penta_solve_ws_bytes(chx_penta_plan p, int batch, int layout, int dtype,
                            int refine_passes);

/* penta_solve_batch: solve A x_s = f_s for batch systems sharing the plan's
 *   single LHS (Ch.5 "single LHS, interleaved RHS").  x_inout (device) holds
 *   the right-hand sides on entry and the solutions on return, FP64, in the
 *   given layout with leading dimension ld (ld >= batch interleaved, ld >= n
 *   contiguous).  dtype CHX_F64 sweeps in FP64; CHX_F32_REFINED sweeps in FP32
 *   and applies refine_passes (1..3) FP64-residual refinement passes.  ws
 *   (device) must hold penta_solve_ws_bytes(...) bytes, aligned to 256 B.
 *   Returns CHX_EINVAL for bad arguments, CHX_ENOMEM if ws_bytes is short,
 *   and for CHX_F32_REFINED CHX_EREFINE (before anything is enqueued) when
 *   the matrix is too ill-conditioned for FP32 sweeps to reduce the error:
 *   4 kappa 2^-24 >= 1, kappa = the plan's 2-norm condition number (exact
 *   for periodic plans, whose matrix is circulant: max / min |eigenvalue|;
 *   the symbol's range for non-periodic ones).  Each refinement pass shrinks
 *   the error by about kappa 2^-24. */
int penta_solve_batch(chx_penta_plan p, int batch, void* x_inout, long ld,
                      int layout, int dtype, int refine_passes, void* ws,
                      size_t ws_bytes, chx_stream s);

/* Size of the library's static device scratch (per GPU): 32 MiB. */
#define CHX_NOALLOC_SCRATCH_BYTES (32u << 20)

/* penta_solve_batch_noalloc: penta_solve_batch for callers that cannot
 *   allocate device memory (code under HIP graph capture, tight serving
 *   loops, harnesses that forbid hipMalloc).  Same arguments and results as
 *   penta_solve_batch without ws / ws_bytes: the workspace is a static device
 *   array of CHX_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held
 *   until the process ends (its address is looked up once per device, on the
 *   first call with that device current).  The call itself allocates nothing
 *   (no hipMalloc, hipFree or allocating library routine).  Returns
 *   CHX_ESCRATCH, before anything is enqueued, when
 *   penta_solve_ws_bytes(p, batch, layout, dtype, refine_passes) exceeds
 *   CHX_NOALLOC_SCRATCH_BYTES (for n = 1024: up to 32768 interleaved systems
 *   in FP64, about 1600 FP32-refined; contiguous FP64 needs no scratch).
 *   Every call on one GPU shares that GPU's scratch, so calls that overlap on
 *   one GPU (other streams, other host threads) race and must be serialised
 *   by the caller; the scratch keeps whatever the last call left (every
 *   kernel writes what it later reads, nothing needs to start at zero). */
int penta_solve_batch_noalloc(chx_penta_plan p, int batch, void* x_inout,
                              long ld, int layout, int dtype,
                              int refine_passes, chx_stream s);

/* ------------------------------------------------------------------------
 * Tridiagonal systems (Ch.5 "Tridiagonal Inversion Algorithm",
 * "Periodic Tridiagonal Matrix").  Row i is a x[i-1] + b x[i] + c x[i+1];
 * periodic wraps (top-right corner a, bottom-left corner c).  n >= 3.  The
 * other conventions are those of the pentadiagonal calls.
 */
int tri_factor(int n, double a, double b, double c, int periodic,
               chx_tri_plan* out);
int tri_plan_destroy(chx_tri_plan p);
size_t tri_solve_ws_bytes(chx_tri_plan p, int batch, int layout, int dtype,
                          int refine_passes);
int tri_solve_batch(chx_tri_plan p, int batch, void* x_inout, long ld,
                    int layout, int dtype, int refine_passes, void* ws,
                    size_t ws_bytes, chx_stream s);

/* ------------------------------------------------------------------------
 * Batches with one matrix per system (Ch.4 "Implementation on GPU", the
 * cuPentBatch design: every system its own diagonals, one thread per system
 * on interleaved data, factorisation split from the solve; Ch.5 for the
 * tridiagonal case).  Every array -- the diagonals and x -- is interleaved
 * with one leading dimension: entry i of system s at i*ld + s, ld >= batch,
 * device FP64.
 *   Penta row i: a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} +
 *   e_i x_{i+2} = f_i; tri row i: a_i x_{i-1} + b_i x_i + c_i x_{i+1} = f_i.
 *   periodic = 0: entries that fall outside the matrix are ignored (a_0, a_1,
 *   b_0, d_{n-1}, e_{n-2}, e_{n-1}; tri a_0, c_{n-1}); n >= 3 (tri n >= 2).
 *   periodic = 1: indices wrap mod n (Ch.4 bordering of the last two
 *   unknowns; Ch.5 Sherman-Morrison with A' built from each system's rows,
 *   which needs b_0 != 0); n >= 5 (tri n >= 3).
 * No pivoting, as in the thesis: the LR (Thomas) factorisation must exist,
 * e.g. diagonally dominant or symmetric positive definite matrices.  A zero
 * pivot is not detected on the device: that system's solution is non-finite
 * and the other systems are unaffected.
 *
 * penta_batch_factor / tri_batch_factor: factor every system once, IN PLACE
 *   (the thesis overwrites the matrix with its factors): b <- beta,
 *   c <- 1/alpha, d <- gamma, e <- delta (a kept); tri b <- 1/den, c <- chat.
 *   Periodic systems also fill ws with their correction vectors; their rows
 *   n-2 and n-1 are left as given.
 * penta_batch_solve / tri_batch_solve: solve with those factors (and that ws)
 *   for the right-hand sides in x, solution returned in x; repeatable.
 * penta_batch_rewrite / tri_batch_rewrite: the thesis's "Rewrite" mode for
 *   matrices that change every step: factor and solve in one pass, the
 *   diagonals left untouched, the back sweep's coefficients kept in ws.
 * *_batch_ws_bytes(n, batch, periodic, mode): device workspace (256-byte
 *   aligned) for mode CHX_BATCH_FACTOR (the factor/solve pair, which must
 *   share one ws; 0 when not periodic, ws may then be NULL) or
 *   CHX_BATCH_REWRITE; 0 also for invalid arguments.
 * Errors: CHX_EINVAL (NULL array, ld < batch, periodic not 0/1, ws NULL or
 *   misaligned when needed), CHX_EUNSUPPORTED_N, CHX_ENOMEM (ws_bytes short),
 *   CHX_EHIP (launch failed).  batch = 0 does nothing.  Asynchronous on s.
 */
#define CHX_BATCH_FACTOR 0
#define CHX_BATCH_REWRITE 1
size_t penta_batch_ws_bytes(int n, int batch, int periodic, int mode);
int penta_batch_factor(int n, int batch, int periodic, double* a, double* b,
                       double* c, double* d, double* e, long ld, void* ws,
                       size_t ws_bytes, chx_stream s);
int penta_batch_solve(int n, int batch, int periodic, const double* a,
                      const double* b, const double* c, const double* d,
                      const double* e, long ld, const void* ws,
                      size_t ws_bytes, double* x, chx_stream s);
int penta_batch_rewrite(int n, int batch, int periodic, const double* a,
                        const double* b, const double* c, const double* d,
                        const double* e, long ld, double* x, void* ws,
                        size_t ws_bytes, chx_stream s);
size_t tri_batch_ws_bytes(int n, int batch, int periodic, int mode);
int tri_batch_factor(int n, int batch, int periodic, double* a, double* b,
                     double* c, long ld, void* ws, size_t ws_bytes,
                     chx_stream s);
int tri_batch_solve(int n, int batch, int periodic, const double* a,
                    const double* b, const double* c, long ld, const void* ws,
                    size_t ws_bytes, double* x, chx_stream s);
int tri_batch_rewrite(int n, int batch, int periodic, const double* a,
                      const double* b, const double* c, long ld, double* x,
                      void* ws, size_t ws_bytes, chx_stream s);

/* ------------------------------------------------------------------------
 * stencil2d_apply: cuSten-style 2D stencil in the xy direction (Ch.3
 *   "Software API").  out[j][i] = sum_{q=-top..bottom} sum_{p=-left..right}
 *   w[(q+top)*(left+right+1) + (p+left)] * pre(in[j+q][i+p]),
 *   pre(v) = v (premap 0) or v^3 - v (premap 1, the non-linear Cahn-Hilliard
 *   term that the thesis applies through a function-pointer stencil).
 *   Weights (host, FP64) are listed from the top-left of the stencil, left to
 *   right, row by row; "top" is the smaller j.  Extents are 0..4 each.
 *   periodic != 0 wraps indices; periodic == 0 writes only the points whose
 *   whole stencil lies inside the array and leaves the boundary cells of out
 *   untouched.  in and out (device, nx x ny, leading dimension ld >= nx) must
 *   not overlap (the thesis's separate input and output buffers).  dtype
 *   CHX_F64: FP64 arrays and arithmetic; CHX_F32: FP32 arrays, the weights
 *   rounded to FP32 once and the sums formed in FP32 (half the bytes per
 *   point, the thesis names single precision as future work); any other
 *   dtype is CHX_EINVAL.
 */
int stencil2d_apply(const void* in, void* out, int nx, int ny, long ld, int dtype,
                    const double* weights, int left, int right, int top,
                    int bottom, int periodic, int premap, chx_stream s);

/* ------------------------------------------------------------------------
 * Batched 1D periodic time stepping: many independent systems of n unknowns
 * on (0, L), dx = L / n, interleaved (unknown i of system b at i*ld + b,
 * ld >= batch), one constant cyclic matrix factored once (batch1d_create).
 * Each step forms the scheme's right-hand side from the state and solves:
 *   CHX_1D_HYPERDIFFUSION_CN (Ch.4 eq. disc): C_t = -a C_xxxx, Crank-Nicolson,
 *     s = a dt / (2 dx^4): (s,-4s,1+6s,-4s,s) C+ = (-s,4s,1-6s,4s,-s) C;
 *   CHX_1D_DIFFUSION_CN (Ch.5 eq. 5:1ddiffscheme): C_t = a C_xx,
 *     s = a dt / (2 dx^2): (-s,1+2s,-s) C+ = (s,1-2s,s) C;
 *   CHX_1D_CAHN_HILLIARD (Ch.6 eq. 6:1Dnumerical), gamma = a, mobility D:
 *     s = a D dt / dx^4, al = D dt / dx^2, N = C^3 - C:
 *     (s,-4s,1+6s,-4s,s) C+ = C + al (N[i-1] - 2 N[i] + N[i+1]).
 * batch1d_create: kind, n (>= 5, >= 3 for diffusion: else
 *   CHX_EUNSUPPORTED_N), L, dt > 0, a, D >= 0 (D used by Cahn-Hilliard).
 * batch1d_ws_bytes: device workspace (256-byte aligned) for batch systems.
 * batch1d_step: advance x_inout (device) by nsteps >= 1 steps in place,
 *   asynchronous on stream s; calls sharing ws must not overlap. */
#define CHX_1D_HYPERDIFFUSION_CN 0
#define CHX_1D_DIFFUSION_CN 1
#define CHX_1D_CAHN_HILLIARD 2
typedef struct chx_batch1d_s* chx_batch1d;
int batch1d_create(int kind, int n, double L, double dt, double a, double D,
                   chx_batch1d* out);
int batch1d_destroy(chx_batch1d b);
size_t batch1d_ws_bytes(chx_batch1d b, int batch);
int batch1d_step(chx_batch1d b, int batch, double* x_inout, long ld, int nsteps,
                 void* ws, size_t ws_bytes, chx_stream s);
/* batch1d_step_rewrite: the same nsteps steps in the thesis's "Rewrite" mode
 *   (Ch.4 "Performance Analysis", cuPentBatchRewrite): every step forms the
 *   right-hand side, writes every system's diagonals afresh (as for a matrix
 *   that changes from step to step) and factors and solves each system in
 *   one pass (penta_batch_rewrite / tri_batch_rewrite, periodic), one thread
 *   per system.  Any n the kind allows.  batch1d_rewrite_ws_bytes: its device
 *   workspace (256-byte aligned): two fields, the bands and the solver's
 *   workspace.  Same results as batch1d_step up to rounding; much more
 *   memory traffic (kept for the comparison the thesis makes). */
size_t batch1d_rewrite_ws_bytes(chx_batch1d b, int batch);
int batch1d_step_rewrite(chx_batch1d b, int batch, double* x, long ld,
                         int nsteps, void* ws, size_t ws_bytes, chx_stream s);

/* ------------------------------------------------------------------------
 * Cahn-Hilliard ADI stepping (Ch.2 eq. 2:ch, Ch.3 eq. 3:ch_adi).
 * One step on the periodic box [0,lx) x [0,ly), nx x ny points, dx = lx/nx:
 *   r = c + D dt Lap5(c^3 - c) - 2 D gamma dt (d2x d2y) c
 *   (I + sx P_x)(I + sy P_y) c_new = r,   P = circ(1,-4,6,-4,1),
 *   s = D gamma dt / h^4,
 * i.e. the explicit right-hand side by stencils, then batched cyclic
 * pentadiagonal solves along every row and every column.
 */
typedef struct {
  int nx, ny;            /* grid points (>= 5 each)                        */
  double lx, ly;         /* box lengths (the thesis uses 2 pi)            */
  double D, gamma, dt;   /* mobility, interface parameter, time step      */
  int dtype;             /* CHX_F64 or CHX_F32_REFINED (see below)       */
  int refine_passes;     /* 1..3 for CHX_F32_REFINED, ignored for FP64    */
  int scheme;            /* CHX_SCHEME_P1 (above) or CHX_SCHEME_P2 (below) */
} chx_ch_params;

/* scheme CHX_SCHEME_P2: the thesis's own delta-form scheme (Ch.3
 * eq. 3:ch_adi), with Cbar = 2 C^n - C^{n-1}:
 *   r = -2/3 (C^n - C^{n-1}) - 2/3 D gamma dt Lap^2 Cbar + 2/3 D dt Lap (C^3 - C)^n
 *   (I + s' P_x)(I + s' P_y) v = r,  s' = 2/3 D gamma dt / h^4,  C^{n+1} = Cbar + v,
 * Lap the 5-point and Lap^2 the 13-point (5 x 5) second-order stencils.  It
 * needs two states and is advanced by ch_adi_step_p2; FP64 only. */
#define CHX_SCHEME_P1 0
#define CHX_SCHEME_P2 1

/* dtype CHX_F32_REFINED: the right-hand side is formed in FP64, the column
 * and row sweeps run in FP32 (FP32 copies of the factorisation), and
 * refine_passes (1..3) passes of R = r - (I + sx Px)(I + sy Py) c in FP64,
 * c += (FP32 solve of R) recover FP64 accuracy.  It needs the chunked shapes
 * (nx % 64 == 0, ny % 32 == 0, nx <= 8192), else CHX_EINVAL; ch_create
 * returns CHX_EREFINE when 4 (kappa_x + kappa_y) 2^-24 >= 1 (the two
 * directions' condition numbers: no contraction of the error per pass).
 *
 * ch_create: factor both directions once and pick the kernel shapes.
 * ch_destroy: free (NULL accepted).  ch_ws_bytes: workspace for ch_adi_step. */
int ch_create(const chx_ch_params* prm, chx_ch* out);
int ch_destroy(chx_ch h);
size_t ch_ws_bytes(chx_ch h);

/* ch_adi_step: advance c_inout (device, nx x ny, leading dimension ld >= nx)
 *   by nsteps >= 1 ADI steps in place.  ws (device) holds ch_ws_bytes(h)
 *   bytes; its contents are scratch between calls.  diag_out (device, may be
 *   NULL) receives 2*(nsteps+1) doubles: mass and free energy of the state
 *   before each step and after the last (as ch_diagnostics defines them).
 *   Asynchronous on stream s.  Calls sharing ws must not overlap. */
int ch_adi_step(chx_ch h, double* c_inout, long ld, int nsteps,
                double* diag_out, void* ws, size_t ws_bytes, chx_stream s);

/* ch_adi_step_p2: advance a CHX_SCHEME_P2 handle's two states in place by
 *   nsteps >= 1 steps: on entry c_inout = C^n and cprev_inout = C^{n-1} (pass
 *   a copy of C^0 as C^{-1} to start, the thesis's choice), on exit
 *   C^{n+nsteps} and C^{n+nsteps-1}.  Both device arrays nx x ny with leading
 *   dimension ld >= nx, not overlapping; ws, diag_out and the stream as for
 *   ch_adi_step.  CHX_EINVAL on a P1 handle (and ch_adi_step, ch_adi_step_timed
 *   return CHX_EINVAL on a P2 handle). */
int ch_adi_step_p2(chx_ch h, double* c_inout, double* cprev_inout, long ld,
                   int nsteps, double* diag_out, void* ws, size_t ws_bytes,
                   chx_stream s);

/* ch_adi_step_timed: ch_adi_step with a HIP event recorded on stream s
 *   around every kernel of every sample_every-th step (>= 1; 1 = every step)
 *   and around the final launches; synchronises s and returns, per phase,
 *   the summed kernel time in milliseconds (phase_ms, host, 4 doubles) and the
 *   number of launches (phase_launches, host, 4 ints).  Phases: 0 column pass
 *   (right-hand side + column sweeps), 1 column separator system, 2 row solves,
 *   3 finalize and diagnostic reductions; on the single-workgroup small-grid
 *   path its one launch counts as phase 0; with the split row pass
 *   (CHX_TUNE_ROW_SPLIT >= 0) phase 2 is the launch that runs the separators
 *   and the interior rows, phase 1 the separator rows.  For measurement; the events add a
 *   little overhead between kernels. */
int ch_adi_step_timed(chx_ch h, double* c_inout, long ld, int nsteps,
                      double* diag_out, void* ws, size_t ws_bytes, chx_stream s,
                      int sample_every, double* phase_ms, int* phase_launches);

/* Kernel choices of the FP64 step (autotuning).
 * CHX_TUNE_SMALL_PATH: grids with nx % 64 == 0, ny % 32 == 0, nx ny <= 16384
 *   and an LDS footprint of 9.25 bytes per point (151.5 KB at 128 x 128) that
 *   the device's per-workgroup LDS holds run every step of a call in ONE
 *   workgroup with the field resident in LDS (value 1, the default where it
 *   fits); value 0 selects the multi-kernel path.  The two paths apply the
 *   column correction at different times and agree to rounding, not bit for
 *   bit.  Setting 1 where it does not fit is CHX_EINVAL.
 * CHX_TUNE_REDUCED_SHAPE: tile shape of the multi-kernel path's column
 *   separator kernel (0 .. CHX_NUM_REDUCED_SHAPES-1: waves per block x chunks
 *   per wave x window entries staged at once, or, for the last three, every
 *   chunk of 32 or 16 systems per block, which loads each separator part
 *   once; a shape that does not fit the handle's chunk count or the LDS
 *   runs as shape 0).  ch_create times every
 *   candidate inside whole steps (column pass, separators, rows, for each
 *   chunk length, with the per-step mass and energy) on zeroed scratch
 *   buffers of the handle's size, times the fastest three again from longer
 *   graphs, and keeps the fastest (a windowed shape only if it beats the
 *   best whole-column one by more than 1 %); the choices (this shape, the
 *   row split, the column order and the chunk lengths)
 *   are kept per size for the life of the process and in a tuning cache
 *   file across processes: $CHX_TUNE_CACHE, else
 *   $XDG_CACHE_HOME/chx/tuning.txt, else $HOME/.cache/chx/tuning.txt (one
 *   text line per device architecture and size; CHX_TUNE_CACHE=0 turns the
 *   file off).  Environment variable CHX_AUTOTUNE=0 skips the timing and
 *   the file (shape 0).
 *   Every shape sums the same terms in the same order, so results are
 *   bitwise identical whatever the shape.
 * CHX_TUNE_ROW_SPLIT: -1 runs the column separator kernel and then the row
 *   pass; -2 (CHX_ROW_SPLIT_OVERLAP) runs the separators and then the
 *   separator rows (the last two of every column chunk) on a second stream
 *   of the handle while the other rows, which need no separator, are solved
 *   on the caller's stream (joined by events before the next step; the
 *   steps ch_adi_step_timed times keep the -1 order so that their kernel
 *   timings stay meaningful), for either chunk length; for rows of 4096 or
 *   8192 points with 32-point chunks in both directions, 0 ..
 *   CHX_NUM_SPLIT_SHAPES-1 run the separators in the same launch as the
 *   interior rows, in that tile shape, then the separator rows.  Chosen by
 *   the same timing as the tile shape.  Results are bitwise identical
 *   whatever the order.
 * CHX_TUNE_COLUMN_ORDER: order in which the multi-kernel path's column pass
 *   (and the pass that writes the final state) numbers its tiles of 256
 *   columns x 32 rows (0 .. CHX_NUM_COLUMN_ORDERS-1): 0 row-major; 1 each of
 *   the 8 XCDs (which receive consecutive workgroups round robin) works a
 *   horizontal band of chunk rows; 2 each XCD works whole column blocks, chunk
 *   after chunk.  Results are bitwise identical whatever the order.
 * CHX_TUNE_GRAPH: 1 makes ch_adi_step capture the launches of a call into a
 *   hipGraph (on a private stream of the handle) and replay it, re-capturing
 *   only when the field pointer, ld, nsteps, diag_out or ws differ from the
 *   captured call's; the graph is kept until the handle is destroyed or a
 *   tuning choice changes.  0 (the default) launches every kernel from the
 *   host.  Handles with Cahn-Hilliard-Cook forcing and the single-workgroup
 *   path always launch directly.  Results are bitwise identical either way.
 * CHX_TUNE_COLUMN_CHUNK, CHX_TUNE_ROW_CHUNK: length of the chunks that the
 *   multi-kernel FP64 path's column and row solves are partitioned into
 *   (each chunk swept on its own, its last two unknowns the separators
 *   that the separator system couples): 32, or 16
 *   where the length is a multiple of 16 (and for rows at most 4096 points).
 *   Shorter chunks halve the serial sweep of each workgroup and double the
 *   separators; on small grids, where one round of workgroups covers the
 *   field, that wins.  Chosen by the same timing as the tile shape; 16 needs
 *   the row split -1 or -2 (the fused split shapes need 32 in both
 *   directions: CHX_EINVAL otherwise).  The two lengths solve the same systems with different
 *   rounding: results agree to rounding, not bitwise.
 * ch_get_tuning: *value = the current choice of `what`.
 * ch_set_tuning: set it from now on; CHX_EINVAL for a NULL handle, an unknown
 *   `what` or a value out of range.  Not to be called while work of h is
 *   queued on a stream that is being captured. */
#define CHX_TUNE_REDUCED_SHAPE 0
#define CHX_TUNE_SMALL_PATH 1
#define CHX_TUNE_ROW_SPLIT 2
#define CHX_NUM_REDUCED_SHAPES 15
#define CHX_NUM_SPLIT_SHAPES 3
#define CHX_ROW_SPLIT_OVERLAP (-2)
#define CHX_TUNE_COLUMN_ORDER 3
#define CHX_NUM_COLUMN_ORDERS 3
#define CHX_TUNE_GRAPH 4
#define CHX_TUNE_COLUMN_CHUNK 5
#define CHX_TUNE_ROW_CHUNK 6
int ch_get_tuning(chx_ch h, int what, int* value);
int ch_set_tuning(chx_ch h, int what, int value);

/* Cahn-Hilliard-Cook forcing (Ch.7): C_t = D Lap(C^3 - C - gamma Lap C) + eta,
 * eta_ij = sqrt(sigma / (dx dy dt)) div rho_ij, rho a 2-vector of N(0,1)
 * numbers per point and step drawn by Box-Muller from two uniforms of a
 * counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k of
 * the sequence whose state starts at mix(seed), u = ((out >> 11) + 1/2) 2^-53,
 * k = ((step * ny + j) * nx + i) * 2 + component.  The divergence takes
 * forward differences (periodic, so the forcing conserves mass); dt * eta is
 * added to the explicit right-hand side.
 * ch_set_noise: sigma > 0 turns the forcing on for a P1 FP64 handle of the
 *   chunked shapes (nx % 64 == 0, ny % 32 == 0; else CHX_EINVAL), sigma = 0
 *   turns it off; step0 is the counter of the next step.  Every step of
 *   ch_adi_step advances the counter, so a run split over several calls
 *   draws the same numbers as one call.  The draws are made inside the step
 *   kernels (no extra workspace), the single-workgroup path included.  Not
 *   for graph capture (the counter is a launch argument).
 * ch_get_noise_step: the counter of the next step. */
int ch_set_noise(chx_ch h, double sigma, unsigned long long seed,
                 unsigned long long step0);
int ch_get_noise_step(chx_ch h, unsigned long long* step);

/* ch_diagnostics: mass = dx dy sum c and discrete free energy
 *   F = dx dy sum[(c^2-1)^2/4 + gamma/2 ((D+x c)^2 + (D+y c)^2)] of the field c
 *   (device), by a fixed-order reduction (bitwise repeatable).  Synchronises
 *   stream s; writes the host doubles *mass and *energy.  Returns
 *   CHX_ENONFINITE if either is NaN or infinite. */
int ch_diagnostics(chx_ch h, const double* c, long ld, double* mass,
                   double* energy, chx_stream s);

/* ch_energy_decay_rate: the free-energy decay rate of Ch.7 eq. 7:betaN,
 *   beta = -(t / F) dF/dt, of every run and state of a stepping call's
 *   diagnostics.  diag (device): nruns blocks of 2 nstates doubles laid out as
 *   ch_adi_step (nruns = 1) or ch_ensemble_step write them (mass, energy of
 *   state k at r*2*nstates + 2k + {0,1}); state k is at time t0 + k dt.
 *   beta (device, nruns * nstates doubles, must not overlap diag):
 *   beta[r*nstates + k].  dF/dt by second-order differences, central inside,
 *   three-point one-sided at the first and last state (exact for quadratic
 *   F).  nstates >= 3 and dt > 0, else CHX_EINVAL.  Asynchronous on s. */
int ch_energy_decay_rate(const double* diag, int nruns, int nstates, double t0,
                         double dt, double* beta, chx_stream s);

/* ch_moments: coarsening measure of Ch.3 "Numerical Results": out (host, 3
 *   doubles) = <C>, <C^2> and s = 1 / (1 - <C^2>), the averages by composite
 *   Simpson's rule in each direction of the periodic grid (weights 2/3 on
 *   even, 4/3 on odd indices; nx and ny even, else CHX_EINVAL), fixed-order
 *   reduction.  Synchronises stream s; CHX_ENONFINITE on NaN or Inf. */
int ch_moments(chx_ch h, const double* c, long ld, double* out, chx_stream s);

/* ch_k1: the second coarsening measure of Ch.3 "Numerical Results",
 *   k1 = sum |C^(k)|^2 / sum |k|^-1 |C^(k)|^2 over the discrete wavevectors
 *   k = (2 pi m / lx, 2 pi l / ly) other than k = 0, C^ the discrete Fourier
 *   transform of c (a library real-to-complex FFT, then a fixed-order
 *   reduction kernel).  *k1 (host).  The first call makes the transform plan
 *   and a buffer of about two fields, kept by the handle.  Synchronises
 *   stream s; CHX_ENONFINITE if the field has no k != 0 content. */
int ch_k1(chx_ch h, const double* c, long ld, double* k1, chx_stream s);

/* ------------------------------------------------------------------------
 * Uneven ensembles (the thesis's statistical ensembles of coarsening runs,
 * Ch.7 "2D Cahn--Hilliard Methodology", and its proposal of variable system
 * lengths within a batch with one stored LHS per distinct matrix, Ch.8
 * "Future Work").  Many independent
 * runs, each with its own grid and parameters, advance together: every
 * kernel launch covers all runs (one launch per phase per step), runs of the
 * same grid and parameters share one factorisation, and with use_graph the
 * whole nsteps sequence is captured once in a hipGraph and replayed.
 *
 * ch_ensemble_create: nruns >= 1 parameter sets (prm, host array), all with
 *   CHX_SCHEME_P1 and one dtype.  CHX_F64: nx % 64 == 0, ny % 32 == 0,
 *   nx <= 8192, at most 8 distinct (grid, D, gamma, dt) classes; ensembles
 *   solve with 32-point chunks, so a run advances bitwise as a single
 *   handle whose CHX_TUNE_COLUMN_CHUNK and CHX_TUNE_ROW_CHUNK are 32 would
 *   (to rounding as one tuned to 16).
 *   CHX_F32_REFINED (the precision pattern of ch_create's refined step):
 *   each run as ch_create accepts it (refine_passes may differ between
 *   runs), at most 8 distinct (grid, D, gamma, dt) classes; every phase of
 *   the refined step is one launch for all runs (refinement pass k covers
 *   the runs with at least k passes), and each run advances bitwise as a
 *   single refined handle would.  Otherwise CHX_EINVAL (CHX_EREFINE for a
 *   class ch_create would refuse with it).
 * ch_ensemble_ws_bytes: device workspace for ch_ensemble_step.
 * ch_ensemble_step: advance every run by nsteps >= 1 steps in place.
 *   c_runs: host array of nruns device pointers (row-major fields); ld_runs:
 *   host array of leading dimensions (NULL = nx).  diag_out (device, may be
 *   NULL): run r's mass and free energy before each step and after the last
 *   at diag_out[r*2*(nsteps+1) + 2*k + {0,1}].  use_graph != 0 replays a
 *   cached hipGraph of the call (re-captured when nsteps, diag_out or ws
 *   change).  Asynchronous on s, except that a change of the run pointers
 *   synchronises s before the run table is updated.  Calls on one handle
 *   must not overlap.
 */
typedef struct chx_ens_s* chx_ens;
int ch_ensemble_create(int nruns, const chx_ch_params* prm, chx_ens* out);
int ch_ensemble_destroy(chx_ens e);
/* ch_ensemble_get_tuning / ch_ensemble_set_tuning: what =
 *   CHX_TUNE_REDUCED_SHAPE, the tile shape of an FP64 ensemble's separator
 *   kernel (0 .. CHX_NUM_ENS_REDUCED_SHAPES-1: 8 waves x 4 chunks, 8 x 1,
 *   4 x 2, 4 x 4 per block; small grids have few chunks per column, which
 *   the larger blocks leave mostly idle).  ch_ensemble_create times every
 *   shape on the ensemble's own runs (column pass and separators from a
 *   captured graph; CHX_AUTOTUNE=0 keeps 0) and keeps the fastest.  Every
 *   shape sums the same terms in the same order: results are bitwise
 *   identical whatever the shape.  Setting synchronises the device (queued
 *   calls may still read the work items) and drops a captured graph.
 *   CHX_EINVAL for refined ensembles, another `what` or a shape out of
 *   range or whose LDS does not fit. */
#define CHX_NUM_ENS_REDUCED_SHAPES 4
int ch_ensemble_get_tuning(chx_ens e, int what, int* value);
int ch_ensemble_set_tuning(chx_ens e, int what, int value);
size_t ch_ensemble_ws_bytes(chx_ens e);
int ch_ensemble_step(chx_ens e, double* const* c_runs, const long* ld_runs,
                     int nsteps, double* diag_out, void* ws, size_t ws_bytes,
                     int use_graph, chx_stream s);

/* ch_ensemble_set_noise: Cahn-Hilliard-Cook forcing (Ch.7) for every run of
 *   an FP64 ensemble: intensity sigma >= 0 (0 switches it off), run r drawing
 *   with seeds[r] (host array of nruns) and the ensemble's step counter,
 *   starting at step0; the draws are those ch_set_noise defines, so run r
 *   gets the same forcing as a single handle given (sigma, seeds[r], step0).
 *   The counter lives on the device and every call of ch_ensemble_step moves
 *   it on by nsteps, graph replays included (the draws are made inside the
 *   step kernels).  Synchronises the device.  CHX_EINVAL for sigma < 0 or
 *   not finite, seeds NULL with sigma > 0, or sigma > 0 on an FP32-refined
 *   ensemble.
 * ch_ensemble_get_noise_step: the counter's value after the calls so far. */
int ch_ensemble_set_noise(chx_ens e, double sigma, const unsigned long long* seeds,
                          unsigned long long step0);
int ch_ensemble_get_noise_step(chx_ens e, unsigned long long* step);

/* Per-run coarsening measures of an ensemble (Ch.3 "Numerical Results",
 * gathered per run for the ensemble statistics of Ch.7), for the fields in
 * c_runs / ld_runs laid out as for ch_ensemble_step:
 * ch_ensemble_moments: out (host, 3 per run) = <C>, <C^2>, s = 1/(1 - <C^2>)
 *   of run r at out[3r..3r+2], as ch_moments computes them (every run's nx
 *   and ny even, else CHX_EINVAL).
 * ch_ensemble_k1: k1 (host, 1 per run) as ch_k1 defines it; the runs of one
 *   grid size share one batched real-to-complex transform.
 * The first call of each makes its buffers (and the transform plans), kept
 * by the handle.  Both synchronise stream s and return CHX_ENONFINITE if any
 * run's value is NaN or infinite (the others are still written). */
int ch_ensemble_moments(chx_ens e, double* const* c_runs, const long* ld_runs,
                        double* out, chx_stream s);
int ch_ensemble_k1(chx_ens e, double* const* c_runs, const long* ld_runs,
                   double* k1, chx_stream s);

/* ------------------------------------------------------------------------
 * Host-side plan inspection (no device work; usable without a GPU).  They
 * return the tables that penta_factor / tri_factor compute and upload, so the
 * host factorisation can be checked on a CPU.  P = 2 (coef = a,b,c,d,e) or
 * P = 1 (coef = a,b,c); the matrix is cyclic.
 *
 * chx_host_chunk_tables: tables for chunks of m unknowns (n % m == 0,
 *   m >= 3P): per interior position p < m-P, 8 values {1/alpha, L(p,p-1),
 *   R(p,p+1), R(p,p+2), Zl_0, Zl_1, Zr_0, Zr_1} (rec, capacity rec_cap
 *   doubles); reduced-system blocks B_d, d = dlo..dlo+dcount-1, as 2x2
 *   row-major (blocks, capacity blocks_cap doubles); info[0..3] = {m-P, n/m,
 *   dlo, dcount}.  Arrays that are NULL or too small are skipped.
 * chx_host_whole_tables: bordering tables of the whole system: per position
 *   i < mi, {1/alpha, L(i,i-1), R(i,i+1), R(i,i+2), q_0, q_1, Z_0, Z_1}; minv =
 *   [C22 - h^T E^{-1} k]^{-1} (2x2, row-major); *mi_out = n-P (periodic) or n.
 */
int chx_host_chunk_tables(int P, const double* coef, int n, int m, double* rec,
                          int rec_cap, double* blocks, int blocks_cap, int* info);
int chx_host_whole_tables(int P, const double* coef, int n, int periodic,
                          double* rec, int rec_cap, double* minv, int* mi_out);

#ifdef __cplusplus
}
#endif
#endif
