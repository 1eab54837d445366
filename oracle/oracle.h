/*
 * oracle.h -- plain serial FP64 CPU oracle for the 2D periodic Cahn-Hilliard
 * ADI step and the batched cyclic banded solves inside it.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library
 * against the paper.  Only the test suite, the smoke entry point and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or constant with the HIP library, and the library never calls it.
 *
 * Everything here is written from the thesis (A. Gloster, arXiv 2101.06550):
 *   - cyclic pentadiagonal systems by Navon's bordering of the last two
 *     unknowns (Ch.4, "The pentadiagonal matrix system", eqs. (solve) and
 *     (first_two)) and the LR factorisation with forward and back sweeps
 *     (Ch.4, "Solution of the pentadiagonal system");
 *   - cyclic tridiagonal systems by the Thomas algorithm with
 *     pre-factorisation (Ch.5, "Tridiagonal Inversion Algorithm") and the
 *     Sherman-Morrison correction (Ch.5, "Periodic Tridiagonal Matrix");
 *   - cuSten-style 2D stencils with periodic / non-periodic boundaries
 *     (Ch.3, "Software API");
 *   - the Cahn-Hilliard equation and its free energy (Ch.2, eq. 2:ch) and
 *     the ADI splitting into row and column solves (Ch.3, eq. 3:ch_adi).
 *
 * Compiled with gcc -O2 -ffp-contract=off (no FMA contraction).  Arrays are
 * row-major with x (index i) fastest: c[j*nx + i].
 */
#ifndef CH_ORACLE_H
#define CH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- general (non-cyclic) banded solves, per-row coefficient arrays ---- */

/* LR factorisation of a strictly pentadiagonal n x n matrix (n >= 3).
 * Row i holds a[i] x[i-2] + b[i] x[i-1] + c[i] x[i] + d[i] x[i+1] + e[i] x[i+2]
 * (entries that fall outside the matrix are ignored).  Outputs the factors
 * alpha, beta, gam (gamma), del (delta), eps (epsilon) of Ch.4; returns 0, or
 * -1 if a pivot alpha_i is zero or not finite. */
int orc_penta_lr_factor(int n, const double* a, const double* b, const double* c,
                        const double* d, const double* e, double* alpha,
                        double* beta, double* gam, double* del, double* eps);
/* Solve L g = f (forward) then R x = g (back) with the factors above. */
void orc_penta_lr_solve(int n, const double* alpha, const double* beta,
                        const double* gam, const double* del, const double* eps,
                        const double* f, double* x);

/* Thomas algorithm with pre-factorisation (Ch.5): row i holds
 * a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = f[i].  chat/den are outputs of the
 * pre-factorisation (den[i] = b_i - a_i chat_{i-1}). */
int orc_tri_prefactor(int n, const double* a, const double* b, const double* c,
                      double* chat, double* den);
void orc_tri_solve(int n, const double* a, const double* chat,
                   const double* den, const double* f, double* x);

/* ---- cyclic constant-coefficient solves ---- */

/* Precomputed Navon bordering for the cyclic pentadiagonal matrix whose row i
 * is a x[i-2] + b x[i-1] + c x[i] + d x[i+1] + e x[i+2] (indices mod n), n>=5. */
typedef struct {
  int n, m;                 /* m = n - 2 = size of the leading block E       */
  double a, b, c, d, e;
  double *alpha, *beta, *gam, *del, *eps;   /* LR factors of E (length m)   */
  double *kcol0, *kcol1;    /* the two columns of k (E x + k x_tail = f)     */
  double *q0, *q1;          /* rows of h^T E^{-1}, i.e. q = E^{-T} h          */
  double minv[2][2];        /* [C22 - h^T E^{-1} k]^{-1}                      */
} orc_cpenta;

int  orc_cpenta_prepare(int n, double a, double b, double c, double d, double e,
                        orc_cpenta* p);
/* The same for a cyclic matrix whose row i holds its own coefficients
 * a[i] x[i-2] + b[i] x[i-1] + c[i] x[i] + d[i] x[i+1] + e[i] x[i+2]. */
int  orc_cpenta_prepare_rows(int n, const double* a, const double* b,
                             const double* c, const double* d, const double* e,
                             orc_cpenta* p);
void orc_cpenta_apply(const orc_cpenta* p, const double* f, double* x);
void orc_cpenta_free(orc_cpenta* p);
/* One-shot convenience: x = A^{-1} f; returns 0 or <0 on bad arguments. */
int  orc_cyclic_penta_solve(int n, double a, double b, double c, double d,
                            double e, const double* f, double* x);

/* Cyclic tridiagonal (row i: a x[i-1] + b x[i] + c x[i+1], mod n, n >= 3). */
typedef struct {
  int n;
  double a, b, c;
  double *sub, *chat, *den; /* pre-factorisation of A' (Sherman-Morrison)   */
  double *z;                /* z = A'^{-1} u                                  */
  double vz;                /* v . z                                          */
} orc_ctri;

int  orc_ctri_prepare(int n, double a, double b, double c, orc_ctri* p);
/* Row i: a[i] x[i-1] + b[i] x[i] + c[i] x[i+1], indices mod n. */
int  orc_ctri_prepare_rows(int n, const double* a, const double* b,
                           const double* c, orc_ctri* p);
void orc_ctri_apply(const orc_ctri* p, const double* f, double* x);
void orc_ctri_free(orc_ctri* p);
int  orc_cyclic_tri_solve(int n, double a, double b, double c, const double* f,
                          double* x);

/* Batches with one matrix per system, interleaved: entry i of system s of
 * every array at [i*ld + s]; x holds the right-hand sides in and the
 * solutions out.  periodic != 0: rows wrap mod n (penta n >= 5, tri n >= 3);
 * otherwise entries outside the matrix are ignored (penta n >= 3, tri n >= 2).
 * Returns 0, -1 on bad arguments, -(2 + s) if system s cannot be factored. */
int orc_penta_rows_batch(int n, int batch, long ld, int periodic,
                         const double* a, const double* b, const double* c,
                         const double* d, const double* e, double* x);
int orc_tri_rows_batch(int n, int batch, long ld, int periodic,
                       const double* a, const double* b, const double* c,
                       double* x);

/* Batched line solves over a 2D array: direction 0 = along x (each row j is
 * one system, elements contiguous), direction 1 = along y (each column i is
 * one system, stride nx).  In place. */
int orc_cpenta_lines(int nx, int ny, int direction, double a, double b,
                     double c, double d, double e, double* data);
int orc_ctri_lines(int nx, int ny, int direction, double a, double b, double c,
                   double* data);

/* ---- stencils ---- */

/* out[j][i] = sum_{q=-top..bottom} sum_{p=-left..right}
 *               w[(q+top)*(left+right+1) + (p+left)] * pre(in[j+q][i+p])
 * where pre(v) = v (premap 0) or v*v*v - v (premap 1).  Weights are listed
 * from the top-left of the stencil, left to right in i, row by row in j
 * (Ch.3, "Application of cuSten"), "top" being the smaller j.
 * periodic != 0: indices wrap.  periodic == 0: only points whose whole
 * stencil lies inside the array are written; the others keep out's value. */
int orc_stencil2d(const double* in, double* out, int nx, int ny,
                  const double* w, int left, int right, int top, int bottom,
                  int periodic, int premap);

/* ---- Cahn-Hilliard ---- */

/* Explicit right-hand side of the first-order ADI scheme on the periodic
 * box [0,lx) x [0,ly):
 *   r = c + D dt Lap5(c^3 - c) - 2 D gamma dt (dxx dyy) c
 * with the 5-point Laplacian and the 9-point cross stencil. */
void orc_ch_rhs(const double* c, double* r, int nx, int ny, double lx,
                double ly, double D, double gamma, double dt);
/* One ADI step in place: r = rhs(c); rows solve (I + sx P); columns solve
 * (I + sy P), P = circ(1,-4,6,-4,1), s = D gamma dt / h^4. */
int orc_ch_step(double* c, int nx, int ny, double lx, double ly, double D,
                double gamma, double dt);
/* Mass dx dy sum(c) (compensated sum) and the discrete free energy
 *   dx dy sum[ (c^2-1)^2/4 + gamma/2 ((D+x c)^2 + (D+y c)^2) ]. */
/* Ch.3 eq. 3:ch_adi (the thesis's own delta-form scheme with 2/3 factors):
 * right-hand side from C^n (c) and C^{n-1} (cprev), and one step that
 * advances both in place (cprev <- C^n, c <- C^{n+1}). */
void orc_ch2_rhs(const double* c, const double* cprev, double* r, int nx,
                 int ny, double lx, double ly, double D, double gamma,
                 double dt);
int orc_ch2_step(double* c, double* cprev, int nx, int ny, double lx,
                 double ly, double D, double gamma, double dt);
/* Batched 1D periodic schemes (unknown i of system s at x[i*batch + s]),
 * one step in place: kind 0 Crank-Nicolson hyperdiffusion C_t = -a C_xxxx
 * (Ch.4), kind 1 Crank-Nicolson diffusion C_t = a C_xx (Ch.5), kind 2 1D
 * Cahn-Hilliard with gamma = a and mobility D (Ch.6 eq. 6:1Dnumerical). */
int orc_batch1d_step(int kind, double* x, int n, int batch, double L,
                     double dt, double a, double D);
/* Ch.7 Cahn-Hilliard-Cook forcing: counter-based SplitMix64 uniform in
 * (0, 1), the Box-Muller N(0,1) vector field rho of one step, the increment
 * dt * eta (eta = sqrt(sigma/(dx dy dt)) div rho, forward differences), and
 * one step of the first-order ADI scheme with dt * eta added to its
 * right-hand side. */
double orc_sm_uniform(uint64_t seed, uint64_t k);
void orc_cook_rho(double* rx, double* ry, int nx, int ny, uint64_t seed,
                  uint64_t step);
void orc_cook_increment(double* out, int nx, int ny, double lx, double ly,
                        double dt, double sigma, uint64_t seed, uint64_t step);
int orc_ch_step_cook(double* c, int nx, int ny, double lx, double ly, double D,
                     double gamma, double dt, double sigma, uint64_t seed,
                     uint64_t step);
/* Ch.3 "Numerical Results": spatial average <C^power> (power 1 or 2) by
 * composite Simpson's rule on the periodic grid (nx, ny even); s(t) =
 * 1 / (1 - <C^2>). */
double orc_simpson_mean(const double* c, int nx, int ny, int power);
double orc_ch_mass(const double* c, int nx, int ny, double lx, double ly);
double orc_ch_energy(const double* c, int nx, int ny, double lx, double ly,
                     double gamma);
/* Free-energy decay rate beta_k = -(t_k / F_k) (dF/dt)_k, t_k = t0 + k dt,
 * second-order differences (Ch.7 eq. 7:betaN). */
int orc_energy_decay_rate(const double* F, int n, double t0, double dt, double* beta);

#ifdef __cplusplus
}
#endif
#endif
