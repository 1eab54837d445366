/*
 * oracle.c -- plain serial FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke entry point and the benchmark's CPU-baseline
 * leg load this code.  It shares nothing with the HIP library.  Every routine
 * follows the thesis (arXiv 2101.06550) in its own order and notation; the
 * section each one follows is named above it.  Build: gcc -O2
 * -ffp-contract=off -shared -fPIC (no FMA contraction, no vector intrinsics).
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Ch.4 "Solution of the pentadiagonal system": A = L R with L lower
 * (diagonals epsilon, beta, alpha) and R unit upper (diagonals gamma, delta).
 * The steps are the paper's, written as one loop in which the terms that
 * refer to rows before the first are absent. */
int orc_penta_lr_factor(int n, const double* a, const double* b, const double* c,
                        const double* d, const double* e, double* alpha,
                        double* beta, double* gam, double* del, double* eps) {
  if (n < 3) return -1;
  for (int i = 0; i < n; ++i) {
    /* beta_i = b_i - a_i gamma_{i-2} */
    double bi = b[i];
    if (i >= 2) bi = bi - a[i] * gam[i - 2];
    beta[i] = (i >= 1) ? bi : 0.0;
    /* alpha_i = c_i - a_i delta_{i-2} - beta_i gamma_{i-1} */
    double al = c[i];
    if (i >= 2) al = al - a[i] * del[i - 2];
    if (i >= 1) al = al - beta[i] * gam[i - 1];
    if (!(al != 0.0) || !isfinite(al)) return -1;
    alpha[i] = al;
    /* gamma_i = (d_i - beta_i delta_{i-1}) / alpha_i, for rows with a d_i */
    if (i <= n - 2) {
      double num = d[i];
      if (i >= 1) num = num - beta[i] * del[i - 1];
      gam[i] = num / al;
    } else {
      gam[i] = 0.0;
    }
    /* delta_i = e_i / alpha_i, for rows with an e_i */
    del[i] = (i <= n - 3) ? e[i] / al : 0.0;
    /* epsilon_i = a_i */
    eps[i] = (i >= 2) ? a[i] : 0.0;
  }
  return 0;
}

void orc_penta_lr_solve(int n, const double* alpha, const double* beta,
                        const double* gam, const double* del, const double* eps,
                        const double* f, double* x) {
  /* forward: f = L g, g_i = (f_i - eps_i g_{i-2} - beta_i g_{i-1}) / alpha_i */
  double* g = (double*)malloc(sizeof(double) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    double num = f[i];
    if (i >= 2) num = num - eps[i] * g[i - 2];
    if (i >= 1) num = num - beta[i] * g[i - 1];
    g[i] = num / alpha[i];
  }
  /* back: R x = g, x_i = g_i - gamma_i x_{i+1} - delta_i x_{i+2} */
  for (int i = n - 1; i >= 0; --i) {
    double v = g[i];
    if (i + 1 <= n - 1) v = v - gam[i] * x[i + 1];
    if (i + 2 <= n - 1) v = v - del[i] * x[i + 2];
    x[i] = v;
  }
  free(g);
}

/* ------------------------------------------------------------------------ */
/* Ch.5 "Tridiagonal Inversion Algorithm": Thomas with pre-factorisation.
 * chat_1 = c_1/b_1, chat_i = c_i / (b_i - a_i chat_{i-1});
 * dhat_i = (f_i - a_i dhat_{i-1}) / (b_i - a_i chat_{i-1});
 * x_N = dhat_N, x_i = dhat_i - chat_i x_{i+1}
 * (the back substitution as it must read; the printed form has a typo). */
int orc_tri_prefactor(int n, const double* a, const double* b, const double* c,
                      double* chat, double* den) {
  if (n < 2) return -1;
  for (int i = 0; i < n; ++i) {
    double dn = b[i];
    if (i >= 1) dn = dn - a[i] * chat[i - 1];
    if (!(dn != 0.0) || !isfinite(dn)) return -1;
    den[i] = dn;
    chat[i] = (i <= n - 2) ? c[i] / dn : 0.0;
  }
  return 0;
}

void orc_tri_solve(int n, const double* a, const double* chat,
                   const double* den, const double* f, double* x) {
  double* dh = (double*)malloc(sizeof(double) * (size_t)n);
  for (int i = 0; i < n; ++i) {
    double num = f[i];
    if (i >= 1) num = num - a[i] * dh[i - 1];
    dh[i] = num / den[i];
  }
  x[n - 1] = dh[n - 1];
  for (int i = n - 2; i >= 0; --i) x[i] = dh[i] - chat[i] * x[i + 1];
  free(dh);
}

/* ------------------------------------------------------------------------ */
/* Ch.4 "The pentadiagonal matrix system": the cyclic matrix, its leading
 * (n-2)x(n-2) block E, the coupling blocks k (columns n-2, n-1 restricted to
 * rows 0..n-3) and h^T (rows n-2, n-1 restricted to columns 0..n-3), and the
 * 2x2 block C22, all read off the periodic pattern entry by entry. */
static double cyc_penta_entry(const double* a, const double* b, const double* c,
                              const double* d, const double* e, int n, int row,
                              int col) {
  /* row `row` of the periodic matrix holds a x[row-2] + b x[row-1] + c x[row]
   * + d x[row+1] + e x[row+2], indices mod n, each coefficient of that row */
  int off = ((col - row) % n + n) % n;
  double v = 0.0;
  if (off == 0) v = v + c[row];
  if (off == 1) v = v + d[row];
  if (off == 2) v = v + e[row];
  if (off == n - 2) v = v + a[row];
  if (off == n - 1) v = v + b[row];
  return v;
}

int orc_cpenta_prepare_rows(int n, const double* a, const double* b,
                            const double* c, const double* d, const double* e,
                            orc_cpenta* p) {
  if (n < 5 || !p) return -1;
  memset(p, 0, sizeof(*p));
  const int m = n - 2;
  p->n = n; p->m = m;
  size_t sz = sizeof(double) * (size_t)m;
  p->alpha = (double*)malloc(sz); p->beta = (double*)malloc(sz);
  p->gam = (double*)malloc(sz);   p->del = (double*)malloc(sz);
  p->eps = (double*)malloc(sz);
  p->kcol0 = (double*)malloc(sz); p->kcol1 = (double*)malloc(sz);
  p->q0 = (double*)malloc(sz);    p->q1 = (double*)malloc(sz);

  /* bands of E and of E^T */
  double *ea = (double*)calloc(m, 8), *eb = (double*)calloc(m, 8),
         *ec = (double*)calloc(m, 8), *ed = (double*)calloc(m, 8),
         *ee = (double*)calloc(m, 8);
  double *ta = (double*)calloc(m, 8), *tb = (double*)calloc(m, 8),
         *tc = (double*)calloc(m, 8), *td = (double*)calloc(m, 8),
         *te = (double*)calloc(m, 8);
  for (int i = 0; i < m; ++i) {
    if (i - 2 >= 0) { ea[i] = cyc_penta_entry(a, b, c, d, e, n, i, i - 2);
                      ta[i] = cyc_penta_entry(a, b, c, d, e, n, i - 2, i); }
    if (i - 1 >= 0) { eb[i] = cyc_penta_entry(a, b, c, d, e, n, i, i - 1);
                      tb[i] = cyc_penta_entry(a, b, c, d, e, n, i - 1, i); }
    ec[i] = cyc_penta_entry(a, b, c, d, e, n, i, i);
    tc[i] = ec[i];
    if (i + 1 < m) { ed[i] = cyc_penta_entry(a, b, c, d, e, n, i, i + 1);
                     td[i] = cyc_penta_entry(a, b, c, d, e, n, i + 1, i); }
    if (i + 2 < m) { ee[i] = cyc_penta_entry(a, b, c, d, e, n, i, i + 2);
                     te[i] = cyc_penta_entry(a, b, c, d, e, n, i + 2, i); }
    p->kcol0[i] = cyc_penta_entry(a, b, c, d, e, n, i, n - 2);
    p->kcol1[i] = cyc_penta_entry(a, b, c, d, e, n, i, n - 1);
  }
  int rc = orc_penta_lr_factor(m, ea, eb, ec, ed, ee, p->alpha, p->beta,
                               p->gam, p->del, p->eps);
  /* h^T E^{-1}: its transpose E^{-T} h is found by solving with E^T, which is
   * pentadiagonal as well (the paper notes (E^{-1})^T h = (h^T E^{-1})^T). */
  double *talpha = (double*)malloc(sz), *tbeta = (double*)malloc(sz),
         *tgam = (double*)malloc(sz), *tdel = (double*)malloc(sz),
         *teps = (double*)malloc(sz), *hcol = (double*)malloc(sz);
  if (rc == 0)
    rc = orc_penta_lr_factor(m, ta, tb, tc, td, te, talpha, tbeta, tgam, tdel,
                             teps);
  if (rc == 0) {
    for (int i = 0; i < m; ++i) hcol[i] = cyc_penta_entry(a, b, c, d, e, n, n - 2, i);
    orc_penta_lr_solve(m, talpha, tbeta, tgam, tdel, teps, hcol, p->q0);
    for (int i = 0; i < m; ++i) hcol[i] = cyc_penta_entry(a, b, c, d, e, n, n - 1, i);
    orc_penta_lr_solve(m, talpha, tbeta, tgam, tdel, teps, hcol, p->q1);
    /* M = C22 - h^T E^{-1} k, then its 2x2 inverse (eq. first_two) */
    double m00 = cyc_penta_entry(a, b, c, d, e, n, n - 2, n - 2);
    double m01 = cyc_penta_entry(a, b, c, d, e, n, n - 2, n - 1);
    double m10 = cyc_penta_entry(a, b, c, d, e, n, n - 1, n - 2);
    double m11 = cyc_penta_entry(a, b, c, d, e, n, n - 1, n - 1);
    for (int i = 0; i < m; ++i) {
      m00 = m00 - p->q0[i] * p->kcol0[i];
      m01 = m01 - p->q0[i] * p->kcol1[i];
      m10 = m10 - p->q1[i] * p->kcol0[i];
      m11 = m11 - p->q1[i] * p->kcol1[i];
    }
    double det = m00 * m11 - m01 * m10;
    if (!(det != 0.0) || !isfinite(det)) {
      rc = -1;
    } else {
      p->minv[0][0] = m11 / det;  p->minv[0][1] = -m01 / det;
      p->minv[1][0] = -m10 / det; p->minv[1][1] = m00 / det;
    }
  }
  free(ea); free(eb); free(ec); free(ed); free(ee);
  free(ta); free(tb); free(tc); free(td); free(te);
  free(talpha); free(tbeta); free(tgam); free(tdel); free(teps); free(hcol);
  if (rc != 0) { orc_cpenta_free(p); return -2; }
  return 0;
}

int orc_cpenta_prepare(int n, double a, double b, double c, double d, double e,
                       orc_cpenta* p) {
  if (n < 5 || !p) return -1;
  size_t sz = sizeof(double) * (size_t)n;
  double *ra = (double*)malloc(sz), *rb = (double*)malloc(sz),
         *rc_ = (double*)malloc(sz), *rd = (double*)malloc(sz),
         *re = (double*)malloc(sz);
  for (int i = 0; i < n; ++i) { ra[i] = a; rb[i] = b; rc_[i] = c; rd[i] = d; re[i] = e; }
  int rc = orc_cpenta_prepare_rows(n, ra, rb, rc_, rd, re, p);
  free(ra); free(rb); free(rc_); free(rd); free(re);
  return rc;
}

/* Per right-hand side: the last two unknowns first (eq. first_two), then the
 * rest from E X^ = f^ - k x_tail (eq. solve) by the LR sweeps. */
void orc_cpenta_apply(const orc_cpenta* p, const double* f, double* x) {
  const int n = p->n, m = p->m;
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < m; ++i) {
    s0 = s0 + p->q0[i] * f[i];
    s1 = s1 + p->q1[i] * f[i];
  }
  double r0 = f[n - 2] - s0, r1 = f[n - 1] - s1;
  double t0 = p->minv[0][0] * r0 + p->minv[0][1] * r1;
  double t1 = p->minv[1][0] * r0 + p->minv[1][1] * r1;
  double* fh = (double*)malloc(sizeof(double) * (size_t)m);
  for (int i = 0; i < m; ++i) fh[i] = f[i] - p->kcol0[i] * t0 - p->kcol1[i] * t1;
  orc_penta_lr_solve(m, p->alpha, p->beta, p->gam, p->del, p->eps, fh, x);
  x[n - 2] = t0;
  x[n - 1] = t1;
  free(fh);
}

void orc_cpenta_free(orc_cpenta* p) {
  if (!p) return;
  free(p->alpha); free(p->beta); free(p->gam); free(p->del); free(p->eps);
  free(p->kcol0); free(p->kcol1); free(p->q0); free(p->q1);
  memset(p, 0, sizeof(*p));
}

int orc_cyclic_penta_solve(int n, double a, double b, double c, double d,
                           double e, const double* f, double* x) {
  orc_cpenta p;
  int rc = orc_cpenta_prepare(n, a, b, c, d, e, &p);
  if (rc) return rc;
  orc_cpenta_apply(&p, f, x);
  orc_cpenta_free(&p);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ch.5 "Periodic Tridiagonal Matrix": A = A' + u v^T with
 * u = (-b_0, 0, ..., 0, c_{n-1})^T, v = (1, 0, ..., 0, -a_0/b_0)^T; A' is A
 * without its corners, with 2 b_0 in the first and b_{n-1} + a_0 c_{n-1}/b_0
 * in the last diagonal entry (the thesis's choice gamma = -b, written with
 * the coefficients of the rows they come from).  A' z = u once; per RHS
 * A' y = f and x = y - (v.y)/(1 + v.z) z. */
int orc_ctri_prepare_rows(int n, const double* a, const double* b,
                          const double* c, orc_ctri* p) {
  if (n < 3 || !p || b[0] == 0.0) return -1;
  memset(p, 0, sizeof(*p));
  p->n = n; p->a = a[0]; p->b = b[0]; p->c = c[n - 1];
  size_t sz = sizeof(double) * (size_t)n;
  p->sub = (double*)malloc(sz); p->chat = (double*)malloc(sz);
  p->den = (double*)malloc(sz); p->z = (double*)malloc(sz);
  double *dg = (double*)malloc(sz), *sp = (double*)malloc(sz),
         *u = (double*)calloc(n, 8);
  for (int i = 0; i < n; ++i) { p->sub[i] = a[i]; dg[i] = b[i]; sp[i] = c[i]; }
  dg[0] = 2.0 * b[0];
  dg[n - 1] = b[n - 1] + a[0] * c[n - 1] / b[0];
  int rc = orc_tri_prefactor(n, p->sub, dg, sp, p->chat, p->den);
  if (rc == 0) {
    u[0] = -b[0];
    u[n - 1] = c[n - 1];
    orc_tri_solve(n, p->sub, p->chat, p->den, u, p->z);
    p->vz = p->z[0] - (a[0] / b[0]) * p->z[n - 1];
    if (!(1.0 + p->vz != 0.0)) rc = -1;
  }
  free(dg); free(sp); free(u);
  if (rc) { orc_ctri_free(p); return -2; }
  return 0;
}

int orc_ctri_prepare(int n, double a, double b, double c, orc_ctri* p) {
  if (n < 3 || !p || b == 0.0) return -1;
  size_t sz = sizeof(double) * (size_t)n;
  double *ra = (double*)malloc(sz), *rb = (double*)malloc(sz),
         *rc_ = (double*)malloc(sz);
  for (int i = 0; i < n; ++i) { ra[i] = a; rb[i] = b; rc_[i] = c; }
  int rc = orc_ctri_prepare_rows(n, ra, rb, rc_, p);
  free(ra); free(rb); free(rc_);
  return rc;
}

void orc_ctri_apply(const orc_ctri* p, const double* f, double* x) {
  const int n = p->n;
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  orc_tri_solve(n, p->sub, p->chat, p->den, f, y);
  double vy = y[0] - (p->a / p->b) * y[n - 1];
  double fac = vy / (1.0 + p->vz);
  for (int i = 0; i < n; ++i) x[i] = y[i] - fac * p->z[i];
  free(y);
}

void orc_ctri_free(orc_ctri* p) {
  if (!p) return;
  free(p->sub); free(p->chat); free(p->den); free(p->z);
  memset(p, 0, sizeof(*p));
}

int orc_cyclic_tri_solve(int n, double a, double b, double c, const double* f,
                         double* x) {
  orc_ctri p;
  int rc = orc_ctri_prepare(n, a, b, c, &p);
  if (rc) return rc;
  orc_ctri_apply(&p, f, x);
  orc_ctri_free(&p);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Batches with one matrix per system (Ch.4 "Implementation on GPU": every
 * system its own five diagonals and right-hand side, interleaved).  Entry i
 * of system s of every array sits at [i*ld + s]; x holds the right-hand sides
 * on entry and the solutions on exit.  Non-periodic systems use the LR
 * factorisation and sweeps of Ch.4 (tridiagonal: Thomas with
 * pre-factorisation, Ch.5); periodic ones the bordering of the last two
 * unknowns (Ch.4) or the Sherman-Morrison correction (Ch.5), each built from
 * that system's own rows.  Returns 0, or -1 on bad arguments, or -(2 + s) if
 * the factorisation of system s fails. */
static void gather_col(const double* src, long ld, int s, int n, double* out) {
  for (int i = 0; i < n; ++i) out[i] = src[(long)i * ld + s];
}

int orc_penta_rows_batch(int n, int batch, long ld, int periodic,
                         const double* a, const double* b, const double* c,
                         const double* d, const double* e, double* x) {
  if (batch < 0 || ld < batch || n < (periodic ? 5 : 3)) return -1;
  size_t sz = sizeof(double) * (size_t)n;
  double *ra = (double*)malloc(sz), *rb = (double*)malloc(sz),
         *rc_ = (double*)malloc(sz), *rd = (double*)malloc(sz),
         *re = (double*)malloc(sz), *f = (double*)malloc(sz),
         *xs = (double*)malloc(sz);
  double *al = (double*)malloc(sz), *be = (double*)malloc(sz),
         *ga = (double*)malloc(sz), *de = (double*)malloc(sz),
         *ep = (double*)malloc(sz);
  int rc = 0;
  for (int s = 0; s < batch && rc == 0; ++s) {
    gather_col(a, ld, s, n, ra); gather_col(b, ld, s, n, rb);
    gather_col(c, ld, s, n, rc_); gather_col(d, ld, s, n, rd);
    gather_col(e, ld, s, n, re); gather_col(x, ld, s, n, f);
    if (periodic) {
      orc_cpenta p;
      if (orc_cpenta_prepare_rows(n, ra, rb, rc_, rd, re, &p) != 0) { rc = -(2 + s); break; }
      orc_cpenta_apply(&p, f, xs);
      orc_cpenta_free(&p);
    } else {
      if (orc_penta_lr_factor(n, ra, rb, rc_, rd, re, al, be, ga, de, ep) != 0) { rc = -(2 + s); break; }
      orc_penta_lr_solve(n, al, be, ga, de, ep, f, xs);
    }
    for (int i = 0; i < n; ++i) x[(long)i * ld + s] = xs[i];
  }
  free(ra); free(rb); free(rc_); free(rd); free(re); free(f); free(xs);
  free(al); free(be); free(ga); free(de); free(ep);
  return rc;
}

int orc_tri_rows_batch(int n, int batch, long ld, int periodic,
                       const double* a, const double* b, const double* c,
                       double* x) {
  if (batch < 0 || ld < batch || n < (periodic ? 3 : 2)) return -1;
  size_t sz = sizeof(double) * (size_t)n;
  double *ra = (double*)malloc(sz), *rb = (double*)malloc(sz),
         *rc_ = (double*)malloc(sz), *f = (double*)malloc(sz),
         *xs = (double*)malloc(sz), *chat = (double*)malloc(sz),
         *den = (double*)malloc(sz);
  int rc = 0;
  for (int s = 0; s < batch && rc == 0; ++s) {
    gather_col(a, ld, s, n, ra); gather_col(b, ld, s, n, rb);
    gather_col(c, ld, s, n, rc_); gather_col(x, ld, s, n, f);
    if (periodic) {
      orc_ctri p;
      if (orc_ctri_prepare_rows(n, ra, rb, rc_, &p) != 0) { rc = -(2 + s); break; }
      orc_ctri_apply(&p, f, xs);
      orc_ctri_free(&p);
    } else {
      if (orc_tri_prefactor(n, ra, rb, rc_, chat, den) != 0) { rc = -(2 + s); break; }
      orc_tri_solve(n, ra, chat, den, f, xs);
    }
    for (int i = 0; i < n; ++i) x[(long)i * ld + s] = xs[i];
  }
  free(ra); free(rb); free(rc_); free(f); free(xs); free(chat); free(den);
  return rc;
}

/* Lines of a 2D array: direction 0 solves along x for every row, direction 1
 * along y for every column; one prepared matrix serves every line (the
 * thesis factors a constant matrix once and reuses it). */
static void gather_line(const double* data, int nx, int ny, int dir, int line,
                        double* buf) {
  if (dir == 0) for (int i = 0; i < nx; ++i) buf[i] = data[(size_t)line * nx + i];
  else          for (int j = 0; j < ny; ++j) buf[j] = data[(size_t)j * nx + line];
}
static void scatter_line(double* data, int nx, int ny, int dir, int line,
                         const double* buf) {
  if (dir == 0) for (int i = 0; i < nx; ++i) data[(size_t)line * nx + i] = buf[i];
  else          for (int j = 0; j < ny; ++j) data[(size_t)j * nx + line] = buf[j];
}

int orc_cpenta_lines(int nx, int ny, int direction, double a, double b,
                     double c, double d, double e, double* data) {
  int n = direction == 0 ? nx : ny, lines = direction == 0 ? ny : nx;
  orc_cpenta p;
  int rc = orc_cpenta_prepare(n, a, b, c, d, e, &p);
  if (rc) return rc;
  double *f = (double*)malloc(8 * (size_t)n), *x = (double*)malloc(8 * (size_t)n);
  for (int l = 0; l < lines; ++l) {
    gather_line(data, nx, ny, direction, l, f);
    orc_cpenta_apply(&p, f, x);
    scatter_line(data, nx, ny, direction, l, x);
  }
  free(f); free(x);
  orc_cpenta_free(&p);
  return 0;
}

int orc_ctri_lines(int nx, int ny, int direction, double a, double b, double c,
                   double* data) {
  int n = direction == 0 ? nx : ny, lines = direction == 0 ? ny : nx;
  orc_ctri p;
  int rc = orc_ctri_prepare(n, a, b, c, &p);
  if (rc) return rc;
  double *f = (double*)malloc(8 * (size_t)n), *x = (double*)malloc(8 * (size_t)n);
  for (int l = 0; l < lines; ++l) {
    gather_line(data, nx, ny, direction, l, f);
    orc_ctri_apply(&p, f, x);
    scatter_line(data, nx, ny, direction, l, x);
  }
  free(f); free(x);
  orc_ctri_free(&p);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ch.3 "Software API": a weighted stencil of arbitrary extents applied in the
 * xy direction, periodic (indices wrap) or non-periodic (boundary cells left
 * untouched); premap 1 applies the stencil to c^3 - c instead of c, the role
 * of the function-pointer stencil in the Cahn-Hilliard example. */
static int wrap(int k, int n) { return ((k % n) + n) % n; }
static double mu_of(double v) { return v * v * v - v; }

int orc_stencil2d(const double* in, double* out, int nx, int ny,
                  const double* w, int left, int right, int top, int bottom,
                  int periodic, int premap) {
  if (nx < 1 || ny < 1 || left < 0 || right < 0 || top < 0 || bottom < 0)
    return -1;
  const int wx = left + right + 1;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      if (!periodic && (i - left < 0 || i + right >= nx || j - top < 0 ||
                        j + bottom >= ny))
        continue;
      double acc = 0.0;
      for (int q = -top; q <= bottom; ++q) {
        for (int p = -left; p <= right; ++p) {
          int jj = periodic ? wrap(j + q, ny) : j + q;
          int ii = periodic ? wrap(i + p, nx) : i + p;
          double v = in[(size_t)jj * nx + ii];
          if (premap == 1) v = v * v * v - v;
          acc = acc + w[(q + top) * wx + (p + left)] * v;
        }
      }
      out[(size_t)j * nx + i] = acc;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ch.2 eq. 2:ch, c_t = D Lap(c^3 - c - gamma Lap c), advanced by the
 * first-order semi-implicit ADI scheme whose implicit operator is
 * (I + D gamma dt dxxxx)(I + D gamma dt dyyyy) (the split hyperdiffusion of
 * Ch.3 eq. 3:ch_adi with the 1D scheme of Ch.6 eq. 6:1Dnumerical in each
 * direction).  The mixed part 2 dxx dyy of Lap^2 stays explicit, via the
 * cross stencil of Ch.3 Fig. "stencil" (weights 1,-2,1 / -2,4,-2 / 1,-2,1). */
void orc_ch_rhs(const double* c, double* r, int nx, int ny, double lx,
                double ly, double D, double gamma, double dt) {
  const double dx = lx / nx, dy = ly / ny;
  for (int j = 0; j < ny; ++j) {
    const int jm = wrap(j - 1, ny), jp = wrap(j + 1, ny);
    for (int i = 0; i < nx; ++i) {
      const int im = wrap(i - 1, nx), ip = wrap(i + 1, nx);
      double cc = c[(size_t)j * nx + i];
      double ce = c[(size_t)j * nx + ip], cw = c[(size_t)j * nx + im];
      double cn = c[(size_t)jp * nx + i], cs = c[(size_t)jm * nx + i];
      double mu_c = cc * cc * cc - cc;
      double mu_e = ce * ce * ce - ce, mu_w = cw * cw * cw - cw;
      double mu_n = cn * cn * cn - cn, mu_s = cs * cs * cs - cs;
      double lap = (mu_e + mu_w - 2.0 * mu_c) / (dx * dx) +
                   (mu_n + mu_s - 2.0 * mu_c) / (dy * dy);
      /* d2x d2y c: second difference in x of the second difference in y */
      double cne = c[(size_t)jp * nx + ip], cnw = c[(size_t)jp * nx + im];
      double cse = c[(size_t)jm * nx + ip], csw = c[(size_t)jm * nx + im];
      double dyy_w = cnw + csw - 2.0 * cw;
      double dyy_c = cn + cs - 2.0 * cc;
      double dyy_e = cne + cse - 2.0 * ce;
      double cross = (dyy_e + dyy_w - 2.0 * dyy_c) / (dx * dx * dy * dy);
      r[(size_t)j * nx + i] = cc + D * dt * lap - 2.0 * D * gamma * dt * cross;
    }
  }
}

int orc_ch_step(double* c, int nx, int ny, double lx, double ly, double D,
                double gamma, double dt) {
  if (nx < 5 || ny < 5) return -1;
  const double dx = lx / nx, dy = ly / ny;
  const double sx = D * gamma * dt / (dx * dx * dx * dx);
  const double sy = D * gamma * dt / (dy * dy * dy * dy);
  double* r = (double*)malloc(sizeof(double) * (size_t)nx * ny);
  orc_ch_rhs(c, r, nx, ny, lx, ly, D, gamma, dt);
  int rc = orc_cpenta_lines(nx, ny, 0, sx, -4.0 * sx, 1.0 + 6.0 * sx,
                            -4.0 * sx, sx, r);
  if (rc == 0)
    rc = orc_cpenta_lines(nx, ny, 1, sy, -4.0 * sy, 1.0 + 6.0 * sy, -4.0 * sy,
                          sy, r);
  if (rc == 0) memcpy(c, r, sizeof(double) * (size_t)nx * ny);
  free(r);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Ch.3 eq. 3:ch_adi, the thesis's own scheme, in its order:
 *   L_x w = -2/3 (C^n - C^{n-1}) - 2/3 D gamma dt Lap^2 Cbar + 2/3 D dt Lap (C^3 - C)^n
 *   L_y v = w,   C^{n+1} = Cbar + v,   L = I + 2/3 D gamma dt d4 (per direction)
 * with the readings: Cbar = 2 C^n - C^{n-1} (the extrapolation of the stable
 * hyperdiffusion ADI the thesis builds on), D gamma in the biharmonic term
 * (as in L_x), C^{-1} = C^0 at the start, second-order central differences:
 * Lap = d2x + d2y (5 points), Lap^2 = d4x + 2 d2x d2y + d4y (13 points in the
 * 5 x 5 square), d4 = (1, -4, 6, -4, 1) / h^4. */
void orc_ch2_rhs(const double* c, const double* cprev, double* r, int nx,
                 int ny, double lx, double ly, double D, double gamma,
                 double dt) {
  const double dx = lx / nx, dy = ly / ny;
  const double dx2 = dx * dx, dy2 = dy * dy;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      /* Cbar at offsets (p, q), p along x, q along y */
#define CB(p, q)                                                      \
  (2.0 * c[(size_t)wrap(j + (q), ny) * nx + wrap(i + (p), nx)] -      \
   cprev[(size_t)wrap(j + (q), ny) * nx + wrap(i + (p), nx)])
#define MU(p, q) mu_of(c[(size_t)wrap(j + (q), ny) * nx + wrap(i + (p), nx)])
      double d4x = (CB(-2, 0) - 4.0 * CB(-1, 0) + 6.0 * CB(0, 0) -
                    4.0 * CB(1, 0) + CB(2, 0)) / (dx2 * dx2);
      double d4y = (CB(0, -2) - 4.0 * CB(0, -1) + 6.0 * CB(0, 0) -
                    4.0 * CB(0, 1) + CB(0, 2)) / (dy2 * dy2);
      /* d2x d2y Cbar: second difference in x of the second differences in y */
      double dyy_w = CB(-1, 1) + CB(-1, -1) - 2.0 * CB(-1, 0);
      double dyy_c = CB(0, 1) + CB(0, -1) - 2.0 * CB(0, 0);
      double dyy_e = CB(1, 1) + CB(1, -1) - 2.0 * CB(1, 0);
      double dxxyy = (dyy_e + dyy_w - 2.0 * dyy_c) / (dx2 * dy2);
      double bih = d4x + 2.0 * dxxyy + d4y;
      double lap = (MU(1, 0) + MU(-1, 0) - 2.0 * MU(0, 0)) / dx2 +
                   (MU(0, 1) + MU(0, -1) - 2.0 * MU(0, 0)) / dy2;
#undef CB
#undef MU
      const size_t k = (size_t)j * nx + i;
      r[k] = -(2.0 / 3.0) * (c[k] - cprev[k]) -
             (2.0 / 3.0) * D * gamma * dt * bih + (2.0 / 3.0) * D * dt * lap;
    }
  }
}

int orc_ch2_step(double* c, double* cprev, int nx, int ny, double lx,
                 double ly, double D, double gamma, double dt) {
  if (nx < 5 || ny < 5) return -1;
  const double dx = lx / nx, dy = ly / ny;
  const double sx = (2.0 / 3.0) * D * gamma * dt / (dx * dx * dx * dx);
  const double sy = (2.0 / 3.0) * D * gamma * dt / (dy * dy * dy * dy);
  const size_t n = (size_t)nx * ny;
  double* w = (double*)malloc(sizeof(double) * n);
  orc_ch2_rhs(c, cprev, w, nx, ny, lx, ly, D, gamma, dt);
  /* L_x w = RHS (rows), then L_y v = w (columns), in place */
  int rc = orc_cpenta_lines(nx, ny, 0, sx, -4.0 * sx, 1.0 + 6.0 * sx,
                            -4.0 * sx, sx, w);
  if (rc == 0)
    rc = orc_cpenta_lines(nx, ny, 1, sy, -4.0 * sy, 1.0 + 6.0 * sy, -4.0 * sy,
                          sy, w);
  if (rc == 0) {
    for (size_t k = 0; k < n; ++k) {
      const double cbar = 2.0 * c[k] - cprev[k];
      cprev[k] = c[k];
      c[k] = cbar + w[k];
    }
  }
  free(w);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Batched 1D periodic schemes on (0, L), dx = L/n, x interleaved: unknown i
 * of system s at x[i * batch + s].  Each step forms the right-hand side of
 * the chapter's scheme and solves the cyclic system of that chapter:
 *  kind 0, Ch.4 eq. disc (Crank-Nicolson hyperdiffusion C_t = -a C_xxxx):
 *    s = a dt / (2 dx^4);  (s, -4s, 1+6s, -4s, s) C^{n+1}
 *                          = (-s, 4s, 1-6s, 4s, -s) C^n
 *  kind 1, Ch.5 eq. 5:1ddiffscheme (Crank-Nicolson diffusion C_t = a C_xx):
 *    s = a dt / (2 dx^2);  (-s, 1+2s, -s) C^{n+1} = (s, 1-2s, s) C^n
 *  kind 2, Ch.6 eq. 6:1Dnumerical (1D Cahn-Hilliard, gamma = a):
 *    s = a D dt / dx^4, al = D dt / dx^2, N = C^3 - C;
 *    (s, -4s, 1+6s, -4s, s) C^{n+1} = C^n + al (N_{i-1} - 2 N_i + N_{i+1})
 * (the printed f of Ch.6 omits the C^n of eq. 6:1Dnumerical; it is kept). */
int orc_batch1d_step(int kind, double* x, int n, int batch, double L,
                     double dt, double a, double D) {
  if (kind < 0 || kind > 2 || batch < 1) return -1;
  if (n < (kind == 1 ? 3 : 5)) return -1;
  const double dx = L / n;
  double* f = (double*)malloc(sizeof(double) * (size_t)n);
  double* y = (double*)malloc(sizeof(double) * (size_t)n);
  double s = 0.0, al = 0.0;
  if (kind == 0) s = a * dt / (2.0 * dx * dx * dx * dx);
  if (kind == 1) s = a * dt / (2.0 * dx * dx);
  if (kind == 2) {
    s = a * D * dt / (dx * dx * dx * dx);
    al = D * dt / (dx * dx);
  }
  int rc = 0;
  for (int b = 0; b < batch && rc == 0; ++b) {
#define XV(i) x[(size_t)wrap((i), n) * batch + b]
    for (int i = 0; i < n; ++i) {
      if (kind == 0)
        f[i] = -s * XV(i - 2) + 4.0 * s * XV(i - 1) + (1.0 - 6.0 * s) * XV(i) +
               4.0 * s * XV(i + 1) - s * XV(i + 2);
      else if (kind == 1)
        f[i] = s * XV(i - 1) + (1.0 - 2.0 * s) * XV(i) + s * XV(i + 1);
      else
        f[i] = XV(i) + al * (mu_of(XV(i - 1)) - 2.0 * mu_of(XV(i)) +
                             mu_of(XV(i + 1)));
    }
#undef XV
    if (kind == 1)
      rc = orc_cyclic_tri_solve(n, -s, 1.0 + 2.0 * s, -s, f, y);
    else
      rc = orc_cyclic_penta_solve(n, s, -4.0 * s, 1.0 + 6.0 * s, -4.0 * s, s,
                                  f, y);
    for (int i = 0; i < n; ++i) x[(size_t)i * batch + b] = y[i];
  }
  free(f);
  free(y);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Ch.7, the Cahn-Hilliard-Cook equation: C_t = D Lap(C^3 - C - gamma Lap C)
 * + eta, eta_ij = sqrt(sigma / (dx dy dt)) div rho_ij, rho a 2-vector of
 * N(0,1) numbers per point and step, drawn from two uniforms by the
 * Box-Muller transformation.  Readings: div by forward differences (periodic,
 * so sum(eta) = 0 and the mass is conserved); eta enters the explicit
 * right-hand side as dt * eta.  The uniforms come from a counter-based
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output k of the sequence
 * whose state starts at mix(seed), u = ((out >> 11) + 1/2) 2^-53 in (0, 1),
 * counter k = ((step * ny + j) * nx + i) * 2 + component. */
static uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double orc_sm_uniform(uint64_t seed, uint64_t k) {
  const uint64_t st = sm_mix(seed) + (k + 1) * 0x9E3779B97F4A7C15ULL;
  return ((double)(sm_mix(st) >> 11) + 0.5) * 0x1.0p-53;
}

void orc_cook_rho(double* rx, double* ry, int nx, int ny, uint64_t seed,
                  uint64_t step) {
  const double two_pi = 6.283185307179586476925286766559;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const uint64_t k = ((step * (uint64_t)ny + (uint64_t)j) * (uint64_t)nx +
                          (uint64_t)i) * 2;
      const double u1 = orc_sm_uniform(seed, k), u2 = orc_sm_uniform(seed, k + 1);
      const double rad = sqrt(-2.0 * log(u1));
      rx[(size_t)j * nx + i] = rad * cos(two_pi * u2);
      ry[(size_t)j * nx + i] = rad * sin(two_pi * u2);
    }
  }
}

void orc_cook_increment(double* out, int nx, int ny, double lx, double ly,
                        double dt, double sigma, uint64_t seed, uint64_t step) {
  const double dx = lx / nx, dy = ly / ny;
  double* rx = (double*)malloc(sizeof(double) * (size_t)nx * ny);
  double* ry = (double*)malloc(sizeof(double) * (size_t)nx * ny);
  orc_cook_rho(rx, ry, nx, ny, seed, step);
  const double amp = sqrt(sigma / (dx * dy * dt));
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      const size_t k = (size_t)j * nx + i;
      const double div = (rx[(size_t)j * nx + wrap(i + 1, nx)] - rx[k]) / dx +
                         (ry[(size_t)wrap(j + 1, ny) * nx + i] - ry[k]) / dy;
      out[k] = dt * amp * div;
    }
  }
  free(rx);
  free(ry);
}

int orc_ch_step_cook(double* c, int nx, int ny, double lx, double ly, double D,
                     double gamma, double dt, double sigma, uint64_t seed,
                     uint64_t step) {
  if (nx < 5 || ny < 5) return -1;
  const double dx = lx / nx, dy = ly / ny;
  const double sx = D * gamma * dt / (dx * dx * dx * dx);
  const double sy = D * gamma * dt / (dy * dy * dy * dy);
  const size_t n = (size_t)nx * ny;
  double* r = (double*)malloc(sizeof(double) * n);
  double* q = (double*)malloc(sizeof(double) * n);
  orc_ch_rhs(c, r, nx, ny, lx, ly, D, gamma, dt);
  orc_cook_increment(q, nx, ny, lx, ly, dt, sigma, seed, step);
  for (size_t k = 0; k < n; ++k) r[k] = r[k] + q[k];
  int rc = orc_cpenta_lines(nx, ny, 0, sx, -4.0 * sx, 1.0 + 6.0 * sx,
                            -4.0 * sx, sx, r);
  if (rc == 0)
    rc = orc_cpenta_lines(nx, ny, 1, sy, -4.0 * sy, 1.0 + 6.0 * sy, -4.0 * sy,
                          sy, r);
  if (rc == 0) memcpy(c, r, sizeof(double) * n);
  free(r);
  free(q);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Ch.3 "Numerical Results": s(t) = 1 / (1 - <C^2>), the spatial average by
 * composite Simpson's rule in each direction of the periodic grid (nx, ny
 * even): weight 2/3 on even and 4/3 on odd indices, so that <f> = sum w_i w_j
 * f_ij / (nx ny).  Returns <C^power> (power 1 or 2); Neumaier sum. */
double orc_simpson_mean(const double* c, int nx, int ny, int power) {
  double s = 0.0, comp = 0.0;
  for (int j = 0; j < ny; ++j) {
    const double wj = (j % 2 == 0) ? 2.0 / 3.0 : 4.0 / 3.0;
    for (int i = 0; i < nx; ++i) {
      const double wi = (i % 2 == 0) ? 2.0 / 3.0 : 4.0 / 3.0;
      const double cv = c[(size_t)j * nx + i];
      const double v = wj * wi * (power == 2 ? cv * cv : cv);
      const double t = s + v;
      if (fabs(s) >= fabs(v)) comp = comp + ((s - t) + v);
      else                    comp = comp + ((v - t) + s);
      s = t;
    }
  }
  return (s + comp) / ((double)nx * ny);
}

/* Ch.2: conservation of the integral of C.  Neumaier-compensated sum. */
double orc_ch_mass(const double* c, int nx, int ny, double lx, double ly) {
  double s = 0.0, comp = 0.0;
  for (size_t k = 0; k < (size_t)nx * ny; ++k) {
    double v = c[k], t = s + v;
    if (fabs(s) >= fabs(v)) comp = comp + ((s - t) + v);
    else                    comp = comp + ((v - t) + s);
    s = t;
  }
  return (s + comp) * (lx / nx) * (ly / ny);
}

/* Ch.2 free energy with the bulk term (C^2-1)^2/4, whose derivative is the
 * C^3 - C of the chemical potential, and forward differences for grad C. */
double orc_ch_energy(const double* c, int nx, int ny, double lx, double ly,
                     double gamma) {
  const double dx = lx / nx, dy = ly / ny;
  double s = 0.0, comp = 0.0;
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      double cc = c[(size_t)j * nx + i];
      double gx = (c[(size_t)j * nx + wrap(i + 1, nx)] - cc) / dx;
      double gy = (c[(size_t)wrap(j + 1, ny) * nx + i] - cc) / dy;
      double w = cc * cc - 1.0;
      double v = 0.25 * w * w + 0.5 * gamma * (gx * gx + gy * gy);
      double t = s + v;
      if (fabs(s) >= fabs(v)) comp = comp + ((s - t) + v);
      else                    comp = comp + ((v - t) + s);
      s = t;
    }
  }
  return (s + comp) * dx * dy;
}

/* ------------------------------------------------------------------------ */
/* Ch.7 eq. 7:betaN: the free-energy decay rate beta = -(t / F) dF/dt of a
 * series F_k = F(t0 + k dt), k = 0 .. n-1 (n >= 3).  The thesis does not say
 * how dF/dt is taken from the sampled series; read here as second-order
 * differences: central at interior samples, the three-point one-sided forms
 * at the two ends (each exact for a quadratic F). */
int orc_energy_decay_rate(const double* F, int n, double t0, double dt, double* beta) {
  if (n < 3 || !(dt > 0.0)) return -1;
  for (int k = 0; k < n; ++k) {
    double dFdt;
    if (k == 0)
      dFdt = (-3.0 * F[0] + 4.0 * F[1] - F[2]) / (2.0 * dt);
    else if (k == n - 1)
      dFdt = (3.0 * F[n - 1] - 4.0 * F[n - 2] + F[n - 3]) / (2.0 * dt);
    else
      dFdt = (F[k + 1] - F[k - 1]) / (2.0 * dt);
    const double t = t0 + k * dt;
    beta[k] = -(t / F[k]) * dFdt;
  }
  return 0;
}
