// plan.cpp -- host factorisation tables (see plan.hpp).  Long double
// throughout; the results are rounded once to FP64 and FP32 for the device.
#include "plan.hpp"

#include <algorithm>
#include <cmath>

#include "chx.h"

namespace chx {
namespace {

using LD = long double;

// Entry (i, j) of the non-wrapped band matrix of size n.
LD band_entry(const Band& b, int n, int i, int j) {
  const int o = j - i;
  if (j < 0 || j >= n || i < 0 || i >= n || o < -b.P || o > b.P) return 0;
  return b.coef[o + b.P];
}

// Entry (i, j) of the cyclic matrix of size n: every band offset o whose
// wrapped column (i + o) mod n equals j contributes.
LD cyc_entry(const Band& b, int n, int i, int j) {
  LD v = 0;
  for (int o = -b.P; o <= b.P; ++o)
    if ((((i + o) % n) + n) % n == j) v += b.coef[o + b.P];
  return v;
}

// A = L R with L lower (diagonal alpha, sub-diagonals Lsub) and R unit upper
// (super-diagonals Rsup): the LR factorisation of Ch.4 "Solution of the
// pentadiagonal system" (alpha, beta, epsilon in L; gamma, delta in R) for
// any half bandwidth, and the Thomas pre-factorisation of Ch.5 for P = 1
// (alpha_i = b_i - a_i chat_{i-1}, chat in R).
struct LR {
  int n = 0, P = 0;
  std::vector<LD> alpha, Lsub, Rsup;  // Lsub[i*P + r-1] = L(i,i-r); Rsup[i*P + r-1] = R(i,i+r)
  LD Lg(int i, int j) const {
    const int r = i - j;
    return (r >= 1 && r <= P && j >= 0) ? Lsub[(size_t)i * P + r - 1] : 0;
  }
  LD Rg(int i, int j) const {
    const int r = j - i;
    return (r >= 1 && r <= P && j < n) ? Rsup[(size_t)i * P + r - 1] : 0;
  }
};

int lr_factor(const Band& b, int n, LR* f) {
  const int P = b.P;
  f->n = n;
  f->P = P;
  f->alpha.assign(n, 0);
  f->Lsub.assign((size_t)n * P, 0);
  f->Rsup.assign((size_t)n * P, 0);
  for (int i = 0; i < n; ++i) {
    for (int r = P; r >= 1; --r) {
      const int j = i - r;
      if (j < 0) continue;
      LD v = band_entry(b, n, i, j);
      for (int t = std::max(0, i - P); t < j; ++t) v -= f->Lg(i, t) * f->Rg(t, j);
      f->Lsub[(size_t)i * P + r - 1] = v;
    }
    LD al = band_entry(b, n, i, i);
    for (int t = std::max(0, i - P); t < i; ++t) al -= f->Lg(i, t) * f->Rg(t, i);
    if (!(al > 0) || !std::isfinite((double)al)) return CHX_EPIVOT;
    f->alpha[i] = al;
    for (int r = 1; r <= P; ++r) {
      const int j = i + r;
      if (j >= n) continue;
      LD v = band_entry(b, n, i, j);
      for (int t = std::max(0, j - P); t < i; ++t) v -= f->Lg(i, t) * f->Rg(t, j);
      f->Rsup[(size_t)i * P + r - 1] = v / al;
    }
  }
  return CHX_OK;
}

// x = E^{-1} f  (forward L g = f, back R x = g)
std::vector<LD> lr_solve(const LR& f, const std::vector<LD>& rhs) {
  const int n = f.n, P = f.P;
  std::vector<LD> g(n), x(n);
  for (int i = 0; i < n; ++i) {
    LD v = rhs[i];
    for (int r = 1; r <= P && i - r >= 0; ++r) v -= f.Lg(i, i - r) * g[i - r];
    g[i] = v / f.alpha[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    LD v = g[i];
    for (int r = 1; r <= P && i + r < n; ++r) v -= f.Rg(i, i + r) * x[i + r];
    x[i] = v;
  }
  return x;
}

// q = E^{-T} h  (E^T = R^T L^T: forward with R^T, back with L^T)
std::vector<LD> lr_solve_transposed(const LR& f, const std::vector<LD>& rhs) {
  const int n = f.n, P = f.P;
  std::vector<LD> w(n), q(n);
  for (int i = 0; i < n; ++i) {
    LD v = rhs[i];
    for (int r = 1; r <= P && i - r >= 0; ++r) v -= f.Rg(i - r, i) * w[i - r];
    w[i] = v;
  }
  for (int i = n - 1; i >= 0; --i) {
    LD v = w[i];
    for (int r = 1; r <= P && i + r < n; ++r) v -= f.Lg(i + r, i) * q[i + r];
    q[i] = v / f.alpha[i];
  }
  return q;
}

bool invert_small(const LD* m, int P, LD* inv) {
  if (P == 1) {
    if (!(m[0] != 0)) return false;
    inv[0] = 1 / m[0];
    return std::isfinite((double)inv[0]);
  }
  const LD det = m[0] * m[3] - m[1] * m[2];
  if (!(det != 0) || !std::isfinite((double)det)) return false;
  inv[0] = m[3] / det;
  inv[1] = -m[1] / det;
  inv[2] = -m[2] / det;
  inv[3] = m[0] / det;
  return true;
}

// Bordering of the last P unknowns of the cyclic system (Navon, Ch.4):
// E (leading block), k, h^T, C22 read off the periodic pattern.
struct Bordered {
  LR E;
  std::vector<std::vector<LD>> Z, q;  // Z[a] = E^{-1} k[:,a], q[a] = E^{-T} h[a,:]
  LD minv[4] = {1, 0, 0, 1};
};

int bordered_factor(const Band& b, int n, Bordered* out) {
  const int P = b.P, mi = n - P;
  Band eb = b;
  int rc = lr_factor(eb, mi, &out->E);
  if (rc) return rc;
  out->Z.assign(P, std::vector<LD>(mi));
  out->q.assign(P, std::vector<LD>(mi));
  for (int a = 0; a < P; ++a) {
    std::vector<LD> kcol(mi), hrow(mi);
    for (int i = 0; i < mi; ++i) {
      kcol[i] = cyc_entry(b, n, i, mi + a);
      hrow[i] = cyc_entry(b, n, mi + a, i);
    }
    out->Z[a] = lr_solve(out->E, kcol);
    out->q[a] = lr_solve_transposed(out->E, hrow);
  }
  LD M[4] = {0, 0, 0, 0};
  for (int a = 0; a < P; ++a)
    for (int c = 0; c < P; ++c) {
      LD v = cyc_entry(b, n, mi + a, mi + c);
      std::vector<LD> hrow(mi);
      for (int i = 0; i < mi; ++i) v -= cyc_entry(b, n, mi + a, i) * out->Z[c][i];
      M[a * P + c] = v;
    }
  LD inv[4];
  if (!invert_small(M, P, inv)) return CHX_EPIVOT;
  for (int t = 0; t < P * P; ++t) out->minv[t] = inv[t];
  return CHX_OK;
}

std::vector<LD> bordered_solve(const Band& b, int n, const Bordered& B,
                               const std::vector<LD>& f) {
  const int P = b.P, mi = n - P;
  std::vector<LD> fh(f.begin(), f.begin() + mi);
  LD r[2] = {0, 0}, t[2] = {0, 0};
  for (int a = 0; a < P; ++a) {
    LD s = 0;
    for (int i = 0; i < mi; ++i) s += B.q[a][i] * fh[i];
    r[a] = f[mi + a] - s;
  }
  for (int a = 0; a < P; ++a)
    for (int c = 0; c < P; ++c) t[a] += B.minv[a * P + c] * r[c];
  std::vector<LD> y = lr_solve(B.E, fh);
  std::vector<LD> x(n);
  for (int i = 0; i < mi; ++i) {
    LD v = y[i];
    for (int a = 0; a < P; ++a) v -= B.Z[a][i] * t[a];
    x[i] = v;
  }
  for (int a = 0; a < P; ++a) x[mi + a] = t[a];
  return x;
}

void fill_rec(const LR& E, int i, double* rec) {
  rec[0] = (double)(1.0L / E.alpha[i]);
  rec[1] = (double)E.Lg(i, i - 1);
  rec[2] = (double)E.Rg(i, i + 1);
  rec[3] = (E.P >= 2) ? (double)E.Rg(i, i + 2) : 0.0;
}

}  // namespace

int circulant_inverse_column(const Band& band, int n, std::vector<long double>* g) {
  Bordered B;
  int rc = bordered_factor(band, n, &B);
  if (rc) return rc;
  std::vector<LD> e0(n, 0);
  e0[0] = 1;
  *g = bordered_solve(band, n, B, e0);
  return CHX_OK;
}

int build_whole(const Band& band, int n, WholeTables* out) {
  const int P = band.P;
  out->n = n;
  out->P = P;
  if (!band.periodic) {
    LR E;
    int rc = lr_factor(band, n, &E);
    if (rc) return rc;
    out->mi = n;
    out->rec.assign((size_t)n * kRec, 0.0);
    for (int i = 0; i < n; ++i) fill_rec(E, i, &out->rec[(size_t)i * kRec]);
  } else {
    Bordered B;
    int rc = bordered_factor(band, n, &B);
    if (rc) return rc;
    const int mi = n - P;
    out->mi = mi;
    out->rec.assign((size_t)mi * kRec, 0.0);
    for (int i = 0; i < mi; ++i) {
      double* r = &out->rec[(size_t)i * kRec];
      fill_rec(B.E, i, r);
      for (int a = 0; a < P; ++a) {
        r[4 + a] = (double)B.q[a][i];
        r[6 + a] = (double)B.Z[a][i];
      }
    }
    for (int t = 0; t < 4; ++t) out->minv[t] = 0.0;
    for (int a = 0; a < P; ++a)
      for (int c = 0; c < P; ++c) out->minv[a * 2 + c] = (double)B.minv[a * P + c];
  }
  out->rec32.assign(out->rec.begin(), out->rec.end());
  for (int t = 0; t < 4; ++t) out->minv32[t] = (float)out->minv[t];
  return CHX_OK;
}

int build_chunk(const Band& band, int n, int m, ChunkTables* out) {
  const int P = band.P;
  if (!band.periodic || m < 3 * P || n % m != 0) return CHX_EINVAL;
  const int S = n / m, mi = m - P;
  out->n = n; out->P = P; out->m = m; out->S = S; out->mi = mi;

  // Interior block of one chunk and its spike vectors.
  LR E;
  int rc = lr_factor(band, mi, &E);
  if (rc) return rc;
  out->rec.assign((size_t)mi * kRec, 0.0);
  for (int a = 0; a < P; ++a) {
    std::vector<LD> kl(mi, 0), kr(mi, 0);
    for (int p = 0; p < mi; ++p) {
      const int ol = (a - P) - p;   // previous chunk's separator a sits at -P + a
      if (ol >= -P && ol <= P) kl[p] = band.coef[ol + P];
      const int orr = mi + a - p;   // this chunk's separator a sits at mi + a
      if (orr >= -P && orr <= P) kr[p] = band.coef[orr + P];
    }
    std::vector<LD> zl = lr_solve(E, kl), zr = lr_solve(E, kr);
    for (int p = 0; p < mi; ++p) {
      out->rec[(size_t)p * kRec + 4 + a] = (double)zl[p];
      out->rec[(size_t)p * kRec + 6 + a] = (double)zr[p];
    }
  }
  for (int p = 0; p < mi; ++p) fill_rec(E, p, &out->rec[(size_t)p * kRec]);

  // Reduced system: the separator-separator block of the circulant A^{-1}.
  std::vector<LD> g;
  rc = circulant_inverse_column(band, n, &g);
  if (rc) return rc;
  auto blk = [&](int d, int a, int c) -> LD {
    long long idx = (long long)(-(long long)d * m + a - c);
    idx %= n;
    if (idx < 0) idx += n;
    return g[(size_t)idx];
  };
  std::vector<LD> nb(S, 0);
  for (int d = 0; d < S; ++d)
    for (int a = 0; a < P; ++a)
      for (int c = 0; c < P; ++c) nb[d] = std::max(nb[d], std::fabs(blk(d, a, c)));
  const LD thresh = std::ldexp((LD)1, -60) * nb[0];
  int W = 0;
  for (;; ++W) {
    LD tail = 0;
    for (int d = 0; d < S; ++d) {
      const int dist = std::min(d, S - d);
      if (dist > W) tail += nb[d];
    }
    if (tail <= thresh || 2 * W + 1 >= S) break;
  }
  if (2 * W + 1 >= S) {
    out->dlo = -((S - 1) / 2);
    out->dcount = S;
  } else {
    out->dlo = -W;
    out->dcount = 2 * W + 1;
  }
  out->max_dropped = 0.0;
  for (int d = 0; d < S; ++d) {
    const int dist = std::min(d, S - d);
    if (out->dcount < S && dist > W) out->max_dropped = std::max(out->max_dropped, (double)nb[d]);
  }
  out->blocks.assign((size_t)out->dcount * 4, 0.0);
  for (int t = 0; t < out->dcount; ++t) {
    const int d = out->dlo + t;
    for (int a = 0; a < P; ++a)
      for (int c = 0; c < P; ++c) out->blocks[(size_t)t * 4 + a * 2 + c] = (double)blk(d, a, c);
  }
  out->rec32.assign(out->rec.begin(), out->rec.end());
  out->blocks32.assign(out->blocks.begin(), out->blocks.end());
  return CHX_OK;
}

}  // namespace chx
