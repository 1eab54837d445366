// varband.hip -- batched banded solves with one matrix per system.
//
// The thesis's cuPentBatch (Ch.4, "Implementation on GPU") solves a batch of
// pentadiagonal systems, each with its own five diagonals, one thread per
// system on interleaved data (entry i of every system contiguous), with the
// factorisation split from the solve so that a constant matrix is factored
// once; its "Rewrite" variant factors again at every step for matrices that
// change (Ch.4, "Performance Analysis").  Ch.5 does the same for tridiagonal
// systems (Thomas with pre-factorisation).  Here:
//
//  - factor / solve: the factors overwrite the diagonals in place (as in the
//    thesis): b <- beta, c <- 1/alpha, d <- gamma, e <- delta, with a kept as
//    epsilon; tridiagonal: b <- 1/den, c <- chat.
//  - rewrite: factor and solve in one kernel that leaves the diagonals alone
//    and keeps the back sweep's coefficients in the workspace.
//  - periodic systems: the last two unknowns are bordered off (Ch.4, Navon)
//    or the corners split off as a rank-one term (Ch.5, Sherman-Morrison),
//    both built from each system's own rows.  The correction that the thesis
//    writes with E^{-1} (h^T E^{-1} f, h^T E^{-1} k, or v.y and v.z) is
//    formed during the forward sweep: with E = L R,
//    h^T E^{-1} f = (R^{-T} h) . (L^{-1} f), and R^{-T} h is itself a forward
//    recurrence in the factors already computed.  So every solve is one
//    forward and one backward pass over the data, periodic or not.
//
// Each thread walks its system serially; rows are staged U at a time in
// registers so that U rows of loads are in flight before the recurrence
// consumes them.  Every access of a wave covers 64 consecutive systems of
// one row: 512 contiguous bytes.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "chx.h"
#include "launch.hpp"

namespace chx_vb {

constexpr int kThreads = 256;
#ifndef CHX_VB_U
#define CHX_VB_U 8
#endif
constexpr int kU = CHX_VB_U;  // rows staged per batch of loads
// The staged loads are non-temporal: every value is used once per pass
// (measured at n = 1024, 65536 systems: factored solves 2-7 % faster,
// rewrites 2-3 %).
// The solve kernels stage fewer rows: with one system per thread the batch
// gives one wave per SIMD, and at 65536 systems x 1024 both factored solves
// ran fastest at 6 (penta 1.46 ms against 1.84 ms at 8; tri 0.89 against
// 1.07), while the fused factor-and-solve kernels were best at 8.
constexpr int kUS = 6;

// ---------------------------------------------------------------------------
// Pentadiagonal.  Row i: a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} +
// e_i x_{i+2}.  Periodic: indices mod n; the leading block E is rows and
// columns 0..m-1 (m = n - 2), k the columns n-2, n-1 of those rows, h the rows
// n-2, n-1 restricted to columns 0..m-1, C22 their 2 x 2 corner.
// ---------------------------------------------------------------------------

// Forward-sweep state of one system.
struct PentaFwd {
  double gm1 = 0, gm2 = 0;  // gamma_{i-1}, gamma_{i-2}
  double dm1 = 0, dm2 = 0;  // delta_{i-1}, delta_{i-2}
  double g1 = 0, g2 = 0;    // g_{i-1}, g_{i-2}
  double p1 = 0, p2 = 0;    // (L^{-1} k0)_{i-1}, _{i-2}
  double q1 = 0, q2 = 0;    // (L^{-1} k1)_{i-1}, _{i-2}
  double u1 = 0, u2 = 0;    // (R^{-T} h0)_{i-1}, _{i-2}
  double v1 = 0, v2 = 0;    // (R^{-T} h1)_{i-1}, _{i-2}
  double s0 = 0, s1 = 0;    // h^T E^{-1} f
  double m00 = 0, m01 = 0, m10 = 0, m11 = 0;  // h^T E^{-1} k
};

// The rows n-2 and n-1 of a periodic system: their entries in h and C22.
struct PentaTail {
  double h0_0, h0_m2, h0_m1;  // row n-2: e (col 0), a (col m-2), b (col m-1)
  double h1_0, h1_1, h1_m1;   // row n-1: d (col 0), e (col 1), a (col m-1)
  double c00, c01, c10, c11;  // C22
  double f0, f1;              // right-hand side of the two rows
};

template <bool PER, bool RHS>
__device__ __forceinline__ void penta_load_tail(int n, long ld, long s, const double* a,
                                                const double* b, const double* c,
                                                const double* d, const double* e,
                                                const double* f, PentaTail& t) {
  const long r0 = (long)(n - 2) * ld + s, r1 = (long)(n - 1) * ld + s;
  t.h0_0 = e[r0];
  t.h0_m2 = a[r0];
  t.h0_m1 = b[r0];
  t.h1_0 = d[r1];
  t.h1_1 = e[r1];
  t.h1_m1 = a[r1];
  t.c00 = c[r0];
  t.c01 = d[r0];
  t.c10 = b[r1];
  t.c11 = c[r1];
  t.f0 = RHS ? f[r0] : 0.0;
  t.f1 = RHS ? f[r1] : 0.0;
}

// One row of the factorisation (and, with RHS, of L g = f) of row i of E.
// ra..re are row i's raw coefficients; the band of E keeps a_i (i >= 2),
// b_i (i >= 1), d_i (i <= m-2), e_i (i <= m-3); the entries that wrap past
// column m-1 form k.  Returns gamma_i, delta_i, 1/alpha_i, beta_i and the
// forward values through the state.
template <bool PER, bool RHS>
__device__ __forceinline__ void penta_fwd_row(int i, int m, double ra, double rb, double rc,
                                              double rd, double re, double rf,
                                              const PentaTail& tl, PentaFwd& st,
                                              double& beta, double& inv, double& gam,
                                              double& del, double& g, double& pk0,
                                              double& pk1, double& wh0, double& wh1) {
  const double ai = (i >= 2) ? ra : 0.0;
  const double bi = (i >= 1) ? rb : 0.0;
  const double di = (i <= m - 2) ? rd : 0.0;
  const double ei = (i <= m - 3) ? re : 0.0;
  beta = bi - ai * st.gm2;
  const double alpha = rc - ai * st.dm2 - beta * st.gm1;
  inv = 1.0 / alpha;
  gam = (di - beta * st.dm1) * inv;
  del = ei * inv;
  g = RHS ? (rf - ai * st.g2 - beta * st.g1) * inv : 0.0;
  pk0 = pk1 = wh0 = wh1 = 0.0;
  if (PER) {
    // columns n-2 and n-1 of row i (k), rows n-2 and n-1 at column i (h)
    double k0 = 0.0, k1 = 0.0, h0 = 0.0, h1 = 0.0;
    if (i == 0) {
      k0 = ra;
      k1 = rb;
      h0 = tl.h0_0;
      h1 = tl.h1_0;
    }
    if (i == 1) {
      k1 = ra;
      h1 = tl.h1_1;
    }
    if (i == m - 2) {
      k0 = k0 + re;
      h0 = h0 + tl.h0_m2;
    }
    if (i == m - 1) {
      k0 = k0 + rd;
      k1 = k1 + re;
      h0 = h0 + tl.h0_m1;
      h1 = h1 + tl.h1_m1;
    }
    pk0 = (k0 - ai * st.p2 - beta * st.p1) * inv;
    pk1 = (k1 - ai * st.q2 - beta * st.q1) * inv;
    // R^T w = h: R is unit upper triangular with gamma above the diagonal
    // and delta two above
    wh0 = h0 - st.gm1 * st.u1 - st.dm2 * st.u2;
    wh1 = h1 - st.gm1 * st.v1 - st.dm2 * st.v2;
    if (RHS) {
      st.s0 = st.s0 + wh0 * g;
      st.s1 = st.s1 + wh1 * g;
    }
    st.m00 = st.m00 + wh0 * pk0;
    st.m01 = st.m01 + wh0 * pk1;
    st.m10 = st.m10 + wh1 * pk0;
    st.m11 = st.m11 + wh1 * pk1;
    st.p2 = st.p1;
    st.p1 = pk0;
    st.q2 = st.q1;
    st.q1 = pk1;
    st.u2 = st.u1;
    st.u1 = wh0;
    st.v2 = st.v1;
    st.v1 = wh1;
  }
  st.gm2 = st.gm1;
  st.gm1 = gam;
  st.dm2 = st.dm1;
  st.dm1 = del;
  st.g2 = st.g1;
  st.g1 = g;
}

// 2 x 2 inverse of C22 - h^T E^{-1} k.
__device__ __forceinline__ void penta_minv(const PentaTail& tl, const PentaFwd& st,
                                           double (&mi)[4]) {
  const double m00 = tl.c00 - st.m00, m01 = tl.c01 - st.m01;
  const double m10 = tl.c10 - st.m10, m11 = tl.c11 - st.m11;
  const double det = m00 * m11 - m01 * m10;
  const double id = 1.0 / det;
  mi[0] = m11 * id;
  mi[1] = -m01 * id;
  mi[2] = -m10 * id;
  mi[3] = m00 * id;
}

// Back sweep R x = g - (L^{-1}k) t over rows m-1..0; x holds g on entry.
template <int U, bool PER>
__device__ __forceinline__ void penta_back(int m, long s, const double* __restrict__ gam,
                                           long ldg, const double* __restrict__ del, long ldd,
                                           const double* __restrict__ pk0,
                                           const double* __restrict__ pk1, long ldw, double t0,
                                           double t1, double* __restrict__ x, long ld) {
  double x1 = 0.0, x2 = 0.0;
  int i = m - 1;
  for (; i + 1 >= U; i -= U) {
    double vg[U], vga[U], vde[U], vp[U], vq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long r = i - u;
      vg[u] = __builtin_nontemporal_load(&x[r * ld + s]);
      vga[u] = __builtin_nontemporal_load(&gam[r * ldg + s]);
      vde[u] = __builtin_nontemporal_load(&del[r * ldd + s]);
      if (PER) {
        vp[u] = __builtin_nontemporal_load(&pk0[r * ldw + s]);
        vq[u] = __builtin_nontemporal_load(&pk1[r * ldw + s]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double v = vg[u];
      if (PER) v = v - vp[u] * t0 - vq[u] * t1;
      v = v - vga[u] * x1 - vde[u] * x2;
      x[(long)(i - u) * ld + s] = v;
      x2 = x1;
      x1 = v;
    }
  }
  for (; i >= 0; --i) {
    double v = x[(long)i * ld + s];
    if (PER) v = v - pk0[(long)i * ldw + s] * t0 - pk1[(long)i * ldw + s] * t1;
    v = v - gam[(long)i * ldg + s] * x1 - del[(long)i * ldd + s] * x2;
    x[(long)i * ld + s] = v;
    x2 = x1;
    x1 = v;
  }
}

// Workspace vectors of a periodic penta batch: rows 0..m-1, stride ldw.
//   factor/solve: [w0 | w1 | pk0 | pk1] then Minv (4 x ldw)
//   rewrite:      [gamma | delta | pk0 | pk1]        (non-periodic: the first two)

template <bool PER>
__global__ __launch_bounds__(kThreads) void penta_batch_factor_k(
    int n, int batch, long ld, double* __restrict__ a, double* __restrict__ b,
    double* __restrict__ c, double* __restrict__ d, double* __restrict__ e,
    double* __restrict__ ws, long ldw) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const int m = PER ? n - 2 : n;
  PentaTail tl{};
  if (PER) penta_load_tail<PER, false>(n, ld, s, a, b, c, d, e, nullptr, tl);
  double* w0 = PER ? ws : nullptr;
  double* w1 = PER ? ws + (long)m * ldw : nullptr;
  double* p0 = PER ? ws + 2L * m * ldw : nullptr;
  double* p1 = PER ? ws + 3L * m * ldw : nullptr;
  PentaFwd st;
  int i = 0;
  for (; i + kU <= m; i += kU) {
    double va[kU], vb[kU], vc[kU], vd[kU], ve[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long r = (long)(i + u) * ld + s;
      va[u] = __builtin_nontemporal_load(&a[r]);
      vb[u] = __builtin_nontemporal_load(&b[r]);
      vc[u] = __builtin_nontemporal_load(&c[r]);
      vd[u] = __builtin_nontemporal_load(&d[r]);
      ve[u] = __builtin_nontemporal_load(&e[r]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      double beta, inv, gam, del, g, pk0, pk1, wh0, wh1;
      penta_fwd_row<PER, false>(i + u, m, va[u], vb[u], vc[u], vd[u], ve[u], 0.0, tl, st, beta,
                                inv, gam, del, g, pk0, pk1, wh0, wh1);
      const long r = (long)(i + u) * ld + s;
      b[r] = beta;
      c[r] = inv;
      d[r] = gam;
      e[r] = del;
      if (PER) {
        const long rw = (long)(i + u) * ldw + s;
        w0[rw] = wh0;
        w1[rw] = wh1;
        p0[rw] = pk0;
        p1[rw] = pk1;
      }
    }
  }
  for (; i < m; ++i) {
    const long r = (long)i * ld + s;
    double beta, inv, gam, del, g, pk0, pk1, wh0, wh1;
    penta_fwd_row<PER, false>(i, m, a[r], b[r], c[r], d[r], e[r], 0.0, tl, st, beta, inv, gam,
                              del, g, pk0, pk1, wh0, wh1);
    b[r] = beta;
    c[r] = inv;
    d[r] = gam;
    e[r] = del;
    if (PER) {
      const long rw = (long)i * ldw + s;
      w0[rw] = wh0;
      w1[rw] = wh1;
      p0[rw] = pk0;
      p1[rw] = pk1;
    }
  }
  if (PER) {
    double mi[4];
    penta_minv(tl, st, mi);
    double* mv = ws + 4L * m * ldw;
#pragma unroll
    for (int q = 0; q < 4; ++q) mv[(long)q * ldw + s] = mi[q];
  }
}

template <bool PER>
__global__ __launch_bounds__(kThreads) void penta_batch_solve_k(
    int n, int batch, long ld, const double* __restrict__ a, const double* __restrict__ b,
    const double* __restrict__ c, const double* __restrict__ d, const double* __restrict__ e,
    const double* __restrict__ ws, long ldw, double* __restrict__ x) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const int m = PER ? n - 2 : n;
  const double* w0 = PER ? ws : nullptr;
  const double* w1 = PER ? ws + (long)m * ldw : nullptr;
  double g1 = 0.0, g2 = 0.0, s0 = 0.0, s1 = 0.0;
  int i = 0;
  for (; i + kUS <= m; i += kUS) {
    double va[kUS], vb[kUS], vc[kUS], vf[kUS], vw0[kUS], vw1[kUS];
#pragma unroll
    for (int u = 0; u < kUS; ++u) {
      const long r = (long)(i + u) * ld + s;
      va[u] = __builtin_nontemporal_load(&a[r]);
      vb[u] = __builtin_nontemporal_load(&b[r]);
      vc[u] = __builtin_nontemporal_load(&c[r]);
      vf[u] = __builtin_nontemporal_load(&x[r]);
      if (PER) {
        vw0[u] = __builtin_nontemporal_load(&w0[(long)(i + u) * ldw + s]);
        vw1[u] = __builtin_nontemporal_load(&w1[(long)(i + u) * ldw + s]);
      }
    }
#pragma unroll
    for (int u = 0; u < kUS; ++u) {
      const double eps = (i + u >= 2) ? va[u] : 0.0;
      const double g = (vf[u] - eps * g2 - vb[u] * g1) * vc[u];
      x[(long)(i + u) * ld + s] = g;
      if (PER) {
        s0 = s0 + vw0[u] * g;
        s1 = s1 + vw1[u] * g;
      }
      g2 = g1;
      g1 = g;
    }
  }
  for (; i < m; ++i) {
    const long r = (long)i * ld + s;
    const double eps = (i >= 2) ? a[r] : 0.0;
    const double g = (x[r] - eps * g2 - b[r] * g1) * c[r];
    x[r] = g;
    if (PER) {
      s0 = s0 + w0[(long)i * ldw + s] * g;
      s1 = s1 + w1[(long)i * ldw + s] * g;
    }
    g2 = g1;
    g1 = g;
  }
  double t0 = 0.0, t1 = 0.0;
  if (PER) {
    const double* mv = ws + 4L * m * ldw;
    const double r0 = x[(long)(n - 2) * ld + s] - s0;
    const double r1 = x[(long)(n - 1) * ld + s] - s1;
    t0 = mv[s] * r0 + mv[ldw + s] * r1;
    t1 = mv[2 * ldw + s] * r0 + mv[3 * ldw + s] * r1;
  }
  penta_back<kUS, PER>(m, s, d, ld, e, ld, PER ? ws + 2L * m * ldw : nullptr,
                  PER ? ws + 3L * m * ldw : nullptr, ldw, t0, t1, x, ld);
  if (PER) {
    x[(long)(n - 2) * ld + s] = t0;
    x[(long)(n - 1) * ld + s] = t1;
  }
}

template <bool PER>
__global__ __launch_bounds__(kThreads) void penta_batch_rewrite_k(
    int n, int batch, long ld, const double* __restrict__ a, const double* __restrict__ b,
    const double* __restrict__ c, const double* __restrict__ d, const double* __restrict__ e,
    double* __restrict__ x, double* __restrict__ ws, long ldw) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const int m = PER ? n - 2 : n;
  PentaTail tl{};
  if (PER) penta_load_tail<PER, true>(n, ld, s, a, b, c, d, e, x, tl);
  double* gm = ws;
  double* dl = ws + (long)m * ldw;
  double* p0 = PER ? ws + 2L * m * ldw : nullptr;
  double* p1 = PER ? ws + 3L * m * ldw : nullptr;
  PentaFwd st;
  int i = 0;
  for (; i + kU <= m; i += kU) {
    double va[kU], vb[kU], vc[kU], vd[kU], ve[kU], vf[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long r = (long)(i + u) * ld + s;
      va[u] = __builtin_nontemporal_load(&a[r]);
      vb[u] = __builtin_nontemporal_load(&b[r]);
      vc[u] = __builtin_nontemporal_load(&c[r]);
      vd[u] = __builtin_nontemporal_load(&d[r]);
      ve[u] = __builtin_nontemporal_load(&e[r]);
      vf[u] = __builtin_nontemporal_load(&x[r]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      double beta, inv, gam, del, g, pk0, pk1, wh0, wh1;
      penta_fwd_row<PER, true>(i + u, m, va[u], vb[u], vc[u], vd[u], ve[u], vf[u], tl, st, beta,
                               inv, gam, del, g, pk0, pk1, wh0, wh1);
      const long rw = (long)(i + u) * ldw + s;
      x[(long)(i + u) * ld + s] = g;
      gm[rw] = gam;
      dl[rw] = del;
      if (PER) {
        p0[rw] = pk0;
        p1[rw] = pk1;
      }
    }
  }
  for (; i < m; ++i) {
    const long r = (long)i * ld + s;
    double beta, inv, gam, del, g, pk0, pk1, wh0, wh1;
    penta_fwd_row<PER, true>(i, m, a[r], b[r], c[r], d[r], e[r], x[r], tl, st, beta, inv, gam,
                             del, g, pk0, pk1, wh0, wh1);
    const long rw = (long)i * ldw + s;
    x[r] = g;
    gm[rw] = gam;
    dl[rw] = del;
    if (PER) {
      p0[rw] = pk0;
      p1[rw] = pk1;
    }
  }
  double t0 = 0.0, t1 = 0.0;
  if (PER) {
    double mi[4];
    penta_minv(tl, st, mi);
    const double r0 = tl.f0 - st.s0, r1 = tl.f1 - st.s1;
    t0 = mi[0] * r0 + mi[1] * r1;
    t1 = mi[2] * r0 + mi[3] * r1;
  }
  penta_back<kU, PER>(m, s, gm, ldw, dl, ldw, p0, p1, ldw, t0, t1, x, ld);
  if (PER) {
    x[(long)(n - 2) * ld + s] = t0;
    x[(long)(n - 1) * ld + s] = t1;
  }
}

// ---------------------------------------------------------------------------
// Tridiagonal.  Row i: a_i x_{i-1} + b_i x_i + c_i x_{i+1}.  Periodic: A =
// A' + u v^T with u = (-b_0, 0, .., 0, c_{n-1}), v = (1, 0, .., 0, -a_0/b_0);
// A' drops the corners and has 2 b_0 and b_{n-1} + a_0 c_{n-1} / b_0 on its
// diagonal ends (Ch.5).  A' = L R with den on L's diagonal, a below it, and
// chat above R's unit diagonal; x = R^{-1}(L^{-1} f - phi L^{-1} u) with
// phi = (w . L^{-1} f) / (1 + w . L^{-1} u), w = R^{-T} v.
// Workspace: factor/solve [zu | w] then 1/(1 + v.z); rewrite [chat | zu].
// ---------------------------------------------------------------------------

struct TriFwd {
  double ch1 = 0;  // chat_{i-1}
  double y1 = 0;   // (L^{-1} f)_{i-1}
  double z1 = 0;   // (L^{-1} u)_{i-1}
  double w1 = 0;   // (R^{-T} v)_{i-1}
  double sy = 0, sz = 0;
};

template <bool PER, bool RHS>
__device__ __forceinline__ void tri_fwd_row(int i, int n, double ra, double rb, double rc,
                                            double rf, double a0, double b0, double cl,
                                            TriFwd& st, double& inv, double& ch, double& y,
                                            double& z, double& w) {
  const double ai = (i >= 1) ? ra : 0.0;
  double bi = rb;
  if (PER && i == 0) bi = 2.0 * b0;
  if (PER && i == n - 1) bi = rb + a0 * cl / b0;
  const double den = bi - ai * st.ch1;
  inv = 1.0 / den;
  ch = (i <= n - 2) ? rc * inv : 0.0;
  y = RHS ? (rf - ai * st.y1) * inv : 0.0;
  z = w = 0.0;
  if (PER) {
    const double ui = (i == 0) ? -b0 : ((i == n - 1) ? cl : 0.0);
    const double vi = (i == 0) ? 1.0 : ((i == n - 1) ? -a0 / b0 : 0.0);
    z = (ui - ai * st.z1) * inv;
    w = vi - st.ch1 * st.w1;
    if (RHS) st.sy = st.sy + w * y;
    st.sz = st.sz + w * z;
    st.z1 = z;
    st.w1 = w;
  }
  st.ch1 = ch;
  st.y1 = y;
}

// x_i = (y_i - phi z_i) - chat_i x_{i+1}, rows n-1..0; x holds y on entry.
template <int U, bool PER>
__device__ __forceinline__ void tri_back(int n, long s, const double* __restrict__ ch, long ldc,
                                         const double* __restrict__ zu, long ldw, double phi,
                                         double* __restrict__ x, long ld) {
  double x1 = 0.0;
  int i = n - 1;
  for (; i + 1 >= U; i -= U) {
    double vy[U], vc[U], vz[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long r = i - u;
      vy[u] = __builtin_nontemporal_load(&x[r * ld + s]);
      vc[u] = __builtin_nontemporal_load(&ch[r * ldc + s]);
      if (PER) vz[u] = __builtin_nontemporal_load(&zu[r * ldw + s]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double v = vy[u];
      if (PER) v = v - phi * vz[u];
      v = v - vc[u] * x1;
      x[(long)(i - u) * ld + s] = v;
      x1 = v;
    }
  }
  for (; i >= 0; --i) {
    double v = x[(long)i * ld + s];
    if (PER) v = v - phi * zu[(long)i * ldw + s];
    v = v - ch[(long)i * ldc + s] * x1;
    x[(long)i * ld + s] = v;
    x1 = v;
  }
}

template <bool PER>
__global__ __launch_bounds__(kThreads) void tri_batch_factor_k(int n, int batch, long ld,
                                                               double* __restrict__ a,
                                                               double* __restrict__ b,
                                                               double* __restrict__ c,
                                                               double* __restrict__ ws,
                                                               long ldw) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const double a0 = PER ? a[s] : 0.0, b0 = PER ? b[s] : 0.0;
  const double cl = PER ? c[(long)(n - 1) * ld + s] : 0.0;
  double* zu = PER ? ws : nullptr;
  double* wv = PER ? ws + (long)n * ldw : nullptr;
  TriFwd st;
  for (int i = 0; i < n; ++i) {
    const long r = (long)i * ld + s;
    double inv, ch, y, z, w;
    tri_fwd_row<PER, false>(i, n, a[r], b[r], c[r], 0.0, a0, b0, cl, st, inv, ch, y, z, w);
    b[r] = inv;
    c[r] = ch;
    if (PER) {
      zu[(long)i * ldw + s] = z;
      wv[(long)i * ldw + s] = w;
    }
  }
  if (PER) ws[2L * n * ldw + s] = 1.0 / (1.0 + st.sz);
}

template <bool PER>
__global__ __launch_bounds__(kThreads) void tri_batch_solve_k(int n, int batch, long ld,
                                                              const double* __restrict__ a,
                                                              const double* __restrict__ b,
                                                              const double* __restrict__ c,
                                                              const double* __restrict__ ws,
                                                              long ldw, double* __restrict__ x) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const double* wv = PER ? ws + (long)n * ldw : nullptr;
  double y1 = 0.0, sy = 0.0;
  int i = 0;
  for (; i + kUS <= n; i += kUS) {
    double va[kUS], vb[kUS], vf[kUS], vw[kUS];
#pragma unroll
    for (int u = 0; u < kUS; ++u) {
      const long r = (long)(i + u) * ld + s;
      va[u] = __builtin_nontemporal_load(&a[r]);
      vb[u] = __builtin_nontemporal_load(&b[r]);
      vf[u] = __builtin_nontemporal_load(&x[r]);
      if (PER) vw[u] = __builtin_nontemporal_load(&wv[(long)(i + u) * ldw + s]);
    }
#pragma unroll
    for (int u = 0; u < kUS; ++u) {
      const double ai = (i + u >= 1) ? va[u] : 0.0;
      const double y = (vf[u] - ai * y1) * vb[u];
      x[(long)(i + u) * ld + s] = y;
      if (PER) sy = sy + vw[u] * y;
      y1 = y;
    }
  }
  for (; i < n; ++i) {
    const long r = (long)i * ld + s;
    const double ai = (i >= 1) ? a[r] : 0.0;
    const double y = (x[r] - ai * y1) * b[r];
    x[r] = y;
    if (PER) sy = sy + wv[(long)i * ldw + s] * y;
    y1 = y;
  }
  const double phi = PER ? sy * ws[2L * n * ldw + s] : 0.0;
  tri_back<kUS, PER>(n, s, c, ld, PER ? ws : nullptr, ldw, phi, x, ld);
}

template <bool PER>
__global__ __launch_bounds__(kThreads) void tri_batch_rewrite_k(
    int n, int batch, long ld, const double* __restrict__ a, const double* __restrict__ b,
    const double* __restrict__ c, double* __restrict__ x, double* __restrict__ ws, long ldw) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  if (s >= batch) return;
  const double a0 = PER ? a[s] : 0.0, b0 = PER ? b[s] : 0.0;
  const double cl = PER ? c[(long)(n - 1) * ld + s] : 0.0;
  double* chv = ws;
  double* zu = PER ? ws + (long)n * ldw : nullptr;
  TriFwd st;
  int i = 0;
  for (; i + kU <= n; i += kU) {
    double va[kU], vb[kU], vc[kU], vf[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long r = (long)(i + u) * ld + s;
      va[u] = __builtin_nontemporal_load(&a[r]);
      vb[u] = __builtin_nontemporal_load(&b[r]);
      vc[u] = __builtin_nontemporal_load(&c[r]);
      vf[u] = __builtin_nontemporal_load(&x[r]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      double inv, ch, y, z, w;
      tri_fwd_row<PER, true>(i + u, n, va[u], vb[u], vc[u], vf[u], a0, b0, cl, st, inv, ch, y,
                             z, w);
      const long rw = (long)(i + u) * ldw + s;
      x[(long)(i + u) * ld + s] = y;
      chv[rw] = ch;
      if (PER) zu[rw] = z;
    }
  }
  for (; i < n; ++i) {
    const long r = (long)i * ld + s;
    double inv, ch, y, z, w;
    tri_fwd_row<PER, true>(i, n, a[r], b[r], c[r], x[r], a0, b0, cl, st, inv, ch, y, z, w);
    const long rw = (long)i * ldw + s;
    x[r] = y;
    chv[rw] = ch;
    if (PER) zu[rw] = z;
  }
  const double phi = PER ? st.sy / (1.0 + st.sz) : 0.0;
  tri_back<kU, PER>(n, s, chv, ldw, zu, ldw, phi, x, ld);
}

// ---------------------------------------------------------------------------
// Host side: argument checks, workspace layout, launches.
// ---------------------------------------------------------------------------

long ws_ld(int batch) { return ((long)batch + 31) / 32 * 32; }  // 256-byte rows

size_t penta_ws_doubles(int n, int batch, int periodic, int mode) {
  const long m = periodic ? n - 2 : n;
  const long ldw = ws_ld(batch);
  if (mode == CHX_BATCH_REWRITE) return (size_t)((periodic ? 4 : 2) * m * ldw);
  return periodic ? (size_t)((4 * m + 4) * ldw) : 0;
}

size_t tri_ws_doubles(int n, int batch, int periodic, int mode) {
  const long ldw = ws_ld(batch);
  if (mode == CHX_BATCH_REWRITE) return (size_t)((periodic ? 2 : 1) * (long)n * ldw);
  return periodic ? (size_t)((2L * n + 1) * ldw) : 0;
}

int check_common(int n, int batch, long ld, int nmin, int periodic) {
  if (batch < 0 || ld < batch || ld < 1 || (periodic != 0 && periodic != 1)) return CHX_EINVAL;
  if (n < nmin) return CHX_EUNSUPPORTED_N;
  return CHX_OK;
}

int check_ws(const void* ws, size_t ws_bytes, size_t need_doubles) {
  if (need_doubles == 0) return CHX_OK;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return CHX_EINVAL;
  if (ws_bytes < need_doubles * sizeof(double)) return CHX_ENOMEM;
  return CHX_OK;
}

dim3 grid_of(int batch) { return dim3((unsigned)((batch + kThreads - 1) / kThreads)); }

int launched() { return hipGetLastError() == hipSuccess ? CHX_OK : CHX_EHIP; }

// Every entry of up to five band arrays set to that band's value.
struct FillBands {
  double* band[5];
  double value[5];
};

__global__ __launch_bounds__(kThreads) void fill_bands_k(FillBands fb, int nb, int n, int batch,
                                                         long ld) {
  const long s = (long)blockIdx.x * kThreads + threadIdx.x;
  const int i = blockIdx.y;
  if (s >= batch) return;
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if (k < nb) fb.band[k][(long)i * ld + s] = fb.value[k];
}

}  // namespace chx_vb

using namespace chx_vb;

// Internal launchers for the batched 1D schemes' rewrite mode.
namespace chx {

hipError_t vb_fill_bands(int nb, double* const* bands, const double* values, int n, int batch,
                         long ld, hipStream_t st) {
  if (nb < 1 || nb > 5) return hipErrorInvalidValue;
  FillBands fb{};
  for (int k = 0; k < nb; ++k) {
    fb.band[k] = bands[k];
    fb.value[k] = values[k];
  }
  hipLaunchKernelGGL(fill_bands_k, dim3((unsigned)((batch + kThreads - 1) / kThreads), n),
                     dim3(kThreads), 0, st, fb, nb, n, batch, ld);
  return hipGetLastError();
}

size_t vb_rewrite_ws_bytes(int P, int n, int batch) {
  return P == 2 ? penta_ws_doubles(n, batch, 1, CHX_BATCH_REWRITE) * sizeof(double)
                : tri_ws_doubles(n, batch, 1, CHX_BATCH_REWRITE) * sizeof(double);
}

hipError_t vb_penta_rewrite_periodic(int n, int batch, const double* const* b, long ld, double* x,
                                     double* ws, hipStream_t st) {
  hipLaunchKernelGGL(penta_batch_rewrite_k<true>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                     ld, b[0], b[1], b[2], b[3], b[4], x, ws, ws_ld(batch));
  return hipGetLastError();
}

hipError_t vb_tri_rewrite_periodic(int n, int batch, const double* const* b, long ld, double* x,
                                   double* ws, hipStream_t st) {
  hipLaunchKernelGGL(tri_batch_rewrite_k<true>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                     ld, b[0], b[1], b[2], x, ws, ws_ld(batch));
  return hipGetLastError();
}

}  // namespace chx

extern "C" {

size_t penta_batch_ws_bytes(int n, int batch, int periodic, int mode) {
  if (n < (periodic ? 5 : 3) || batch < 0 || (mode != CHX_BATCH_FACTOR && mode != CHX_BATCH_REWRITE))
    return 0;
  return penta_ws_doubles(n, batch, periodic != 0, mode) * sizeof(double);
}

size_t tri_batch_ws_bytes(int n, int batch, int periodic, int mode) {
  if (n < (periodic ? 3 : 2) || batch < 0 || (mode != CHX_BATCH_FACTOR && mode != CHX_BATCH_REWRITE))
    return 0;
  return tri_ws_doubles(n, batch, periodic != 0, mode) * sizeof(double);
}

int penta_batch_factor(int n, int batch, int periodic, double* a, double* b, double* c, double* d,
                       double* e, long ld, void* ws, size_t ws_bytes, chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 5 : 3, periodic);
  if (rc) return rc;
  if (!a || !b || !c || !d || !e) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, penta_ws_doubles(n, batch, periodic, CHX_BATCH_FACTOR));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* w = static_cast<double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(penta_batch_factor_k<true>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, w, ws_ld(batch));
  else
    hipLaunchKernelGGL(penta_batch_factor_k<false>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, w, ws_ld(batch));
  return launched();
}

int penta_batch_solve(int n, int batch, int periodic, const double* a, const double* b,
                      const double* c, const double* d, const double* e, long ld, const void* ws,
                      size_t ws_bytes, double* x, chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 5 : 3, periodic);
  if (rc) return rc;
  if (!a || !b || !c || !d || !e || !x) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, penta_ws_doubles(n, batch, periodic, CHX_BATCH_FACTOR));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  const double* w = static_cast<const double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(penta_batch_solve_k<true>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, w, ws_ld(batch), x);
  else
    hipLaunchKernelGGL(penta_batch_solve_k<false>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, w, ws_ld(batch), x);
  return launched();
}

int penta_batch_rewrite(int n, int batch, int periodic, const double* a, const double* b,
                        const double* c, const double* d, const double* e, long ld, double* x,
                        void* ws, size_t ws_bytes, chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 5 : 3, periodic);
  if (rc) return rc;
  if (!a || !b || !c || !d || !e || !x) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, penta_ws_doubles(n, batch, periodic, CHX_BATCH_REWRITE));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* w = static_cast<double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(penta_batch_rewrite_k<true>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, x, w, ws_ld(batch));
  else
    hipLaunchKernelGGL(penta_batch_rewrite_k<false>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, d, e, x, w, ws_ld(batch));
  return launched();
}

int tri_batch_factor(int n, int batch, int periodic, double* a, double* b, double* c, long ld,
                     void* ws, size_t ws_bytes, chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 3 : 2, periodic);
  if (rc) return rc;
  if (!a || !b || !c) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, tri_ws_doubles(n, batch, periodic, CHX_BATCH_FACTOR));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* w = static_cast<double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(tri_batch_factor_k<true>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                       ld, a, b, c, w, ws_ld(batch));
  else
    hipLaunchKernelGGL(tri_batch_factor_k<false>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                       ld, a, b, c, w, ws_ld(batch));
  return launched();
}

int tri_batch_solve(int n, int batch, int periodic, const double* a, const double* b,
                    const double* c, long ld, const void* ws, size_t ws_bytes, double* x,
                    chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 3 : 2, periodic);
  if (rc) return rc;
  if (!a || !b || !c || !x) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, tri_ws_doubles(n, batch, periodic, CHX_BATCH_FACTOR));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  const double* w = static_cast<const double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(tri_batch_solve_k<true>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                       ld, a, b, c, w, ws_ld(batch), x);
  else
    hipLaunchKernelGGL(tri_batch_solve_k<false>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                       ld, a, b, c, w, ws_ld(batch), x);
  return launched();
}

int tri_batch_rewrite(int n, int batch, int periodic, const double* a, const double* b,
                      const double* c, long ld, double* x, void* ws, size_t ws_bytes,
                      chx_stream s) {
  int rc = check_common(n, batch, ld, periodic ? 3 : 2, periodic);
  if (rc) return rc;
  if (!a || !b || !c || !x) return CHX_EINVAL;
  rc = check_ws(ws, ws_bytes, tri_ws_doubles(n, batch, periodic, CHX_BATCH_REWRITE));
  if (rc) return rc;
  if (batch == 0) return CHX_OK;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* w = static_cast<double*>(ws);
  if (periodic)
    hipLaunchKernelGGL(tri_batch_rewrite_k<true>, grid_of(batch), dim3(kThreads), 0, st, n, batch,
                       ld, a, b, c, x, w, ws_ld(batch));
  else
    hipLaunchKernelGGL(tri_batch_rewrite_k<false>, grid_of(batch), dim3(kThreads), 0, st, n,
                       batch, ld, a, b, c, x, w, ws_ld(batch));
  return launched();
}

}  // extern "C"
