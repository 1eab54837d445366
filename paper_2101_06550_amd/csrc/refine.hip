// refine.hip -- column kernels of the FP32-refined ADI step (FP32 sweeps,
// FP64 right-hand side, residual and state).
//
// One step of (I + sx Px)(I + sy Py) c_new = r with FP32 sweeps and FP64
// residual refinement (x_0 = A32^{-1} r; x_{k+1} = x_k + A32^{-1}(r - A x_k)),
// laid out like the FP64 step: a column kernel that sweeps every 32-row chunk
// of every column in registers, the column separators, and a row kernel that
// solves whole rows in LDS.  The column-chunk correction is deferred: the row
// kernel writes V_k (FP32, interior rows uncorrected, separator rows final)
// and every later kernel rebuilds the correction d_k = V_k - Zl T_prev - Zr T_own
// as it reads V_k.  Since that rebuild is linear, the sum V_0 + ... + V_m is
// formed first (FP64) and corrected once, giving x_m.  Per point and pass:
//   rstep_first : read c (8 B), write r (8) and the FP32 chunk interiors (4)
//   rstep_resid : read r (8) and V_0 .. V_{k-1} (4 k), write the FP32 chunk
//                 interiors of R = r - A x_{k-1} swept (4)
//   rows (FP32) : read 4, write V_k (4)
//   rstep_final : read V_0 .. V_p (4 (p + 1)), write c (8)
// Every kernel runs one wave per 64 columns (i0 = 64 seg .. i0 + 63) of one
// 32-row chunk, so every row segment it loads or stores is whole, aligned
// cache lines.  Neighbours at distance 1 and 2 come from DPP lane shifts --
// no LDS, no barrier: the lanes at the wave's edges also form the state of
// the columns just outside it (lane 0: i0 - 1, lane 1: i0 - 2, lane 63:
// i0 + 64, lane 62: i0 + 65, wrapped), the same arithmetic the owning wave
// does, and the shifts take those values in at the edges.  A wave's (mass,
// energy) partial goes to slot kc * nseg + seg.
#include <hip/hip_runtime.h>

#include "ch_launch.hpp"
#include "common.hpp"
#include "ens.hpp"

namespace chx {

namespace {

constexpr int M = kChunk;
constexpr int P = 2;
constexpr int MI = M - P;
constexpr int kSegR = 64;  // output columns per wave
constexpr int kPfR = 4;    // rows of loads in flight ahead of the row worked

__device__ __forceinline__ double wave_sum_r(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int wrap_row(int j, int ny) {
  j += (j < 0) ? ny : 0;
  j -= (j >= ny) ? ny : 0;
  return j;
}

// Lane geometry of wave `seg` (nx is a multiple of 64): the lane's column i,
// and the column ex whose state it also forms for the shifts -- with HALO = 2
// the two columns on either side of the wave (lanes 0, 1, 62, 63), with
// HALO = 1 the nearest one (lanes 0 and 63); the other lanes their own.
struct Lanes {
  int i, ex;
};
template <int HALO>
__device__ __forceinline__ Lanes lanes_of(int seg, int nx) {
  const int lane = threadIdx.x & 63;
  const int i0 = seg * kSegR;
  Lanes L;
  L.i = i0 + lane;
  int ex = L.i;
  if (lane == 0) ex = i0 - 1;
  if (lane == 63) ex = i0 + 64;
  if (HALO == 2 && lane == 1) ex = i0 - 2;
  if (HALO == 2 && lane == 62) ex = i0 + 65;
  ex += (ex < 0) ? nx : 0;
  ex -= (ex >= nx) ? nx : 0;
  L.ex = ex;
  return L;
}

// Value of the column at distance 1 / 2 to the left / right of the lane's,
// h being the edge lanes' halo values of the same row (lanes_of).
__device__ __forceinline__ double left1(double x, double h) { return dpp_from_left(x, h); }
__device__ __forceinline__ double left2(double l1, double h) {
  return dpp_from_left(l1, dpp_from_right(h, h));
}
__device__ __forceinline__ double right1(double x, double h) { return dpp_from_right(x, h); }
__device__ __forceinline__ double right2(double r1, double h) {
  return dpp_from_right(r1, dpp_from_left(h, h));
}

// Forward-sweep step p of the FP32 chunk interior (the g of chunk_sweep).
template <typename TP32>
__device__ __forceinline__ float fwd32(float v, int p, const float (&f)[M],
                                       TP32 __restrict__ rec, float eps) {
  if (p < MI) {
    if (p >= 2) v = v - eps * f[p - 2];
    if (p >= 1) v = v - rec[p * 8 + 1] * f[p - 1];
    v = v * rec[p * 8 + 0];
  }
  return v;
}

// Back sweep, separator parts and stores of one FP32 chunk.
template <typename TP32>
__device__ __forceinline__ void finish32(float (&f)[M], TP32 __restrict__ rec,
                                         const BandT<float>& bd, float* __restrict__ y32,
                                         float* __restrict__ rho, int nx, int kc, int io) {
#pragma unroll
  for (int p = MI - 1; p >= 0; --p) {
    float v = f[p];
    if (p + 2 < MI) v = v - rec[p * 8 + 3] * f[p + 2];
    if (p + 1 < MI) v = v - rec[p * 8 + 2] * f[p + 1];
    f[p] = v;
  }
  float pa[P], pb[P];
  chunk_parts<P, M, float>(f, bd, pa, pb);
#pragma unroll
  for (int p = 0; p < MI; ++p) __builtin_nontemporal_store(f[p], &y32[((long)kc * M + p) * nx + io]);
#pragma unroll
  for (int a = 0; a < P; ++a) {
    rho[((long)kc * 2 * P + a) * nx + io] = pa[a];
    rho[((long)kc * 2 * P + P + a) * nx + io] = pb[a];
  }
}

}  // namespace

// The deferred FP32 solutions V_0 .. V_{NB-1} of a step (dense, ld = nx).
struct RBufs {
  const float* v[4];
};

// The bodies below take their pointers' types as template parameters: the
// single-field kernels pass their restrict kernel arguments, the ensemble
// kernels pointers read out of run records, typed by address space.
struct RBufsG {
  GCF v[4];
};

// Sum over the buffers of rows j (FP64).
template <int NB, typename BV>
__device__ __forceinline__ double vsum(const BV& B, long j, int nx, int i) {
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < NB; ++b) s += (double)B.v[b][j * nx + i];
  return s;
}

// First pass of a refined step: r = RHS(c) in FP64 (written out for the
// residuals of the later passes), swept in FP32; DIAG: mass and free energy
// of c.  Window rows kc M - 1 .. kc M + M.  NB = 0: c is read from the
// caller's array; NB > 0 (every step of a call after the first): c is the
// previous step's solution, rebuilt from its deferred FP32 solutions
// V_0 .. V_{NB-1} as it is read (so the state is not written and read back
// between the steps of a call).
template <bool DIAG, int NB = 0, typename CP = const double*, typename TP32 = const float*,
          typename BV = RBufs, typename TP = const double*>
__device__ __forceinline__ void rstep_first_body(CP __restrict__ c, long ld,
                                                 double* __restrict__ rbuf,
                                                 float* __restrict__ y32,
                                                 float* __restrict__ rho, int nx, int ny,
                                                 int nseg, TP32 __restrict__ rec32,
                                                 const BandT<float>& bd, const ChCoef& K,
                                                 double* __restrict__ part, int seg, int kc,
                                                 const BV& Bv = BV{}, int Sc = 1,
                                                 TP __restrict__ rec = nullptr) {
  const Lanes L = lanes_of<1>(seg, nx);
  constexpr int Q = M + 2;
  // separator rows (final values) of chunks kc - 1, kc, kc + 1 at the lane's
  // column (s[0]) and at its halo column (s[1])
  double tp[2][P] = {}, to[2][P] = {}, tn[2][P] = {};
  if (NB > 0) {
    const int kcm = (kc == 0) ? Sc - 1 : kc - 1, kcp = (kc + 1 == Sc) ? 0 : kc + 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = h ? L.ex : L.i;
#pragma unroll
      for (int a = 0; a < P; ++a) {
        tp[h][a] = vsum<NB>(Bv, (long)kcm * M + MI + a, nx, col);
        to[h][a] = vsum<NB>(Bv, (long)kc * M + MI + a, nx, col);
        tn[h][a] = vsum<NB>(Bv, (long)kcp * M + MI + a, nx, col);
      }
    }
  }
  double X[Q], XH[Q];
  auto value = [&](int t, int h) {
    const int col = h ? L.ex : L.i;
    if (NB == 0) return (double)c[(long)wrap_row(kc * M - 1 + t, ny) * ld + col];
    // window row t: t = 0 is chunk kc-1's last separator, t = 1 .. M chunk
    // kc's position t - 1, t = M + 1 chunk kc+1's position 0
    double x = vsum<NB>(Bv, wrap_row(kc * M - 1 + t, ny), nx, col);
    if (t >= 1) {
      const bool below = t == M + 1;
      const int pp = below ? 0 : t - 1;
      if (pp < MI) {
#pragma unroll
        for (int a = 0; a < P; ++a)
          x = x - rec[pp * 8 + 4 + a] * (below ? to[h][a] : tp[h][a]) -
              rec[pp * 8 + 6 + a] * (below ? tn[h][a] : to[h][a]);
      }
    }
    return x;
  };
  auto load = [&](int t) {
    X[t] = value(t, 0);
    XH[t] = value(t, 1);
  };
#pragma unroll
  for (int t = 0; t < kPfR; ++t) load(t);
  double XL[Q], XR[Q];
  float f[M];
  double msum = 0.0, esum = 0.0;
  const float eps = bd.c[0];
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    if (t + kPfR < Q) load(t + kPfR);
    XL[t] = left1(X[t], XH[t]);
    XR[t] = right1(X[t], XH[t]);
    if (t >= 2) {  // own row p = t - 2 at window index w = t - 1
      const int p = t - 2, w = t - 1;
      const double xc = X[w], xl = XL[w], xr = XR[w];
      const double mu_c = xc * xc * xc - xc;
      const double mu_l = xl * xl * xl - xl;
      const double mu_r = xr * xr * xr - xr;
      const double mu_s = X[w - 1] * X[w - 1] * X[w - 1] - X[w - 1];
      const double mu_n = X[w + 1] * X[w + 1] * X[w + 1] - X[w + 1];
      const double lap = K.cx * (mu_r + mu_l - 2.0 * mu_c) + K.cy * (mu_n + mu_s - 2.0 * mu_c);
      const double dyy_w = XL[w + 1] + XL[w - 1] - 2.0 * xl;
      const double dyy_c = X[w + 1] + X[w - 1] - 2.0 * xc;
      const double dyy_e = XR[w + 1] + XR[w - 1] - 2.0 * xr;
      const double r = xc + lap - K.ccross * (dyy_e + dyy_w - 2.0 * dyy_c);
      if (DIAG) {
        const double q = xc * xc - 1.0;
        const double gx = (xr - xc) * K.inv_dx, gy = (X[w + 1] - xc) * K.inv_dy;
        msum += xc;
        esum += 0.25 * q * q + K.half_gamma * (gx * gx + gy * gy);
      }
      __builtin_nontemporal_store(r, &rbuf[((long)kc * M + p) * nx + L.i]);
      f[p] = fwd32((float)r, p, f, rec32, eps);
      asm volatile("" : "+v"(f[p]));
    }
    asm volatile("" : "+v"(X[t]), "+v"(XH[t]), "+v"(XL[t]), "+v"(XR[t])::"memory");
  }
  finish32(f, rec32, bd, y32, rho, nx, kc, L.i);
  if (DIAG) {
    msum = wave_sum_r(msum);
    esum = wave_sum_r(esum);
    if ((threadIdx.x & 63) == 0) {
      part[2 * ((long)kc * nseg + seg)] = msum;
      part[2 * ((long)kc * nseg + seg) + 1] = esum;
    }
  }
}

// Later pass k = NB of a refined step: x = sum of the rebuilt V_0 .. V_{NB-1}
// (window rows kc M - 2 .. kc M + M + 1, separators of chunks kc - 1, kc,
// kc + 1 first), R = r - (I + sx Px)(I + sy Py) x in FP64, swept in FP32.
template <int NB, typename BV, typename TP, typename TP32>
__device__ __forceinline__ void rstep_resid_body(const double* __restrict__ rbuf, const BV& B,
                                                 float* __restrict__ y32,
                                                 float* __restrict__ rho, int nx, int ny,
                                                 int Sc, TP __restrict__ rec,
                                                 TP32 __restrict__ rec32,
                                                 const BandT<float>& bd, const BandT<double>& ax,
                                                 const BandT<double>& ay, int seg, int kc) {
  const Lanes L = lanes_of<2>(seg, nx);
  const int kcm = (kc == 0) ? Sc - 1 : kc - 1, kcp = (kc + 1 == Sc) ? 0 : kc + 1;
  // separators at the lane's column (h = 0) and at its halo column (h = 1)
  double tp[2][P], to[2][P], tn[2][P];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int col = h ? L.ex : L.i;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      tp[h][a] = vsum<NB>(B, (long)kcm * M + MI + a, nx, col);
      to[h][a] = vsum<NB>(B, (long)kc * M + MI + a, nx, col);
      tn[h][a] = vsum<NB>(B, (long)kcp * M + MI + a, nx, col);
    }
  }
  constexpr int Q = M + 4;  // window rows kc M - 2 .. kc M + M + 1
  double U[Q], UH[Q], R[M];
  auto load = [&](int t) {
    U[t] = vsum<NB>(B, wrap_row(kc * M - 2 + t, ny), nx, L.i);
    UH[t] = vsum<NB>(B, wrap_row(kc * M - 2 + t, ny), nx, L.ex);
    if (t >= 2 && t < M + 2) R[t - 2] = rbuf[((long)kc * M + t - 2) * nx + L.i];
  };
#pragma unroll
  for (int t = 0; t < kPfR; ++t) load(t);
  double X[Q], XH[Q];
  float f[M];
  const float eps = bd.c[0];
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    if (t + kPfR < Q) load(t + kPfR);
    // the state at window row t: rows above (t < 2) are chunk kc-1's
    // separators; own rows (2 .. M+1) chunk kc, position t - 2; the two rows
    // below chunk kc+1, positions 0 and 1
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double x = h ? UH[t] : U[t];
      if (t >= 2) {
        const bool below = t >= M + 2;
        const int pp = below ? t - M - 2 : t - 2;
        if (pp < MI) {
#pragma unroll
          for (int a = 0; a < P; ++a)
            x = x - rec[pp * 8 + 4 + a] * (below ? to[h][a] : tp[h][a]) -
                rec[pp * 8 + 6 + a] * (below ? tn[h][a] : to[h][a]);
        }
      }
      if (h) XH[t] = x;
      else X[t] = x;
    }
    if (t >= 4) {  // own row p = t - 4 at window index w = t - 2
      const int p = t - 4, w = t - 2;
      const double Ty = ay.c[0] * X[w - 2] + ay.c[1] * X[w - 1] + ay.c[2] * X[w] +
                        ay.c[3] * X[w + 1] + ay.c[4] * X[w + 2];
      const double TyH = ay.c[0] * XH[w - 2] + ay.c[1] * XH[w - 1] + ay.c[2] * XH[w] +
                         ay.c[3] * XH[w + 1] + ay.c[4] * XH[w + 2];
      const double l1 = left1(Ty, TyH), l2 = left2(l1, TyH);
      const double r1 = right1(Ty, TyH), r2 = right2(r1, TyH);
      const double Ax = ax.c[0] * l2 + ax.c[1] * l1 + ax.c[2] * Ty + ax.c[3] * r1 + ax.c[4] * r2;
      f[p] = fwd32((float)(R[p] - Ax), p, f, rec32, eps);
      asm volatile("" : "+v"(f[p]));
    }
    asm volatile("" : "+v"(X[t]), "+v"(XH[t])::"memory");
  }
  finish32(f, rec32, bd, y32, rho, nx, kc, L.i);
}

// End of a refined step: x = sum of the rebuilt V_0 .. V_{NB-1}, written to
// c (FP64); DIAG: mass and free energy of x.  Window rows kc M .. kc M + M.
template <int NB, bool DIAG, typename BV, typename CP, typename TP>
__device__ __forceinline__ void rstep_final_body(const BV& B, CP __restrict__ c, long ld,
                                                 int nx, int ny, int nseg, int Sc,
                                                 TP __restrict__ rec, const ChCoef& K,
                                                 double* __restrict__ part, int seg, int kc) {
  // DIAG needs the right neighbour: lane 63 also forms column i0 + 64
  const Lanes L = lanes_of<1>(seg, nx);
  constexpr int NH = DIAG ? 2 : 1;
  const int kcm = (kc == 0) ? Sc - 1 : kc - 1, kcp = (kc + 1 == Sc) ? 0 : kc + 1;
  double tp[2][P] = {}, to[2][P] = {}, tn[2][P] = {};
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    const int col = h ? L.ex : L.i;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      tp[h][a] = vsum<NB>(B, (long)kcm * M + MI + a, nx, col);
      to[h][a] = vsum<NB>(B, (long)kc * M + MI + a, nx, col);
      tn[h][a] = DIAG ? vsum<NB>(B, (long)kcp * M + MI + a, nx, col) : 0.0;
    }
  }
  constexpr int Q = M + 1;  // own rows and (DIAG) row 0 of chunk kc + 1
  double U[Q], UH[Q];
  auto load = [&](int t) {
    if (t < M || DIAG) U[t] = vsum<NB>(B, wrap_row(kc * M + t, ny), nx, L.i);
    if (DIAG) UH[t] = vsum<NB>(B, wrap_row(kc * M + t, ny), nx, L.ex);
  };
#pragma unroll
  for (int t = 0; t < kPfR; ++t) load(t);
  double X[Q], XH[Q];
  double msum = 0.0, esum = 0.0;
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    if (t + kPfR < Q) load(t + kPfR);
    if (t == M && !DIAG) break;
    const bool below = t == M;
    const int pp = below ? 0 : t;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      double x = h ? UH[t] : U[t];
      if (pp < MI) {
#pragma unroll
        for (int a = 0; a < P; ++a)
          x = x - rec[pp * 8 + 4 + a] * (below ? to[h][a] : tp[h][a]) -
              rec[pp * 8 + 6 + a] * (below ? tn[h][a] : to[h][a]);
      }
      if (h) XH[t] = x;
      else X[t] = x;
    }
    if (t < M) __builtin_nontemporal_store(X[t], &c[((long)kc * M + t) * ld + L.i]);
    if (DIAG && t >= 1) {  // row t - 1 with its neighbours (i + 1, j) and (i, j + 1)
      const double xc = X[t - 1];
      const double xr = right1(xc, XH[t - 1]);
      const double q = xc * xc - 1.0;
      const double gx = (xr - xc) * K.inv_dx, gy = (X[t] - xc) * K.inv_dy;
      msum += xc;
      esum += 0.25 * q * q + K.half_gamma * (gx * gx + gy * gy);
    }
    asm volatile("" : "+v"(X[t])::"memory");
    if (DIAG) asm volatile("" : "+v"(XH[t])::"memory");
  }
  if (DIAG) {
    msum = wave_sum_r(msum);
    esum = wave_sum_r(esum);
    if ((threadIdx.x & 63) == 0) {
      part[2 * ((long)kc * nseg + seg)] = msum;
      part[2 * ((long)kc * nseg + seg) + 1] = esum;
    }
  }
}

// Single-field kernels: block = 4 waves = 4 consecutive (64-column segment,
// chunk) pairs, segments fastest (full blocks whatever the segment count).
template <bool DIAG, int NB>
__global__ __launch_bounds__(256) void rstep_first(const double* __restrict__ c, long ld,
                                                   double* __restrict__ rbuf,
                                                   float* __restrict__ y32,
                                                   float* __restrict__ rho, int nx, int ny,
                                                   int nseg, const float* __restrict__ rec32,
                                                   BandT<float> bd, ChCoef K,
                                                   double* __restrict__ part, RBufs Bv, int Sc,
                                                   const double* __restrict__ rec) {
  const int li = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int seg = li % nseg, kc = li / nseg;
  if (kc >= Sc) return;  // no barrier in this kernel
  rstep_first_body<DIAG, NB>(c, ld, rbuf, y32, rho, nx, ny, nseg, rec32, bd, K, part, seg, kc,
                             Bv, Sc, rec);
}

template <int NB>
__global__ __launch_bounds__(256) void rstep_resid(const double* __restrict__ rbuf, RBufs B,
                                                   float* __restrict__ y32,
                                                   float* __restrict__ rho, int nx, int ny,
                                                   int nseg, int Sc,
                                                   const double* __restrict__ rec,
                                                   const float* __restrict__ rec32,
                                                   BandT<float> bd, BandT<double> ax,
                                                   BandT<double> ay) {
  const int li = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int seg = li % nseg, kc = li / nseg;
  if (kc >= Sc) return;  // no barrier in this kernel
  rstep_resid_body<NB>(rbuf, B, y32, rho, nx, ny, Sc, rec, rec32, bd, ax, ay, seg, kc);
}

template <int NB, bool DIAG>
__global__ __launch_bounds__(256) void rstep_final(RBufs B, double* __restrict__ c, long ld,
                                                   int nx, int ny, int nseg, int Sc,
                                                   const double* __restrict__ rec, ChCoef K,
                                                   double* __restrict__ part) {
  const int li = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int seg = li % nseg, kc = li / nseg;
  if (kc >= Sc) return;  // no barrier in this kernel
  rstep_final_body<NB, DIAG>(B, c, ld, nx, ny, nseg, Sc, rec, K, part, seg, kc);
}

// Ensemble kernels: block = work item {run, segment block, chunk}; each run
// reads its class's plan tables and its own buffers, and calls the bodies
// the single-field kernels call (so a run advances bitwise as it would alone).
__device__ __forceinline__ RBufsG ens_vbufs(unsigned char* ws, const EnsRun& R) {
  RBufsG B{};
#pragma unroll
  for (int b = 0; b < 4; ++b) B.v[b] = (GCF)(ws + R.off_v[b]);
  return B;
}

template <int PASS, bool DIAG, bool FROMV = false>
__global__ __launch_bounds__(256) void ens_rstep_column(const EnsRun* __restrict__ runs,
                                                        EnsClasses cls,
                                                        const int4* __restrict__ items,
                                                        unsigned char* ws) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  // a run's (segment, chunk) pairs packed four to a block, so that blocks
  // are full on grids whose rows span few 64-column segments
  const int li = it.y * 4 + (threadIdx.x >> 6);
  const int seg = li % R.nseg, kc = li / R.nseg;
  if (kc >= R.Sc) return;  // no barrier in these kernels
  const EnsClass& C = cls.c[R.cls];
  BandT<float> bd;
#pragma unroll
  for (int k = 0; k < 5; ++k) bd.c[k] = (float)C.py.coef[k];
  double* rbuf = reinterpret_cast<double*>(ws + R.off_r);
  float* y32 = reinterpret_cast<float*>(ws + R.off_y32);
  float* rho = reinterpret_cast<float*>(ws + R.off_rho32);
  if (PASS == 0 && !FROMV) {
    rstep_first_body<DIAG>((GCD)R.c, R.ldc, rbuf, y32, rho, R.nx, R.ny, R.nseg,
                           (TabF)C.py.rec32, bd, C.K, reinterpret_cast<double*>(ws + R.off_part),
                           seg, kc);
  } else if (PASS == 0) {  // the state rebuilt from the previous step's solutions
    double* part = reinterpret_cast<double*>(ws + R.off_part);
    const RBufsG Bv = ens_vbufs(ws, R);
    switch (R.passes) {  // uniform per block
      case 1: rstep_first_body<DIAG, 2>((GCD)R.c, R.ldc, rbuf, y32, rho, R.nx, R.ny, R.nseg, (TabF)C.py.rec32, bd, C.K, part, seg, kc, Bv, R.Sc, (TabD)C.py.rec); break;
      case 2: rstep_first_body<DIAG, 3>((GCD)R.c, R.ldc, rbuf, y32, rho, R.nx, R.ny, R.nseg, (TabF)C.py.rec32, bd, C.K, part, seg, kc, Bv, R.Sc, (TabD)C.py.rec); break;
      default: rstep_first_body<DIAG, 4>((GCD)R.c, R.ldc, rbuf, y32, rho, R.nx, R.ny, R.nseg, (TabF)C.py.rec32, bd, C.K, part, seg, kc, Bv, R.Sc, (TabD)C.py.rec); break;
    }
  } else {
    BandT<double> ax, ay;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      ax.c[k] = C.px.coef[k];
      ay.c[k] = C.py.coef[k];
    }
    rstep_resid_body<PASS>(rbuf, ens_vbufs(ws, R), y32, rho, R.nx, R.ny, R.Sc, (TabD)C.py.rec,
                           (TabF)C.py.rec32, bd, ax, ay, seg, kc);
  }
}

template <bool DIAG>
__global__ __launch_bounds__(256) void ens_rstep_final(const EnsRun* __restrict__ runs,
                                                       EnsClasses cls,
                                                       const int4* __restrict__ items,
                                                       unsigned char* ws) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const int li = it.y * 4 + (threadIdx.x >> 6);  // packed as in ens_rstep_column
  const int seg = li % R.nseg, kc = li / R.nseg;
  if (kc >= R.Sc) return;
  const EnsClass& C = cls.c[R.cls];
  const RBufsG B = ens_vbufs(ws, R);
  double* part = reinterpret_cast<double*>(ws + R.off_part);
  switch (R.passes) {  // uniform per block
    case 1: rstep_final_body<2, DIAG>(B, (GD)R.c, R.ldc, R.nx, R.ny, R.nseg, R.Sc, (TabD)C.py.rec, C.K, part, seg, kc); break;
    case 2: rstep_final_body<3, DIAG>(B, (GD)R.c, R.ldc, R.nx, R.ny, R.nseg, R.Sc, (TabD)C.py.rec, C.K, part, seg, kc); break;
    default: rstep_final_body<4, DIAG>(B, (GD)R.c, R.ldc, R.nx, R.ny, R.nseg, R.Sc, (TabD)C.py.rec, C.K, part, seg, kc); break;
  }
}

hipError_t launch_ens_rstep_column(int pass, bool diag, const EnsRun* runs, const EnsClasses& cls,
                                   const int4* items, int nitems, unsigned char* ws,
                                   hipStream_t st, bool from_v) {
  if (nitems <= 0) return hipSuccess;
#define CHX_ERC(P_, D_, F_)                                                                      \
  hipLaunchKernelGGL((ens_rstep_column<P_, D_, F_>), dim3(nitems), dim3(256), 0, st, runs, cls, \
                     items, ws)
  if (pass == 0) {
    if (from_v) {
      if (diag) CHX_ERC(0, true, true);
      else CHX_ERC(0, false, true);
    } else {
      if (diag) CHX_ERC(0, true, false);
      else CHX_ERC(0, false, false);
    }
  } else if (pass == 1) CHX_ERC(1, false, false);
  else if (pass == 2) CHX_ERC(2, false, false);
  else CHX_ERC(3, false, false);
#undef CHX_ERC
  return hipGetLastError();
}

hipError_t launch_ens_rstep_final(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                  int nitems, const int* big, int nbig, unsigned char* ws,
                                  double* diag_out, long diag_stride, int index, hipStream_t st) {
  if (diag_out) {
    hipLaunchKernelGGL((ens_rstep_final<true>), dim3(nitems), dim3(256), 0, st, runs, cls, items,
                       ws);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ens_diag_final(runs, cls, big, nbig, ws, diag_out, diag_stride, index, st);
  }
  hipLaunchKernelGGL((ens_rstep_final<false>), dim3(nitems), dim3(256), 0, st, runs, cls, items,
                     ws);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
int rstep_segments(int nx) { return (nx + kSegR - 1) / kSegR; }
long rstep_parts(int nx, int ny) { return (long)rstep_segments(nx) * (ny / M); }

static dim3 rstep_grid(int nx, int ny) {
  const long pairs = (long)((nx + kSegR - 1) / kSegR) * (ny / M);
  return dim3((unsigned)((pairs + 3) / 4));
}

hipError_t launch_rstep_first(const double* c, long ld, double* rbuf, float* y32, float* rho,
                              int nx, int ny, const DevChunk& cy, const ChCoef& K, double* part,
                              hipStream_t st, const float* const* vprev, int nbprev) {
  if (nx % kSegR != 0 || ny % M != 0 || cy.S * M != ny || nbprev < 0 || nbprev > 4) return hipErrorInvalidValue;
  BandT<float> bd;
  for (int k = 0; k < 5; ++k) bd.c[k] = (float)cy.coef[k];
  const int nseg = (nx + kSegR - 1) / kSegR;
  RBufs B{};
  for (int b = 0; b < nbprev; ++b) B.v[b] = vprev[b];
#define CHX_RFIRST(D_, NB_)                                                                     \
  hipLaunchKernelGGL((rstep_first<D_, NB_>), rstep_grid(nx, ny), dim3(256), 0, st, c, ld, rbuf, \
                     y32, rho, nx, ny, nseg, cy.rec32, bd, K, part, B, cy.S, cy.rec)
  const bool d = part != nullptr;
  switch (nbprev) {
    case 0: if (d) CHX_RFIRST(true, 0); else CHX_RFIRST(false, 0); break;
    case 2: if (d) CHX_RFIRST(true, 2); else CHX_RFIRST(false, 2); break;
    case 3: if (d) CHX_RFIRST(true, 3); else CHX_RFIRST(false, 3); break;
    case 4: if (d) CHX_RFIRST(true, 4); else CHX_RFIRST(false, 4); break;
    default: return hipErrorInvalidValue;  // a refined step leaves 2 .. 4 solutions
  }
#undef CHX_RFIRST
  return hipGetLastError();
}

hipError_t launch_rstep_resid(const double* rbuf, const float* const* v, int nb, float* y32,
                              float* rho, int nx, int ny, const DevChunk& cy, const double* cx5,
                              const double* cy5, hipStream_t st) {
  if (nx % kSegR != 0 || ny % M != 0 || cy.S * M != ny || nb < 1 || nb > 3) return hipErrorInvalidValue;
  BandT<float> bd;
  BandT<double> ax, ay;
  for (int k = 0; k < 5; ++k) {
    bd.c[k] = (float)cy.coef[k];
    ax.c[k] = cx5[k];
    ay.c[k] = cy5[k];
  }
  RBufs B{};
  for (int b = 0; b < nb; ++b) B.v[b] = v[b];
  const int nseg = (nx + kSegR - 1) / kSegR;
#define CHX_RRES(NB_)                                                                           \
  hipLaunchKernelGGL((rstep_resid<NB_>), rstep_grid(nx, ny), dim3(256), 0, st, rbuf, B, y32, rho, \
                     nx, ny, nseg, cy.S, cy.rec, cy.rec32, bd, ax, ay)
  if (nb == 1) CHX_RRES(1);
  else if (nb == 2) CHX_RRES(2);
  else CHX_RRES(3);
#undef CHX_RRES
  return hipGetLastError();
}

hipError_t launch_rstep_final(const float* const* v, int nb, double* c, long ld, int nx, int ny,
                              const DevChunk& cy, const ChCoef& K, double* part, double* diag_out,
                              hipStream_t st) {
  if (nx % kSegR != 0 || ny % M != 0 || cy.S * M != ny || nb < 1 || nb > 4) return hipErrorInvalidValue;
  RBufs B{};
  for (int b = 0; b < nb; ++b) B.v[b] = v[b];
  const int nseg = (nx + kSegR - 1) / kSegR;
#define CHX_RFIN(NB_, D_)                                                                         \
  hipLaunchKernelGGL((rstep_final<NB_, D_>), rstep_grid(nx, ny), dim3(256), 0, st, B, c, ld, nx, \
                     ny, nseg, cy.S, cy.rec, K, part)
  if (diag_out) {
    if (nb == 1) CHX_RFIN(1, true);
    else if (nb == 2) CHX_RFIN(2, true);
    else if (nb == 3) CHX_RFIN(3, true);
    else CHX_RFIN(4, true);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ch_diag_final(part, rstep_parts(nx, ny), K.dxdy, diag_out, st);
  }
  if (nb == 1) CHX_RFIN(1, false);
  else if (nb == 2) CHX_RFIN(2, false);
  else if (nb == 3) CHX_RFIN(3, false);
  else CHX_RFIN(4, false);
#undef CHX_RFIN
  return hipGetLastError();
}

}  // namespace chx
