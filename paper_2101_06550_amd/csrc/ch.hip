// ch.hip -- Cahn-Hilliard ADI step kernels (thesis Ch.2 eq. 2:ch, Ch.3
// eq. 3:ch_adi; first-order splitting with the 1D operator of Ch.6
// eq. 6:1Dnumerical in each direction).
//
// One step is  r = c + D dt Lap5(c^3 - c) - 2 D gamma dt d2x d2y c,
//              (I + sx Px)(I + sy Py) c_new = r.
// The two factors commute, so the step runs the column (y) solves first and
// the row (x) solves second:
//   ch_column_pass   reads the state, forms r on the fly (rolling 3-row window
//                    in registers, x-neighbours by DPP lane shifts), sweeps the
//                    interior of each 32-row chunk of every column in registers,
//                    writes the chunk-local solution y and the separator parts,
//                    and (optionally) per-block mass / free-energy partial sums.
//   reduced_il       (solve.hip) writes the separator unknowns into the
//                    separator rows of the same buffer.
//   row_solve_lds    (solve.hip) solves every row of that buffer completely.
// The column-chunk correction x = y - Zl s_prev - Zr s_own mixes rows only and
// the row solve mixes columns only, so the correction is applied AFTER the row
// solve, by the next step's column pass while it reads the state (or by
// the final pass ch_column_final after the last step).  Separator rows then hold the row-solved
// separator values T, and the state is X(j) = V(j) - Zl T_prev - Zr T_own.
#include <hip/hip_runtime.h>

#include "ch_launch.hpp"
#include "common.hpp"
#include "ens.hpp"

namespace chx {

namespace {

constexpr int M = kChunk;
constexpr int P = 2;
constexpr int MI = M - P;

// Wave-level fixed-order butterfly sum (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block (256 threads) fixed-order sum of two values; result valid in thread 0.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wave * 2] = a;
    sh[wave * 2 + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sh[0] + sh[2] + sh[4] + sh[6];
    b = sh[1] + sh[3] + sh[5] + sh[7];
  }
}

// State value at row-position p (0..M-1) of a chunk for one column, given V
// at that row and the separator rows (row-solved values T) of the previous
// chunk (tp) and of the chunk itself (to).  Separator rows are the state.
template <bool RECON, int MM = kChunk, typename RecP>
__device__ __forceinline__ double recon_value(double v, int p, RecP __restrict__ rec,
                                              const double (&tp)[P], const double (&to)[P]) {
  constexpr int MMI = MM - P;
  if (!RECON || p >= MMI) return v;
  double x = v;
#pragma unroll
  for (int a = 0; a < P; ++a) x = x - rec[p * 8 + 4 + a] * tp[a] - rec[p * 8 + 6 + a] * to[a];
  return x;
}

}  // namespace

// Block = 4 waves = 4 adjacent 64-column segments (256 columns) of one
// 32-row chunk; every load is a full, aligned 512-byte row segment.  The
// x-neighbours come from the DPP lane shifts inside a wave; across waves the
// lane-0 and lane-63 state values are exchanged through LDS (one barrier),
// and the two columns just outside the block are loaded and reconstructed by
// 68 threads of the block before the barrier.
template <bool RECON, int MM = kChunk, typename RecP>
__device__ __forceinline__ double recon_row(double v, int q, RecP __restrict__ rec,
                                            const double (&tp)[P], const double (&to)[P],
                                            const double (&tn)[P]) {
  // q = 0: last row of chunk kc-1 (separator); q = 1..MM: own row q-1;
  // q = MM+1: row 0 of chunk kc+1
  if (q == 0) return v;
  if (q == MM + 1) return recon_value<RECON, MM>(v, 0, rec, to, tn);
  return recon_value<RECON, MM>(v, q - 1, rec, tp, to);
}

// Cahn-Hilliard-Cook forcing (Ch.7): q = dt eta, eta = amp div rho with
// amp = sqrt(sigma / (dx dy dt)), rho = (rho_x, rho_y) N(0,1) per point and
// step by Box-Muller from two counter-based SplitMix64 uniforms (Steele, Lea
// and Flood 2014; output k of the sequence whose state starts at mix(seed),
// u = ((out >> 11) + 1/2) 2^-53, k = ((step ny + j) nx + i) 2 + component),
// forward-difference divergence.  The kernels that add it draw rho where
// they form the right-hand side (no increment field in memory).
// One N(0,1) pair (rho_x, rho_y) of point (i, j) at step `step`.
__device__ __forceinline__ void cook_pair(unsigned long long seed_state, unsigned long long step,
                                          int j, int i, int nx, int ny, double& rx, double& ry) {
  const unsigned long long k =
      ((step * (unsigned long long)ny + (unsigned long long)j) * (unsigned long long)nx +
       (unsigned long long)i) * 2ULL;
  const unsigned long long z1 = chx_sm_mix(seed_state + (k + 1) * 0x9E3779B97F4A7C15ULL);
  const unsigned long long z2 = chx_sm_mix(seed_state + (k + 2) * 0x9E3779B97F4A7C15ULL);
  const double u1 = ((double)(z1 >> 11) + 0.5) * 0x1.0p-53;
  const double u2 = ((double)(z2 >> 11) + 0.5) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);  // sin, cos of 2 pi u2 without a general range reduction
  rx = rad * cs;
  ry = rad * sn;
}

// Body shared by the single-field kernel and the ensemble kernel: column
// block cb (256 columns), chunk kc; slot = where this block's (mass, energy)
// partial goes (DIAG only); NOISE adds the Cahn-Hilliard-Cook increment of
// step nz.step0, drawn here: each thread carries its column's pair down the
// rows and takes the right neighbour's rho_x from the next lane (the wave's
// last lane from LDS, drawn before the barrier).
// FINAL: the pass after the last step of a call: the state is reconstructed
// as it is read (RECON), its mass and free energy summed (DIAG), and the
// state itself written to ybuf (the caller's array) -- no right-hand side, no
// sweep; one streaming pass instead of a correction pass and a separate
// diagnostics pass over the result.
template <bool RECON, bool DIAG, bool NOISE = false, bool FINAL = false, int MM = kChunk,
          bool LOADS_FIRST = false, typename RecP = const double*, typename SrcP = const double*>
__device__ __forceinline__ void column_pass_body(SrcP __restrict__ src, long lds,
                                                 double* __restrict__ ybuf, long ldy, int nx,
                                                 int ny, int Sc, RecP __restrict__ rec,
                                                 const BandT<double>& bd, double* __restrict__ rho,
                                                 const ChCoef& K, double* __restrict__ slot,
                                                 int cb, int kc, const SmallNoise& nz = {}) {
  constexpr int MMI = MM - P;
  __shared__ double red[8];
  __shared__ double edge[10][MM + 2];  // 0: outer left, 1: outer right, 2+w: lane 0, 6+w: lane 63
  __shared__ double nedge[NOISE ? 4 : 1][MM];  // rho_x right of wave w's last lane
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nseg = nx >> 6;
  const int seg0 = cb * 4;
  const int nw = (nseg - seg0 < 4) ? nseg - seg0 : 4;  // active waves of this block
  const bool live = wave < nw;
  const int i = (seg0 + wave) * 64 + lane;
  const int kcm = (kc - 1 + Sc) % Sc, kcp = (kc + 1) % Sc;
  const long rowm1 = ((long)kc * MM - 1 + ny) % ny;
  const long rowp = ((long)kc * MM + MM) % ny;

  double tp[P] = {0, 0}, to[P] = {0, 0}, tn[P] = {0, 0};
  double X[MM + 2];
  // the column's own rows (and, RECON, the separator rows of the chunk and
  // its neighbours); LOADS_FIRST issues them before the two outer columns'
  // loads, so that the waves which also load those do not wait for them
  // first (measured: the ensemble's passes over 128^2-512^2 runs 2.5 %
  // faster, the 8192^2 pass 1 % slower)
  auto load_own = [&]() {
    if (live) {
      if (RECON) {
#pragma unroll
        for (int a = 0; a < P; ++a) {
          tp[a] = src[((long)kcm * MM + MMI + a) * lds + i];
          to[a] = src[((long)kc * MM + MMI + a) * lds + i];
          tn[a] = src[((long)kcp * MM + MMI + a) * lds + i];
        }
      }
      X[0] = src[rowm1 * lds + i];
#pragma unroll
      for (int p = 0; p < MM; ++p) X[p + 1] = src[((long)kc * MM + p) * lds + i];
      X[MM + 1] = src[rowp * lds + i];
    }
  };
  if constexpr (LOADS_FIRST) load_own();

  // the two columns outside the block: thread t < 2(MM+2) takes side t/(MM+2), row t%(MM+2)
  if (threadIdx.x < 2 * (MM + 2)) {
    const int side = threadIdx.x / (MM + 2), q = threadIdx.x - side * (MM + 2);
    const int ic = side == 0 ? (seg0 * 64 - 1 + nx) % nx : (seg0 * 64 + nw * 64) % nx;
    const long row = q == 0 ? rowm1 : (q == MM + 1 ? rowp : (long)kc * MM + q - 1);
    double v = src[row * lds + ic];
    if (RECON) {
      double tp[P], to[P], tn[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        tp[a] = src[((long)kcm * MM + MMI + a) * lds + ic];
        to[a] = src[((long)kc * MM + MMI + a) * lds + ic];
        tn[a] = src[((long)kcp * MM + MMI + a) * lds + ic];
      }
      v = recon_row<RECON, MM>(v, q, rec, tp, to, tn);
    }
    edge[side][q] = v;
  }
  if (NOISE && (int)threadIdx.x < nw * MM) {
    const int w = threadIdx.x / MM, p = threadIdx.x - w * MM;
    double rx, ry;
    cook_pair(nz.seed_state, nz.step0, kc * MM + p, ((seg0 + w + 1) * 64) % nx, nx, ny, rx, ry);
    nedge[w][p] = rx;
  }

  if constexpr (!LOADS_FIRST) load_own();
  if (live) {
    // (left to the compiler, these sums sink into the row loop and the
    // correction table spills through VGPR lanes; computing each where its
    // load completes removes the spills and a sixth of the vector
    // instructions but waits for every load before the first row, and
    // measured 2-3 % slower)
#pragma unroll
    for (int q = 0; q < MM + 2; ++q) X[q] = recon_row<RECON, MM>(X[q], q, rec, tp, to, tn);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < MM + 2; ++q) edge[2 + wave][q] = X[q];
    } else if (lane == 63) {
#pragma unroll
      for (int q = 0; q < MM + 2; ++q) edge[6 + wave][q] = X[q];
    }
  }
  __syncthreads();

  double msum = 0.0, esum = 0.0;
  if (live) {
    // the neighbour slot this lane reads: lane 0 <- left, lane 63 <- right
    const int slot = (lane == 0) ? (wave > 0 ? 6 + wave - 1 : 0)
                                 : (wave < nw - 1 ? 2 + wave + 1 : 1);
    const double* es = &edge[slot][0];
    // Rows are processed strictly in order: an empty volatile asm on the next
    // row's value (volatile asms keep their order) and on each row's result
    // stop the compiler from computing every row's neighbours up front.
    double f[MM];
    const double eps = bd.c[0];
    double xc_m = X[0];
    double xl_m = dpp_from_left(xc_m, es[0]), xr_m = dpp_from_right(xc_m, es[0]);
    double xc_c = X[1];
    double xl_c = dpp_from_left(xc_c, es[1]), xr_c = dpp_from_right(xc_c, es[1]);
    double nrx = 0.0, nry = 0.0;  // this column's forcing pair at the current row
    if (NOISE) cook_pair(nz.seed_state, nz.step0, kc * MM, i, nx, ny, nrx, nry);
#pragma unroll
    for (int p = 0; p < MM; ++p) {
      double xc_p = X[p + 2];
      double en = es[p + 2];
      asm volatile("" : "+v"(xc_p), "+v"(en));
      const double xl_p = dpp_from_left(xc_p, en);
      const double xr_p = dpp_from_right(xc_p, en);
      const double mu_c = xc_c * xc_c * xc_c - xc_c;
      const double mu_l = xl_c * xl_c * xl_c - xl_c;
      const double mu_r = xr_c * xr_c * xr_c - xr_c;
      const double mu_s = xc_m * xc_m * xc_m - xc_m;
      const double mu_n = xc_p * xc_p * xc_p - xc_p;
      const double lap = K.cx * (mu_r + mu_l - 2.0 * mu_c) + K.cy * (mu_n + mu_s - 2.0 * mu_c);
      const double dyy_w = xl_p + xl_m - 2.0 * xl_c;
      const double dyy_c = xc_p + xc_m - 2.0 * xc_c;
      const double dyy_e = xr_p + xr_m - 2.0 * xr_c;
      double r = xc_c + lap - K.ccross * (dyy_e + dyy_w - 2.0 * dyy_c);
      if (NOISE && !FINAL) {
        const int j = kc * MM + p, jn = (j + 1 == ny) ? 0 : j + 1;
        double rx_n, ry_n;
        cook_pair(nz.seed_state, nz.step0, jn, i, nx, ny, rx_n, ry_n);
        const double rx_e = dpp_from_right(nrx, nedge[wave][p]);
        const double div = (rx_e - nrx) * nz.inv_dx + (ry_n - nry) * nz.inv_dy;
        r = r + nz.scale * div;
        nrx = rx_n;
        nry = ry_n;
      }
      if (DIAG) {
        const double w = xc_c * xc_c - 1.0;
        const double gx = (xr_c - xc_c) * K.inv_dx, gy = (xc_p - xc_c) * K.inv_dy;
        msum += xc_c;
        esum += 0.25 * w * w + K.half_gamma * (gx * gx + gy * gy);
      }
      if (FINAL) {
        __builtin_nontemporal_store(xc_c, &ybuf[((long)kc * MM + p) * ldy + i]);
        if (DIAG) asm volatile("" : "+v"(msum), "+v"(esum));
      } else {
        if (p < MMI) {  // forward sweep step of the chunk interior (g overwrites f)
          if (p >= 2) r = r - eps * f[p - 2];
          if (p >= 1) r = r - rec[p * 8 + 1] * f[p - 1];
          r = r * rec[p * 8 + 0];
        }
        if (DIAG) asm volatile("" : "+v"(r), "+v"(msum), "+v"(esum));
        else asm volatile("" : "+v"(r));
        f[p] = r;
      }
      xl_m = xl_c; xc_m = xc_c; xr_m = xr_c;
      xl_c = xl_p; xc_c = xc_p; xr_c = xr_p;
    }
    if (!FINAL) {
      // back sweep of the interior (y = R^{-1} g)
#pragma unroll
      for (int p = MMI - 1; p >= 0; --p) {
        double v = f[p];
        if (p + 2 < MMI) v = v - rec[p * 8 + 3] * f[p + 2];
        if (p + 1 < MMI) v = v - rec[p * 8 + 2] * f[p + 1];
        f[p] = v;
      }
      double pa[P], pb[P];
      chunk_parts<P, MM, double>(f, bd, pa, pb);
      // streamed stores (non-temporal): the row pass reads y back from HBM; on
      // gfx950 this keeps the stores out of the way of the loads (measured:
      // both passes faster than with ordinary stores, the loads stay ordinary)
#pragma unroll
      for (int p = 0; p < MMI; ++p)
        __builtin_nontemporal_store(f[p], &ybuf[((long)kc * MM + p) * ldy + i]);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        rho[((long)kc * 2 * P + a) * nx + i] = pa[a];
        rho[((long)kc * 2 * P + P + a) * nx + i] = pb[a];
      }
    }
  }
  if (DIAG) {
    block_sum2(msum, esum, red);
    if (threadIdx.x == 0) {
      slot[0] = msum;
      slot[1] = esum;
    }
  }
}

// Tile (column block cb, chunk kc) of launch block b (1D grid of ncb * Sc
// blocks).  Consecutive blocks go to the 8 XCDs round robin, so the blocks of
// XCD g are b = g, g + 8, ...; orders 1 and 2 number them so that each XCD
// works one contiguous range of tiles: order 1 in chunk-row order (an XCD
// holds a horizontal band of chunk rows), order 2 chunk-fastest down column
// blocks (an XCD holds whole columns).  Order 0: plain row-major tile order.
// A tile's diagnostics slot is its tile number, so every order sums the same
// partials in the same order.
__device__ __forceinline__ void column_tile(int order, long b, int ncb, int Sc, int& cb, int& kc) {
  long t = b;
  if (order != 0) {
    const long T = (long)ncb * Sc, base = T >> 3, rem = T & 7;
    const long g = b & 7, q = b >> 3;
    t = g * base + (g < rem ? g : rem) + q;
  }
  if (order == 2) {
    cb = (int)(t / Sc);
    kc = (int)(t - (long)cb * Sc);
  } else {
    kc = (int)(t / ncb);
    cb = (int)(t - (long)kc * ncb);
  }
}

template <bool RECON, bool DIAG, bool NOISE, int MM>
__global__ __launch_bounds__(256) void ch_column_pass(const double* __restrict__ src, long lds,
                                                      double* __restrict__ ybuf, long ldy, int nx,
                                                      int ny, int Sc,
                                                      const double* __restrict__ rec,
                                                      BandT<double> bd, double* __restrict__ rho,
                                                      ChCoef K, double* __restrict__ part,
                                                      SmallNoise nz, int ncb, int order) {
  int cb, kc;
  column_tile(order, blockIdx.x, ncb, Sc, cb, kc);
  const long slot = (long)kc * ncb + cb;
  column_pass_body<RECON, DIAG, NOISE, false, MM>(src, lds, ybuf, ldy, nx, ny, Sc, rec, bd, rho, K,
                                                  DIAG ? part + 2 * slot : nullptr, cb, kc, nz);
}

// The pass after the last step: reconstruct the state, write it to dst and
// (DIAG) leave one (mass, energy) partial per block in part.
template <bool DIAG, int MM>
__global__ __launch_bounds__(256) void ch_column_final(const double* __restrict__ src, long lds,
                                                       double* __restrict__ dst, long ldd, int nx,
                                                       int ny, int Sc,
                                                       const double* __restrict__ rec,
                                                       ChCoef K, double* __restrict__ part,
                                                       int ncb, int order) {
  int cb, kc;
  column_tile(order, blockIdx.x, ncb, Sc, cb, kc);
  const long slot = (long)kc * ncb + cb;
  const BandT<double> bd{};
  column_pass_body<true, DIAG, false, true, MM>(src, lds, dst, ldd, nx, ny, Sc, rec, bd, nullptr,
                                                K, DIAG ? part + 2 * slot : nullptr, cb, kc);
}

// ---------------------------------------------------------------------------

// Mass and free-energy partial sums of a plain field, one per block of
// 64 columns x 16 rows (fixed order within the block).
__device__ __forceinline__ void diag_partial_body(const double* __restrict__ c, long ld, int nx,
                                                  int ny, const ChCoef& K,
                                                  double* __restrict__ slot, int bx, int by) {
  __shared__ double red[8];
  const int i = bx * 64 + (threadIdx.x & 63);
  const int j0 = by * 16 + (threadIdx.x >> 6) * 4;
  double ms = 0.0, es = 0.0;
  if (i < nx) {
    const int ip = (i + 1) % nx;
    for (int u = 0; u < 4; ++u) {
      const int j = j0 + u;
      if (j >= ny) break;
      const int jp = (j + 1) % ny;
      const double x = c[(long)j * ld + i];
      const double gx = (c[(long)j * ld + ip] - x) * K.inv_dx;
      const double gy = (c[(long)jp * ld + i] - x) * K.inv_dy;
      const double w = x * x - 1.0;
      ms += x;
      es += 0.25 * w * w + K.half_gamma * (gx * gx + gy * gy);
    }
  }
  block_sum2(ms, es, red);
  if (threadIdx.x == 0) {
    slot[0] = ms;
    slot[1] = es;
  }
}

__global__ __launch_bounds__(256) void ch_diag_partial(const double* __restrict__ c, long ld,
                                                       int nx, int ny, ChCoef K,
                                                       double* __restrict__ part) {
  const long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
  diag_partial_body(c, ld, nx, ny, K, part + 2 * b, blockIdx.x, blockIdx.y);
}

// Fixed-order final sum of nparts (mass, energy) pairs, scaled by dx dy.
// Each thread owns a contiguous slice and issues 8 independent loads per
// round; the partial sums are then combined by a fixed tree.
__device__ __forceinline__ void diag_final_body(const double* __restrict__ part, long nparts,
                                                double scale, double* __restrict__ out) {
  __shared__ double sm[256], se[256];
  const long per = (nparts + 255) / 256;
  const long b0 = (long)threadIdx.x * per, b1 = (b0 + per < nparts) ? b0 + per : nparts;
  double m = 0.0, e = 0.0;
  long b = b0;
  for (; b + 8 <= b1; b += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = reinterpret_cast<const double2*>(part)[b + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      m += v[u].x;
      e += v[u].y;
    }
  }
  for (; b < b1; ++b) {
    m += part[2 * b];
    e += part[2 * b + 1];
  }
  sm[threadIdx.x] = m;
  se[threadIdx.x] = e;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sm[threadIdx.x] += sm[threadIdx.x + h];
      se[threadIdx.x] += se[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sm[0] * scale;
    out[1] = se[0] * scale;
  }
}

__global__ __launch_bounds__(256) void ch_diag_final(const double* __restrict__ part, long nparts,
                                                     double scale, double* __restrict__ out) {
  diag_final_body(part, nparts, scale, out);
}

// Plain RHS kernel for grids the fused path does not cover.
__global__ __launch_bounds__(256) void ch_rhs_plain(const double* __restrict__ c, long ld,
                                                    double* __restrict__ r, long ldr, int nx,
                                                    int ny, ChCoef K) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  const int im = (i - 1 + nx) % nx, ip = (i + 1) % nx;
  const int jm = (j - 1 + ny) % ny, jp = (j + 1) % ny;
  auto at = [&](int jj, int ii) { return c[(long)jj * ld + ii]; };
  const double xc = at(j, i), xl = at(j, im), xr = at(j, ip), xs = at(jm, i), xn = at(jp, i);
  const double mu_c = xc * xc * xc - xc, mu_l = xl * xl * xl - xl, mu_r = xr * xr * xr - xr;
  const double mu_s = xs * xs * xs - xs, mu_n = xn * xn * xn - xn;
  const double lap = K.cx * (mu_r + mu_l - 2.0 * mu_c) + K.cy * (mu_n + mu_s - 2.0 * mu_c);
  const double dyy_w = at(jp, im) + at(jm, im) - 2.0 * xl;
  const double dyy_c = xn + xs - 2.0 * xc;
  const double dyy_e = at(jp, ip) + at(jm, ip) - 2.0 * xr;
  r[(long)j * ldr + i] = xc + lap - K.ccross * (dyy_e + dyy_w - 2.0 * dyy_c);
}

// Residual of the implicit operator, R = r - (I + sx Px)(I + sy Py) c, in
// FP64 (the refinement step of the FP32-sweep path); one thread per point.
__global__ __launch_bounds__(256) void ch_residual2d(const double* __restrict__ r, long ldr,
                                                     const double* __restrict__ c, long ldc,
                                                     double* __restrict__ R, long ldR, int nx,
                                                     int ny, BandT<double> bx, BandT<double> by) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  int ii[5];
#pragma unroll
  for (int p = 0; p < 5; ++p) ii[p] = ((i + p - 2) % nx + nx) % nx;
  double acc = r[(long)j * ldr + i];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const long jj = ((j + q - 2) % ny + ny) % ny;
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < 5; ++p) t += bx.c[p] * c[jj * ldc + ii[p]];
    acc -= by.c[q] * t;
  }
  R[(long)j * ldR + i] = acc;
}

hipError_t launch_ch_residual2d(const double* r, long ldr, const double* c, long ldc, double* R,
                                long ldR, int nx, int ny, const double* cx, const double* cy,
                                hipStream_t st) {
  BandT<double> bx, by;
  for (int k = 0; k < 5; ++k) {
    bx.c[k] = cx[k];
    by.c[k] = cy[k];
  }
  dim3 grid((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(ch_residual2d, grid, dim3(256), 0, st, r, ldr, c, ldc, R, ldR, nx, ny, bx, by);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_ch_column_pass(bool recon, bool diag, const double* src, long lds,
                                 double* ybuf, long ldy, int nx, int ny, const DevChunk& cy,
                                 double* rho, const ChCoef& K, double* part, hipStream_t st,
                                 const SmallNoise* nz, int order) {
  BandT<double> bd;
  for (int k = 0; k < 5; ++k) bd.c[k] = cy.coef[k];
  const int ncb = ((nx >> 6) + 3) / 4;
  const int Sc = cy.S;
  dim3 grid((unsigned)((long)ncb * Sc));
  const SmallNoise z = nz ? *nz : SmallNoise{};
#define CHX_COLPASS(R, D, N)                                                                    \
  do {                                                                                          \
    if (cy.M == 16)                                                                             \
      hipLaunchKernelGGL((ch_column_pass<R, D, N, 16>), grid, dim3(256), 0, st, src, lds, ybuf, \
                         ldy, nx, ny, Sc, cy.rec, bd, rho, K, part, z, ncb, order);             \
    else                                                                                        \
      hipLaunchKernelGGL((ch_column_pass<R, D, N, kChunk>), grid, dim3(256), 0, st, src, lds,   \
                         ybuf, ldy, nx, ny, Sc, cy.rec, bd, rho, K, part, z, ncb, order);       \
  } while (0)
  if (nz) {
    if (recon && diag) CHX_COLPASS(true, true, true);
    else if (recon) CHX_COLPASS(true, false, true);
    else if (diag) CHX_COLPASS(false, true, true);
    else CHX_COLPASS(false, false, true);
  } else {
    if (recon && diag) CHX_COLPASS(true, true, false);
    else if (recon) CHX_COLPASS(true, false, false);
    else if (diag) CHX_COLPASS(false, true, false);
    else CHX_COLPASS(false, false, false);
  }
#undef CHX_COLPASS
  return hipGetLastError();
}

long ch_column_pass_blocks(int nx, int Sc) { return (long)(((nx >> 6) + 3) / 4) * Sc; }


hipError_t launch_ch_column_final(const double* src, long lds, double* dst, long ldd, int nx,
                                  int ny, const DevChunk& cy, const ChCoef& K, double* part,
                                  double* diag_out, hipStream_t st, int order) {
  const int ncb = ((nx >> 6) + 3) / 4;
  dim3 grid((unsigned)((long)ncb * cy.S));
#define CHX_COLFIN(D, MM_)                                                                       \
  hipLaunchKernelGGL((ch_column_final<D, MM_>), grid, dim3(256), 0, st, src, lds, dst, ldd, nx, ny, \
                     cy.S, cy.rec, K, part, ncb, order)
  if (diag_out) {
    if (cy.M == 16) CHX_COLFIN(true, 16);
    else CHX_COLFIN(true, kChunk);
    hipLaunchKernelGGL(ch_diag_final, dim3(1), dim3(256), 0, st, part, (long)grid.x, K.dxdy,
                       diag_out);
  } else {
    if (cy.M == 16) CHX_COLFIN(false, 16);
    else CHX_COLFIN(false, kChunk);
  }
#undef CHX_COLFIN
  return hipGetLastError();
}

long ch_diag_partial_blocks(int nx, int ny) { return (long)((nx + 63) / 64) * ((ny + 15) / 16); }

hipError_t launch_ch_diag(const double* c, long ld, int nx, int ny, const ChCoef& K, double* part,
                          double* out, hipStream_t st) {
  dim3 grid((nx + 63) / 64, (ny + 15) / 16);
  hipLaunchKernelGGL(ch_diag_partial, grid, dim3(256), 0, st, c, ld, nx, ny, K, part);
  hipLaunchKernelGGL(ch_diag_final, dim3(1), dim3(256), 0, st, part,
                     (long)grid.x * grid.y, K.dxdy, out);
  return hipGetLastError();
}

// Ch.3 "Numerical Results": Simpson averages <C>, <C^2> on the periodic grid
// (weights 2/3 on even, 4/3 on odd indices in each direction); one (sum w c,
// sum w c^2) pair per 64 x 16 block, summed in fixed order by ch_diag_final.
__global__ __launch_bounds__(256) void ch_simpson_partial(const double* __restrict__ c, long ld,
                                                          int nx, int ny,
                                                          double* __restrict__ part) {
  __shared__ double red[8];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double s1 = 0.0, s2 = 0.0;
  if (i < nx) {
    const double wi = (i & 1) ? 4.0 / 3.0 : 2.0 / 3.0;
    for (int r = 0; r < 16; r += 4) {
      const int j = blockIdx.y * 16 + r + wave;
      if (j >= ny) break;
      const double w = wi * ((j & 1) ? 4.0 / 3.0 : 2.0 / 3.0);
      const double v = c[(long)j * ld + i];
      s1 += w * v;
      s2 += w * v * v;
    }
  }
  block_sum2(s1, s2, red);
  if (threadIdx.x == 0) {
    const long b = (long)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = s1;
    part[2 * b + 1] = s2;
  }
}

hipError_t launch_ch_simpson(const double* c, long ld, int nx, int ny, double* part, double* out,
                             hipStream_t st) {
  dim3 grid((nx + 63) / 64, (ny + 15) / 16);
  hipLaunchKernelGGL(ch_simpson_partial, grid, dim3(256), 0, st, c, ld, nx, ny, part);
  hipLaunchKernelGGL(ch_diag_final, dim3(1), dim3(256), 0, st, part, (long)grid.x * grid.y,
                     1.0 / ((double)nx * ny), out);
  return hipGetLastError();
}

// Ch.3 "Numerical Results": k1 = sum |C^|^2 / sum |k|^-1 |C^|^2 from the
// half spectrum of a real-to-complex transform (ny rows of nx/2 + 1 values;
// columns 0 and nx/2 count once, the others twice for their conjugates),
// k = (2 pi m / lx, 2 pi l / ly), k = 0 left out.  One (sum, weighted sum)
// pair per block of 256 values, summed in fixed order by ch_diag_final.
__global__ __launch_bounds__(256) void ch_k1_partial(const double2* __restrict__ spec, int nx,
                                                     int ny, double kx0, double ky0,
                                                     double* __restrict__ part) {
  __shared__ double red[8];
  const int nh = nx / 2 + 1;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  double s1 = 0.0, s2 = 0.0;
  if (e < (long)nh * ny) {
    const int l = (int)(e / nh), m = (int)(e - (long)l * nh);
    if (l != 0 || m != 0) {
      const double2 v = spec[e];
      const double w = (m == 0 || 2 * m == nx) ? 1.0 : 2.0;
      const int ls = (2 * l <= ny) ? l : l - ny;
      const double kx = kx0 * m, ky = ky0 * ls;
      const double pw = w * (v.x * v.x + v.y * v.y);
      s1 = pw;
      s2 = pw / sqrt(kx * kx + ky * ky);
    }
  }
  block_sum2(s1, s2, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1;
    part[2 * blockIdx.x + 1] = s2;
  }
}

long ch_k1_blocks(int nx, int ny) { return ((long)(nx / 2 + 1) * ny + 255) / 256; }

hipError_t launch_ch_k1(const double2* spec, int nx, int ny, double lx, double ly, double* part,
                        double* out, hipStream_t st) {
  const long nb = ch_k1_blocks(nx, ny);
  const double two_pi = 6.283185307179586476925286766559;
  hipLaunchKernelGGL(ch_k1_partial, dim3((unsigned)nb), dim3(256), 0, st, spec, nx, ny,
                     two_pi / lx, two_pi / ly, part);
  hipLaunchKernelGGL(ch_diag_final, dim3(1), dim3(256), 0, st, part, nb, 1.0, out);
  return hipGetLastError();
}

// Ch.7 free-energy decay rate beta = -(t / F) dF/dt from the energies a
// stepping call wrote (diag: run r, state k at r * 2 nstates + 2 k + {0: mass,
// 1: energy}), t_k = t0 + k dt: second-order differences, central inside and
// three-point one-sided at the first and last state.  One thread per value.
__global__ __launch_bounds__(256) void ch_decay_rate(const double* __restrict__ diag, int nruns,
                                                     int nstates, double t0, double dt,
                                                     double* __restrict__ beta) {
  const long idx = (long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long)nruns * nstates) return;
  const long r = idx / nstates;
  const int k = (int)(idx - r * nstates);
  const double* F = diag + r * 2L * nstates + 1;  // energies at stride 2
  double dFdt;
  if (k == 0)
    dFdt = (-3.0 * F[0] + 4.0 * F[2] - F[4]) / (2.0 * dt);
  else if (k == nstates - 1)
    dFdt = (3.0 * F[2 * k] - 4.0 * F[2 * k - 2] + F[2 * k - 4]) / (2.0 * dt);
  else
    dFdt = (F[2 * k + 2] - F[2 * k - 2]) / (2.0 * dt);
  const double t = t0 + k * dt;
  beta[idx] = -(t / F[2 * k]) * dFdt;
}

hipError_t launch_ch_decay_rate(const double* diag, int nruns, int nstates, double t0, double dt,
                                double* beta, hipStream_t st) {
  const long n = (long)nruns * nstates;
  hipLaunchKernelGGL(ch_decay_rate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, diag,
                     nruns, nstates, t0, dt, beta);
  return hipGetLastError();
}

hipError_t launch_ch_diag_final(const double* part, long nparts, double scale, double* out,
                                hipStream_t st) {
  hipLaunchKernelGGL(ch_diag_final, dim3(1), dim3(256), 0, st, part, nparts, scale, out);
  return hipGetLastError();
}

hipError_t launch_ch_rhs_plain(const double* c, long ld, double* r, long ldr, int nx, int ny,
                               const ChCoef& K, hipStream_t st) {
  dim3 grid((nx + 63) / 64, (ny + 3) / 4);
  hipLaunchKernelGGL(ch_rhs_plain, grid, dim3(256), 0, st, c, ld, r, ldr, nx, ny, K);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The thesis's own scheme (Ch.3 eq. 3:ch_adi, delta form with 2/3 factors):
//   r = -2/3 (C - Cp) - a Lap^2 (2C - Cp) + b Lap (C^3 - C),  a = 2/3 D gamma dt,
//   b = 2/3 D dt;  v = (I + s' Px)^{-1} (I + s' Py)^{-1} r;  Cp <- C, C <- 2C - Cp + v.
// ch2_rhs stages a 16 x 64 tile with a 2-point halo of Cbar = 2C - Cp,
// mu = C^3 - C and d = C - Cp in LDS and evaluates the 13-point biharmonic and
// the 5-point Laplacian from there.
constexpr int kT2X = 64, kT2Y = 32, kT2H = 2;
constexpr int kT2T = 512;  // threads of a ch2_rhs block: 8 waves, 4 rows each
constexpr int kT2W = kT2X + 2 * kT2H, kT2R = kT2Y + 2 * kT2H;

// UPD: the state is first advanced from the previous step's solution,
// C_new = 2 C - Cp + v, at every staged point (C_new of the tile's own points
// is written to cnew), and the right-hand side is formed from (C_new, C).
// RECON: v is the solution with the column-chunk correction still to apply
// (chunk interiors uncorrected, separator rows final), corrected here as it
// is loaded: v = V - Zl T_prev - Zr T_own.
__device__ __forceinline__ double ch2_recon(const double* __restrict__ v, long ldv, int j, int i,
                                            int Sc, const double* __restrict__ rec) {
  const int kc = j / M, p = j - kc * M;
  double x = v[(long)j * ldv + i];
  if (p >= MI) return x;
  const int kp = (kc == 0) ? Sc - 1 : kc - 1;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    const double tp = v[((long)kp * M + MI + a) * ldv + i];
    const double to = v[((long)kc * M + MI + a) * ldv + i];
    x = x - rec[p * 8 + 4 + a] * tp - rec[p * 8 + 6 + a] * to;
  }
  return x;
}

// SWEEP: the tile is one 32-row column chunk, so the block also runs that
// chunk's column sweep: r goes to LDS (over the staged tile) instead of
// memory, one wave sweeps the 64 columns and writes the chunk interiors y
// into r and the separator parts into rho, as the interleaved chunk sweep
// would (same helpers, same arithmetic).
static_assert(kT2Y == M, "a fused column sweep needs one chunk per tile");
template <bool UPD, bool RECON, bool SWEEP>
__global__ __launch_bounds__(kT2T) void ch2_rhs(const double* __restrict__ c, long ld,
                                                const double* __restrict__ cp, long ldp,
                                                const double* __restrict__ v, long ldv,
                                                double* __restrict__ cnew, long ldn,
                                                double* __restrict__ r, long ldr, int nx, int ny,
                                                Ch2Coef K, int Sc, const double* __restrict__ rec,
                                                const double* __restrict__ srec, BandT<double> sbd,
                                                double* __restrict__ rhop) {
  __shared__ double cb[kT2R][kT2W];
  __shared__ double mu[kT2R][kT2W];
  // RECON: the separator rows of the chunks kb-2 .. kb+1 (kb = the chunk of
  // the tile's first row), which hold every correction the tile's rows need
  __shared__ double sep[RECON ? 4 : 1][P][kT2W];
  const int i0 = blockIdx.x * kT2X, j0 = blockIdx.y * kT2Y;
  const int kb = j0 / M;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  constexpr int kRows = kT2Y / (kT2T / 64);  // output rows per thread
  constexpr int kHalo = kT2R * kT2W - kT2Y * kT2X;
  constexpr int kItH = (kHalo + kT2T - 1) / kT2T;
  if (RECON) {
    for (int e = threadIdx.x; e < 4 * P * kT2W; e += kT2T) {
      const int sl = e / (P * kT2W), rem = e - sl * P * kT2W;
      const int a = rem / kT2W, tc = rem - a * kT2W;
      int kc = kb - 2 + sl;
      while (kc < 0) kc += Sc;
      while (kc >= Sc) kc -= Sc;
      int i = i0 - kT2H + tc;
      i += (i < 0) ? nx : 0;
      while (i >= nx) i -= nx;
      sep[sl][a][tc] = v[((long)kc * M + MI + a) * ldv + i];
    }
  }
  // staged points: first this thread's own output points (tile row
  // kT2H + ty + 8u, column kT2H + tx: aligned 64-wide rows), then the halo
  // ring; every load is issued before any is used
  auto halo_rc = [&](int e, int& tr, int& tc) {
    if (e < 2 * kT2H * kT2W) {  // the kT2H rows above and below, full width
      const int r4 = e / kT2W;
      tc = e - r4 * kT2W;
      tr = r4 < kT2H ? r4 : kT2Y + r4;
    } else {  // the kT2H columns left and right of the interior rows
      const int e2 = e - 2 * kT2H * kT2W;
      const int row = e2 / (2 * kT2H), c4 = e2 - row * (2 * kT2H);
      tr = kT2H + row;
      tc = c4 < kT2H ? c4 : kT2X + c4;
    }
  };
  auto wrapped = [&](int tr, int tc, int& j, int& i) {
    j = j0 - kT2H + tr;
    i = i0 - kT2H + tc;
    j += (j < 0) ? ny : 0;
    while (j >= ny) j -= ny;
    i += (i < 0) ? nx : 0;
    while (i >= nx) i -= nx;
  };
  double lc[kRows + kItH], lp[kRows + kItH], lv[kRows + kItH];
#pragma unroll
  for (int k = 0; k < kRows + kItH; ++k) {
    int tr, tc;
    bool ok = true;
    if (k < kRows) {
      tr = kT2H + ty + (kT2T / 64) * k;
      tc = kT2H + tx;
    } else {
      const int e = threadIdx.x + kT2T * (k - kRows);
      ok = e < kHalo;
      halo_rc(ok ? e : 0, tr, tc);
    }
    lc[k] = lp[k] = lv[k] = 0.0;
    if (ok) {
      int j, i;
      wrapped(tr, tc, j, i);
      lc[k] = c[(long)j * ld + i];
      lp[k] = cp[(long)j * ldp + i];
      if (UPD) lv[k] = v[(long)j * ldv + i];
    }
  }
  if (RECON) __syncthreads();  // sep
  double dfo[kRows];
#pragma unroll
  for (int k = 0; k < kRows + kItH; ++k) {
    int tr, tc;
    if (k < kRows) {
      tr = kT2H + ty + (kT2T / 64) * k;
      tc = kT2H + tx;
    } else {
      const int e = threadIdx.x + kT2T * (k - kRows);
      if (e >= kHalo) break;
      halo_rc(e, tr, tc);
    }
    const int ju = j0 - kT2H + tr, iu = i0 - kT2H + tc;  // unwrapped
    double vc = lc[k], vp = lp[k];
    if (UPD) {
      double vv = lv[k];
      if (RECON) {
        // chunk of the unwrapped row, relative to kb: -1, 0 or 1
        const int kcu = (ju + M) / M - 1;
        const int pp = ju - kcu * M;
        if (pp < MI) {
          const int so = kcu - kb + 2, sp = so - 1;
#pragma unroll
          for (int a = 0; a < P; ++a)
            vv = vv - rec[pp * 8 + 4 + a] * sep[sp][a][tc] - rec[pp * 8 + 6 + a] * sep[so][a][tc];
        }
      }
      const double vn = (2.0 * vc - vp) + vv;
      vp = vc;
      vc = vn;
      if (k < kRows && ju < ny && iu < nx)
        __builtin_nontemporal_store(vn, &cnew[(long)ju * ldn + iu]);
    }
    if (k < kRows) dfo[k] = vc - vp;
    cb[tr][tc] = 2.0 * vc - vp;
    mu[tr][tc] = vc * vc * vc - vc;
  }
  __syncthreads();
  const int i = i0 + tx;
  const int q = tx + kT2H;
  double rv[kRows];
#pragma unroll
  for (int u = 0; u < kRows; ++u) {
    const int j = j0 + ty + (kT2T / 64) * u;
    rv[u] = 0.0;
    if (i >= nx || j >= ny) continue;
    const int w = ty + (kT2T / 64) * u + kT2H;
    const double d4x = (cb[w][q - 2] - 4.0 * cb[w][q - 1] + 6.0 * cb[w][q] - 4.0 * cb[w][q + 1] +
                        cb[w][q + 2]) * K.inv_dx4;
    const double d4y = (cb[w - 2][q] - 4.0 * cb[w - 1][q] + 6.0 * cb[w][q] - 4.0 * cb[w + 1][q] +
                        cb[w + 2][q]) * K.inv_dy4;
    const double dyy_w = cb[w + 1][q - 1] + cb[w - 1][q - 1] - 2.0 * cb[w][q - 1];
    const double dyy_c = cb[w + 1][q] + cb[w - 1][q] - 2.0 * cb[w][q];
    const double dyy_e = cb[w + 1][q + 1] + cb[w - 1][q + 1] - 2.0 * cb[w][q + 1];
    const double dxxyy = (dyy_e + dyy_w - 2.0 * dyy_c) * K.inv_dx2dy2;
    const double bih = d4x + 2.0 * dxxyy + d4y;
    const double lap = (mu[w][q + 1] + mu[w][q - 1] - 2.0 * mu[w][q]) * K.inv_dx2 +
                       (mu[w + 1][q] + mu[w - 1][q] - 2.0 * mu[w][q]) * K.inv_dy2;
    rv[u] = -(2.0 / 3.0) * dfo[u] - K.a * bih + K.b * lap;
    if (!SWEEP) __builtin_nontemporal_store(rv[u], &r[(long)j * ldr + i]);
  }
  if (SWEEP) {
    __syncthreads();  // every read of the staged tile is done
    double* rt = &cb[0][0];  // r of the chunk: row p at rt[p * kT2W + column]
#pragma unroll
    for (int u = 0; u < kRows; ++u) rt[(ty + (kT2T / 64) * u) * kT2W + tx] = rv[u];
    __syncthreads();
    if (ty == 0 && i < nx) {
      double f[M];
#pragma unroll
      for (int p = 0; p < M; ++p) f[p] = rt[p * kT2W + tx];
      chunk_sweep<P, M, double>(f, srec, sbd.c[0]);
      double pa[P], pb[P];
      chunk_parts<P, M, double>(f, sbd, pa, pb);
#pragma unroll
      for (int p = 0; p < MI; ++p) __builtin_nontemporal_store(f[p], &r[(long)(j0 + p) * ldr + i]);
      const int kc = j0 / M;
#pragma unroll
      for (int a = 0; a < P; ++a) {
        rhop[((long)kc * 2 * P + a) * nx + i] = pa[a];
        rhop[((long)kc * 2 * P + P + a) * nx + i] = pb[a];
      }
    }
  }
}

// out_prev <- C, out <- (2C - Cp) + v, elementwise: every thread reads its
// element of all inputs before writing it, so the outputs may alias them.
template <bool RECON>
__global__ __launch_bounds__(256) void ch2_update(const double* c, long ldc, const double* cp,
                                                  long ldp, const double* __restrict__ v, long ldv,
                                                  double* out, double* out_prev, long ld, int nx,
                                                  int ny, int Sc, const double* __restrict__ rec) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= nx || j >= ny) return;
  const double vc = c[(long)j * ldc + i], vp = cp[(long)j * ldp + i];
  const double vv = RECON ? ch2_recon(v, ldv, j, i, Sc, rec) : v[(long)j * ldv + i];
  out_prev[(long)j * ld + i] = vc;
  out[(long)j * ld + i] = (2.0 * vc - vp) + vv;
}

// The same right-hand side and column chunk sweep in column-streaming form:
// one wave per 60 output columns of one 32-row chunk.  The wave's 64 lanes
// hold columns i0 - 2 .. i0 + 61 (periodically wrapped), so the x-neighbours
// at distance 1 and 2 of the 60 output lanes (2 .. 61) come from DPP lane
// shifts, with no LDS and no barrier; every lane walks the chunk's rows and
// two halo rows on each side, issuing the loads of row t + kPf2 while it works
// on row t, and sweeps its own column in registers.  The arithmetic is that of
// ch2_rhs + chunk_sweep, in the same order.
constexpr int kSeg2 = 60;  // output columns per wave
constexpr int kPf2 = 8;    // rows of loads in flight ahead of the row being worked

template <bool UPD, bool RECON>
__global__ __launch_bounds__(256) void ch2_column_pass(
    const double* __restrict__ c, long ld, const double* __restrict__ cp, long ldp,
    const double* __restrict__ v, long ldv, double* __restrict__ cnew, long ldn,
    double* __restrict__ r, long ldr, int nx, int ny, Ch2Coef K, int Sc,
    const double* __restrict__ rec, const double* __restrict__ srec, BandT<double> sbd,
    double* __restrict__ rhop) {
  constexpr int Q = M + 4;  // rows kc M - 2 .. kc M + M + 1
  const int lane = threadIdx.x & 63;
  const int seg = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (seg >= (nx + kSeg2 - 1) / kSeg2) return;  // no barrier in this kernel
  const int kc = blockIdx.y;
  int i = (seg * kSeg2 - 2 + lane) % nx;
  i += (i < 0) ? nx : 0;
  const int io = seg * kSeg2 + lane - 2;
  const bool own = lane >= 2 && lane < 62 && io < nx;

  auto row = [&](int t) -> long {
    int j = kc * M - 2 + t;
    j += (j < 0) ? ny : 0;
    j -= (j >= ny) ? ny : 0;
    return j;
  };
  // separator rows (final values) of the chunks kc - 1, kc, kc + 1
  double tp[P] = {}, to[P] = {}, tn[P] = {};
  if (RECON) {
    const int kcm = (kc == 0) ? Sc - 1 : kc - 1, kcp = (kc + 1 == Sc) ? 0 : kc + 1;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      tp[a] = v[((long)kcm * M + MI + a) * ldv + i];
      to[a] = v[((long)kc * M + MI + a) * ldv + i];
      tn[a] = v[((long)kcp * M + MI + a) * ldv + i];
    }
  }
  double lc[Q], lp[Q], lv[Q];
  auto load = [&](int t) {
    const long j = row(t);
    lc[t] = c[j * ld + i];
    lp[t] = cp[j * ldp + i];
    lv[t] = UPD ? v[j * ldv + i] : 0.0;
  };
#pragma unroll
  for (int t = 0; t < kPf2; ++t) load(t);

  double C[Q], Pv[Q], B[Q], U[Q], BL[Q], BR[Q], f[M];
#pragma unroll
  for (int t = 0; t < Q; ++t) {
    if (t + kPf2 < Q) load(t + kPf2);
    // row t: state update (with the deferred column correction of v)
    double vc = lc[t], vp = lp[t];
    if (UPD) {
      double vv = lv[t];
      if (RECON && t >= 2) {
        // own rows: chunk kc, position t - 2; the two rows below: chunk kc + 1,
        // positions 0 and 1; the two rows above are kc - 1's separators
        const bool below = t >= M + 2;
        const int pp = below ? t - M - 2 : t - 2;
        if (pp < MI) {
#pragma unroll
          for (int a = 0; a < P; ++a)
            vv = vv - rec[pp * 8 + 4 + a] * (below ? to[a] : tp[a]) -
                 rec[pp * 8 + 6 + a] * (below ? tn[a] : to[a]);
        }
      }
      const double vn = (2.0 * vc - vp) + vv;
      vp = vc;
      vc = vn;
      if (t >= 2 && t < M + 2 && own)
        __builtin_nontemporal_store(vn, &cnew[((long)kc * M + t - 2) * ldn + io]);
    }
    C[t] = vc;
    Pv[t] = vp;
    B[t] = 2.0 * vc - vp;
    U[t] = vc * vc * vc - vc;
    BL[t] = dpp_from_left(B[t], B[t]);
    BR[t] = dpp_from_right(B[t], B[t]);
    if (t >= 4) {  // right-hand side of row w = t - 2 (own row w - 2)
      const int w = t - 2;
      const double BL2 = dpp_from_left(BL[w], BL[w]), BR2 = dpp_from_right(BR[w], BR[w]);
      // mu of the x-neighbours: their own C^3 - C, moved over by DPP
      const double mu_l = dpp_from_left(U[w], U[w]), mu_r = dpp_from_right(U[w], U[w]);
      const double d4x = (BL2 - 4.0 * BL[w] + 6.0 * B[w] - 4.0 * BR[w] + BR2) * K.inv_dx4;
      const double d4y =
          (B[w - 2] - 4.0 * B[w - 1] + 6.0 * B[w] - 4.0 * B[w + 1] + B[w + 2]) * K.inv_dy4;
      const double dyy_w = BL[w + 1] + BL[w - 1] - 2.0 * BL[w];
      const double dyy_c = B[w + 1] + B[w - 1] - 2.0 * B[w];
      const double dyy_e = BR[w + 1] + BR[w - 1] - 2.0 * BR[w];
      const double dxxyy = (dyy_e + dyy_w - 2.0 * dyy_c) * K.inv_dx2dy2;
      const double bih = d4x + 2.0 * dxxyy + d4y;
      const double lap = (mu_r + mu_l - 2.0 * U[w]) * K.inv_dx2 +
                         (U[w + 1] + U[w - 1] - 2.0 * U[w]) * K.inv_dy2;
      f[w - 2] = -(2.0 / 3.0) * (C[w] - Pv[w]) - K.a * bih + K.b * lap;
    }
    // this row's values are complete here and the next row's loads are issued
    // after this point (empty volatile asms keep their order)
    asm volatile("" : "+v"(B[t]), "+v"(BL[t]), "+v"(BR[t]), "+v"(U[t]), "+v"(C[t]),
                 "+v"(Pv[t])::"memory");
    if (t >= 4) asm volatile("" : "+v"(f[t - 4]));
  }
  chunk_sweep<P, M, double>(f, srec, sbd.c[0]);
  double pa[P], pb[P];
  chunk_parts<P, M, double>(f, sbd, pa, pb);
  if (!own) return;
#pragma unroll
  for (int p = 0; p < MI; ++p) __builtin_nontemporal_store(f[p], &r[((long)kc * M + p) * ldr + io]);
#pragma unroll
  for (int a = 0; a < P; ++a) {
    rhop[((long)kc * 2 * P + a) * nx + io] = pa[a];
    rhop[((long)kc * 2 * P + P + a) * nx + io] = pb[a];
  }
}

hipError_t launch_ch2_rhs(const double* c, long ld, const double* cp, long ldp, const double* v,
                          long ldv, double* cnew, long ldn, double* r, long ldr, int nx, int ny,
                          const Ch2Coef& K, const DevChunk* recon, const DevChunk* sweep,
                          double* rho, hipStream_t st) {
  dim3 grid((nx + kT2X - 1) / kT2X, (ny + kT2Y - 1) / kT2Y);
  const int Sc = recon ? recon->S : 0;
  const double* rec = recon ? recon->rec : nullptr;
  BandT<double> sbd{};
  const double* srec = nullptr;
  if (sweep) {
    for (int k = 0; k < 5; ++k) sbd.c[k] = sweep->coef[k];
    srec = sweep->rec;
  }
#define CHX_CH2(U, R, W)                                                                        \
  hipLaunchKernelGGL((ch2_rhs<U, R, W>), grid, dim3(kT2T), 0, st, c, ld, cp, ldp, v, ldv, cnew, \
                     ldn, r, ldr, nx, ny, K, Sc, rec, srec, sbd, rho)
  // the column-streaming kernel runs one wave per (60-column segment, chunk):
  // it takes over once that fills every SIMD twice; smaller grids keep the
  // tile kernel, whose eight waves per 64 x 32 tile fill the chip sooner
  // (1024 x 1024: 0.039 ms per step with it, 0.043 with the column kernel)
  const bool columns = sweep && (long)((nx + kSeg2 - 1) / kSeg2) * sweep->S >= 2048;
  if (columns) {
    const int Scol = sweep->S;
    if ((long)Scol * M != ny || (recon && recon->S != Scol)) return hipErrorInvalidValue;
    // blocks in chunk-row order (measured: banding whole chunk rows onto one
    // XCD, so shared halo rows meet in one L2, was 3-4 % slower)
    const dim3 g2((unsigned)(((nx + kSeg2 - 1) / kSeg2 + 3) / 4), (unsigned)Scol);
#define CHX_CH2C(U, R)                                                                       \
  hipLaunchKernelGGL((ch2_column_pass<U, R>), g2, dim3(256), 0, st, c, ld, cp, ldp, v, ldv, cnew, \
                     ldn, r, ldr, nx, ny, K, Scol, rec, srec, sbd, rho)
    if (v && recon) CHX_CH2C(true, true);
    else if (v) CHX_CH2C(true, false);
    else CHX_CH2C(false, false);
#undef CHX_CH2C
  } else if (sweep) {
    if (v && recon) CHX_CH2(true, true, true);
    else if (v) CHX_CH2(true, false, true);
    else CHX_CH2(false, false, true);
  } else {
    if (v && recon) CHX_CH2(true, true, false);
    else if (v) CHX_CH2(true, false, false);
    else CHX_CH2(false, false, false);
  }
#undef CHX_CH2
  return hipGetLastError();
}

hipError_t launch_ch2_update(const double* c, long ldc, const double* cp, long ldp,
                             const double* v, long ldv, double* out, double* out_prev, long ld,
                             int nx, int ny, const DevChunk* recon, hipStream_t st) {
  dim3 grid((nx + 63) / 64, (ny + 3) / 4);
  const int Sc = recon ? recon->S : 0;
  const double* rec = recon ? recon->rec : nullptr;
  if (recon)
    hipLaunchKernelGGL(ch2_update<true>, grid, dim3(256), 0, st, c, ldc, cp, ldp, v, ldv, out,
                       out_prev, ld, nx, ny, Sc, rec);
  else
    hipLaunchKernelGGL(ch2_update<false>, grid, dim3(256), 0, st, c, ldc, cp, ldp, v, ldv, out,
                       out_prev, ld, nx, ny, Sc, rec);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small grids: the whole field stays in one workgroup's LDS for every step of
// a call, so a step costs no HBM traffic and no launch.  LDS holds the field F
// (row pitch nx + nx/32: one pad element after every 32-element row segment,
// so the row phase's per-thread segments start on different banks) and the
// separator parts Q (four arrays of one value per task).  Every phase gives
// one task to each thread: column phases take (column chunk kc, column i),
// row phases (row j, row chunk kr); both count nx ny / 32 tasks.  Per step:
//   C1  right-hand side of the state (3-row register window, x-neighbours by
//       DPP lane shifts, wave edges read from F), diagnostics of the state;
//   C2  interior sweep of the column chunk, separator parts -> Q, y -> F;
//   C3  column separators (window convolution with the reduced blocks) -> F;
//   C4  column correction x = y - Zl s_prev - Zr s_own in F;
//   R1  row chunk sweep in registers, parts -> Q;
//   R2  row separators -> F;  R3  row correction, row chunk -> F.
// The correction is applied at once here (the multi-kernel path defers it to
// the next step's column pass), so the two paths agree to rounding, not bit
// for bit.
__device__ __forceinline__ int sfi(int j, int i, int PX) { return j * PX + i + (i >> 5); }

__device__ __forceinline__ int wrap_mod(int j, int S) {
  j %= S;
  return j < 0 ? j + S : j;
}

template <bool DIAG, bool NOISE>
__device__ __forceinline__ void small_steps_body(double* __restrict__ c, long ldc, int nx, int ny,
                                                 int nsteps, const DevChunk& cy,
                                                 const DevChunk& cx, const ChCoef& K,
                                                 double* __restrict__ diag, double* smem,
                                                 const SmallNoise& nz) {
  __shared__ double red[2 * (kSmallMaxThreads / 64)];
  const int PX = nx + (nx >> 5);
  double* F = smem;
  const int ntask = nx * ny / M;
  double* Q = smem + (long)ny * PX;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nwave = ntask >> 6;
  const int Sy = ny / M, Sx = nx / M;
  const bool act = tid < ntask;  // whole waves: ntask is a multiple of 64
  // the plans arrive inside structs (kernel argument or class record)
  const TabD yrec = (TabD)cy.rec, xrec = (TabD)cx.rec;
  const TabD yblk = (TabD)cy.blocks, xblk = (TabD)cx.blocks;
  for (int e = tid; e < nx * ny; e += blockDim.x) {
    const int j = e / nx, i = e - j * nx;
    F[sfi(j, i, PX)] = c[(long)j * ldc + i];
  }
  BandT<double> bdy, bdx;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    bdy.c[k] = cy.coef[k];
    bdx.c[k] = cx.coef[k];
  }
  __syncthreads();
  for (int n = 0;; ++n) {
    if (!DIAG && n == nsteps) break;
    // task coordinates, re-derived every step from an opaque copy of the
    // thread index: otherwise the compiler keeps every LDS address of every
    // phase live across the step loop (well over the register budget)
    int tv = tid;
    asm volatile("" : "+v"(tv));
    const int kc = tv / nx, ic = tv - kc * nx;
    const int il = (ic == 0) ? nx - 1 : ic - 1, ir = (ic == nx - 1) ? 0 : ic + 1;
    const int jr = tv / Sx, kr = tv - jr * Sx;
    const int rbase = jr * PX + kr * (M + 1);  // = sfi(jr, kr * M, PX)
    // C1: right-hand side of the state and its diagnostics
    double f[M];
    double msum = 0.0, esum = 0.0;
    if (act) {
      auto row_of = [&](int q) {  // q = 0 .. M+1 -> rows kc*M - 1 .. kc*M + M
        int r = kc * M - 1 + q;
        r += (r < 0) ? ny : 0;
        r -= (r >= ny) ? ny : 0;
        return r;
      };
      auto edge = [&](int row) {
        return lane == 0 ? F[sfi(row, il, PX)] : (lane == 63 ? F[sfi(row, ir, PX)] : 0.0);
      };
      double xc_m = F[sfi(row_of(0), ic, PX)];
      double e0 = edge(row_of(0));
      double xl_m = dpp_from_left(xc_m, e0), xr_m = dpp_from_right(xc_m, e0);
      double xc_c = F[sfi(row_of(1), ic, PX)];
      double e1 = edge(row_of(1));
      double xl_c = dpp_from_left(xc_c, e1), xr_c = dpp_from_right(xc_c, e1);
      // forcing: the draws of this row's point and of the one below it are
      // carried from row to row; the right neighbour's are drawn per row
      const unsigned long long nstep = nz.step0 + (unsigned long long)n;
      double nrx_c = 0.0, nry_c = 0.0;
      if (NOISE) cook_pair(nz.seed_state, nstep, kc * M, ic, nx, ny, nrx_c, nry_c);
#pragma unroll
      for (int p = 0; p < M; ++p) {
        const int rp = row_of(p + 2);
        double xc_p = F[sfi(rp, ic, PX)];
        double en = edge(rp);
        asm volatile("" : "+v"(xc_p), "+v"(en));
        const double xl_p = dpp_from_left(xc_p, en);
        const double xr_p = dpp_from_right(xc_p, en);
        const double mu_c = xc_c * xc_c * xc_c - xc_c;
        const double mu_l = xl_c * xl_c * xl_c - xl_c;
        const double mu_r = xr_c * xr_c * xr_c - xr_c;
        const double mu_s = xc_m * xc_m * xc_m - xc_m;
        const double mu_n = xc_p * xc_p * xc_p - xc_p;
        const double lap = K.cx * (mu_r + mu_l - 2.0 * mu_c) + K.cy * (mu_n + mu_s - 2.0 * mu_c);
        const double dyy_w = xl_p + xl_m - 2.0 * xl_c;
        const double dyy_c = xc_p + xc_m - 2.0 * xc_c;
        const double dyy_e = xr_p + xr_m - 2.0 * xr_c;
        double r = xc_c + lap - K.ccross * (dyy_e + dyy_w - 2.0 * dyy_c);
        if (NOISE) {
          const int j = kc * M + p, jn = (j + 1 == ny) ? 0 : j + 1;
          double rx_e, ry_e, rx_n, ry_n;
          cook_pair(nz.seed_state, nstep, j, ir, nx, ny, rx_e, ry_e);
          cook_pair(nz.seed_state, nstep, jn, ic, nx, ny, rx_n, ry_n);
          const double div = (rx_e - nrx_c) * nz.inv_dx + (ry_n - nry_c) * nz.inv_dy;
          r = r + nz.scale * div;
          nrx_c = rx_n;
          nry_c = ry_n;
        }
        if (DIAG) {
          const double w = xc_c * xc_c - 1.0;
          const double gx = (xr_c - xc_c) * K.inv_dx, gy = (xc_p - xc_c) * K.inv_dy;
          msum += xc_c;
          esum += 0.25 * w * w + K.half_gamma * (gx * gx + gy * gy);
          asm volatile("" : "+v"(r), "+v"(msum), "+v"(esum));
        } else {
          asm volatile("" : "+v"(r));
        }
        f[p] = r;
        xl_m = xl_c; xc_m = xc_c; xr_m = xr_c;
        xl_c = xl_p; xc_c = xc_p; xr_c = xr_p;
        // keep the next row's LDS loads below this row's work (bounded
        // register pressure: the 32 right-hand sides stay live to C2)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (DIAG && act) {
      msum = wave_sum(msum);
      esum = wave_sum(esum);
      if (lane == 0) {
        red[2 * wave] = msum;
        red[2 * wave + 1] = esum;
      }
    }
    __syncthreads();
    if (DIAG && tid == 0) {
      double m = 0.0, e = 0.0;
      for (int w = 0; w < nwave; ++w) {
        m += red[2 * w];
        e += red[2 * w + 1];
      }
      diag[2 * n] = m * K.dxdy;
      diag[2 * n + 1] = e * K.dxdy;
    }
    if (n == nsteps) break;
    // C2: column chunk sweep, separator parts, y
    if (act) {
      chunk_sweep<2, M, double>(f, yrec, bdy.c[0]);
      double pa[P], pb[P];
      chunk_parts<P, M, double>(f, bdy, pa, pb);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        Q[a * ntask + tid] = pa[a];
        Q[(P + a) * ntask + tid] = pb[a];
      }
#pragma unroll
      for (int p = 0; p < MI; ++p) F[sfi(kc * M + p, ic, PX)] = f[p];
    }
    __syncthreads();
    // C3: column separators s_kc(ic) from the parts of the window chunks
    if (act) {
      double acc[P] = {0.0, 0.0};
      for (int t = 0; t < cy.dcount; ++t) {
        const int j = wrap_mod(kc + cy.dlo + t, Sy);
        const int jn = (j + 1 == Sy) ? 0 : j + 1;
        double rv[P];
#pragma unroll
        for (int a = 0; a < P; ++a)
          rv[a] = Q[a * ntask + j * nx + ic] - Q[(P + a) * ntask + jn * nx + ic];
        const TabD B = yblk + t * 4;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int q = 0; q < P; ++q) acc[a] = acc[a] + B[a * 2 + q] * rv[q];
      }
#pragma unroll
      for (int a = 0; a < P; ++a) F[sfi(kc * M + MI + a, ic, PX)] = acc[a];
    }
    __syncthreads();
    // C4: column correction of the chunk interior
    if (act) {
      const int kp = (kc == 0) ? Sy - 1 : kc - 1;
      double sp[P], so[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        sp[a] = F[sfi(kp * M + MI + a, ic, PX)];
        so[a] = F[sfi(kc * M + MI + a, ic, PX)];
      }
#pragma unroll
      for (int p = 0; p < MI; ++p) {
        double v = F[sfi(kc * M + p, ic, PX)];
#pragma unroll
        for (int a = 0; a < P; ++a)
          v = v - yrec[p * 8 + 4 + a] * sp[a] - yrec[p * 8 + 6 + a] * so[a];
        F[sfi(kc * M + p, ic, PX)] = v;
      }
    }
    __syncthreads();
    // R1: row chunk sweep, parts
    double so[P] = {0.0, 0.0};
    if (act) {
#pragma unroll
      for (int p = 0; p < M; ++p) f[p] = F[rbase + p];
      chunk_sweep<2, M, double>(f, xrec, bdx.c[0]);
      double pa[P], pb[P];
      chunk_parts<P, M, double>(f, bdx, pa, pb);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        Q[a * ntask + tid] = pa[a];
        Q[(P + a) * ntask + tid] = pb[a];
      }
    }
    __syncthreads();
    // R2: row separators
    if (act) {
      const int rs = jr * Sx;
      for (int t = 0; t < cx.dcount; ++t) {
        const int j = wrap_mod(kr + cx.dlo + t, Sx);
        const int jn = (j + 1 == Sx) ? 0 : j + 1;
        double rv[P];
#pragma unroll
        for (int a = 0; a < P; ++a)
          rv[a] = Q[a * ntask + rs + j] - Q[(P + a) * ntask + rs + jn];
        const TabD B = xblk + t * 4;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int q = 0; q < P; ++q) so[a] = so[a] + B[a * 2 + q] * rv[q];
      }
#pragma unroll
      for (int a = 0; a < P; ++a) F[rbase + MI + a] = so[a];
    }
    __syncthreads();
    // R3: row correction, the row chunk back into F
    if (act) {
      const int kp = (kr == 0) ? Sx - 1 : kr - 1;
      double sp[P];
#pragma unroll
      for (int a = 0; a < P; ++a) sp[a] = F[jr * PX + kp * (M + 1) + MI + a];
      chunk_correct<P, M, double>(f, xrec, sp, so);
#pragma unroll
      for (int p = 0; p < M; ++p) F[rbase + p] = f[p];
    }
    __syncthreads();
  }
  for (int e = tid; e < nx * ny; e += blockDim.x) {
    const int j = e / nx, i = e - j * nx;
    c[(long)j * ldc + i] = F[sfi(j, i, PX)];
  }
}

template <bool DIAG, bool NOISE>
__global__ __launch_bounds__(kSmallMaxThreads) void ch_small_steps(double* c, long ldc, int nx,
                                                                   int ny, int nsteps, DevChunk cy,
                                                                   DevChunk cx, ChCoef K,
                                                                   double* diag, SmallNoise nz) {
  extern __shared__ double smem_small[];
  small_steps_body<DIAG, NOISE>(c, ldc, nx, ny, nsteps, cy, cx, K, diag, smem_small, nz);
}

size_t ch_small_lds_bytes(int nx, int ny) {
  return ((size_t)ny * (nx + nx / M) + (size_t)4 * nx * ny / M) * sizeof(double);
}

bool ch_small_fits(int nx, int ny, size_t max_lds) {
  if (nx % 64 != 0 || ny % M != 0) return false;
  const long ntask = (long)nx * ny / M;
  return ntask <= kSmallMaxThreads && ch_small_lds_bytes(nx, ny) <= max_lds;
}

hipError_t launch_ch_small_steps(double* c, long ldc, int nx, int ny, int nsteps,
                                 const DevChunk& cy, const DevChunk& cx, const ChCoef& K,
                                 double* diag, const SmallNoise* nz, hipStream_t st) {
  const int nt = nx * ny / M;
  const size_t lds = ch_small_lds_bytes(nx, ny);
  const SmallNoise z = nz ? *nz : SmallNoise{};
#define CHX_SMALL(D, N)                                                                     \
  hipLaunchKernelGGL((ch_small_steps<D, N>), dim3(1), dim3(nt), lds, st, c, ldc, nx, ny, nsteps, \
                     cy, cx, K, diag, z)
  if (diag && nz) CHX_SMALL(true, true);
  else if (diag) CHX_SMALL(true, false);
  else if (nz) CHX_SMALL(false, true);
  else CHX_SMALL(false, false);
#undef CHX_SMALL
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ensemble kernels: block = work item {run, a, b}; buffers by step parity.
// Their run's pointers come out of memory, so they pass them typed by
// address space (TabD, GCD).
__device__ __forceinline__ double* ens_buf(unsigned char* ws, const EnsRun& R, int step) {
  return reinterpret_cast<double*>(ws + ((step & 1) ? R.off_b1 : R.off_b0));
}

template <bool RECON, bool DIAG, bool NOISE>
__global__ __launch_bounds__(256) void ens_column_pass(const EnsRun* __restrict__ runs,
                                                       EnsClasses cls,
                                                       const int4* __restrict__ items,
                                                       unsigned char* ws, int step,
                                                       const unsigned long long* noise_step) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const EnsClass& C = cls.c[R.cls];
  const auto src = (GCD)((step == 0) ? R.c : ens_buf(ws, R, step - 1));
  const long lds = (step == 0) ? R.ldc : (long)R.nx;
  BandT<double> bd;
#pragma unroll
  for (int k = 0; k < 5; ++k) bd.c[k] = C.py.coef[k];
  double* part = reinterpret_cast<double*>(ws + R.off_part);
  double* rho = reinterpret_cast<double*>(ws + R.off_rho);
  column_pass_body<RECON, DIAG, NOISE, false, kChunk, true>(src, lds, ens_buf(ws, R, step), R.nx,
                                                           R.nx, R.ny, R.Sc,
                                       (TabD)C.py.rec, bd, rho, C.K,
                                       DIAG ? part + 2 * ((long)it.z * R.ncb + it.y) : nullptr,
                                       it.y, it.z,
                                       NOISE ? SmallNoise{R.nseed,
                                                          *noise_step + (unsigned long long)step,
                                                          R.nscale, R.ninv_dx, R.ninv_dy}
                                             : SmallNoise{});
}

// The ensemble's forcing counter moves on by the steps of one call (one
// thread, an ordinary global store).
__global__ void ens_noise_advance(unsigned long long* noise_step, int nsteps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *noise_step += (unsigned long long)nsteps;
}


// The pass after the last step for every multi-kernel run (column-pass work
// items): state reconstructed into the caller's field, with its diagnostics
// partials (DIAG) in the run's column-pass partial slots.
template <bool DIAG>
__global__ __launch_bounds__(256) void ens_column_final(const EnsRun* __restrict__ runs,
                                                        EnsClasses cls,
                                                        const int4* __restrict__ items,
                                                        unsigned char* ws, int last_step) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const EnsClass& C = cls.c[R.cls];
  double* part = reinterpret_cast<double*>(ws + R.off_part);
  const BandT<double> bd{};
  column_pass_body<true, DIAG, false, true>(ens_buf(ws, R, last_step), R.nx, R.c, R.ldc, R.nx,
                                            R.ny, R.Sc, (TabD)C.py.rec, bd, nullptr, C.K,
                                            DIAG ? part + 2 * ((long)it.z * R.ncb + it.y)
                                                 : nullptr,
                                            it.y, it.z);
}


__global__ __launch_bounds__(256) void ens_diag_final(const EnsRun* __restrict__ runs,
                                                      EnsClasses cls, const int* __restrict__ big,
                                                      unsigned char* ws, double* diag_out,
                                                      long diag_stride, int index) {
  const int r = big[blockIdx.x];
  const EnsRun R = runs[r];
  const double* part = reinterpret_cast<const double*>(ws + R.off_part);
  diag_final_body(part, R.ncolblocks, cls.c[R.cls].K.dxdy,
                  diag_out + r * diag_stride + 2 * (long)index);
}

// Small runs of an ensemble: block b advances run small[b] through all nsteps
// steps with its field resident in LDS (blockDim and LDS sized for the
// largest small run; the threads beyond a smaller run's tasks stay idle).
template <bool DIAG, bool NOISE>
__global__ __launch_bounds__(kSmallMaxThreads) void ens_small_steps(
    const EnsRun* __restrict__ runs, EnsClasses cls, const int* __restrict__ small, int nsteps,
    double* diag_out, long diag_stride, const unsigned long long* noise_step) {
  extern __shared__ double smem_small[];
  const int r = small[blockIdx.x];
  const EnsRun R = runs[r];
  const EnsClass& C = cls.c[R.cls];
  SmallNoise nz{};
  if (NOISE) nz = SmallNoise{R.nseed, *noise_step, R.nscale, R.ninv_dx, R.ninv_dy};
  small_steps_body<DIAG, NOISE>(R.c, R.ldc, R.nx, R.ny, nsteps, C.py, C.px, C.K,
                                DIAG ? diag_out + r * diag_stride : nullptr, smem_small, nz);
}

hipError_t launch_ens_small_steps(const EnsRun* runs, const EnsClasses& cls, const int* small,
                                  int nsmall, int threads, size_t lds, int nsteps,
                                  double* diag_out, long diag_stride,
                                  const unsigned long long* noise_step, hipStream_t st) {
#define CHX_ENSSMALL(D, N)                                                                   \
  hipLaunchKernelGGL((ens_small_steps<D, N>), dim3(nsmall), dim3(threads), lds, st, runs, cls, \
                     small, nsteps, diag_out, diag_stride, noise_step)
  if (diag_out && noise_step) CHX_ENSSMALL(true, true);
  else if (diag_out) CHX_ENSSMALL(true, false);
  else if (noise_step) CHX_ENSSMALL(false, true);
  else CHX_ENSSMALL(false, false);
#undef CHX_ENSSMALL
  return hipGetLastError();
}

hipError_t launch_ens_noise_advance(unsigned long long* noise_step, int nsteps, hipStream_t st) {
  hipLaunchKernelGGL(ens_noise_advance, dim3(1), dim3(64), 0, st, noise_step, nsteps);
  return hipGetLastError();
}

hipError_t launch_ens_column_pass(bool recon, bool diag, const unsigned long long* noise_step,
                                  const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                  int nitems, unsigned char* ws, int step, hipStream_t st) {
  const bool noise = noise_step != nullptr;
#define CHX_ENSCOL(R, D, N)                                                                        \
  hipLaunchKernelGGL((ens_column_pass<R, D, N>), dim3(nitems), dim3(256), 0, st, runs, cls, items, \
                     ws, step, noise_step)
#define CHX_ENSCOL2(R, D) \
  if (noise) CHX_ENSCOL(R, D, true); else CHX_ENSCOL(R, D, false)
  if (recon && diag) { CHX_ENSCOL2(true, true); }
  else if (recon) { CHX_ENSCOL2(true, false); }
  else if (diag) { CHX_ENSCOL2(false, true); }
  else { CHX_ENSCOL2(false, false); }
#undef CHX_ENSCOL2
#undef CHX_ENSCOL
  return hipGetLastError();
}



hipError_t launch_ens_diag_final(const EnsRun* runs, const EnsClasses& cls, const int* big,
                                 int nbig, unsigned char* ws, double* diag_out, long diag_stride,
                                 int index, hipStream_t st) {
  hipLaunchKernelGGL(ens_diag_final, dim3(nbig), dim3(256), 0, st, runs, cls, big, ws, diag_out,
                     diag_stride, index);
  return hipGetLastError();
}

hipError_t launch_ens_column_final(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                   int nitems, const int* big, int nbig, unsigned char* ws,
                                   int last_step, double* diag_out, long diag_stride, int index,
                                   hipStream_t st) {
  if (diag_out) {
    hipLaunchKernelGGL((ens_column_final<true>), dim3(nitems), dim3(256), 0, st, runs, cls, items,
                       ws, last_step);
    hipLaunchKernelGGL(ens_diag_final, dim3(nbig), dim3(256), 0, st, runs, cls, big, ws,
                       diag_out, diag_stride, index);
  } else {
    hipLaunchKernelGGL((ens_column_final<false>), dim3(nitems), dim3(256), 0, st, runs, cls,
                       items, ws, last_step);
  }
  return hipGetLastError();
}

}  // namespace chx
