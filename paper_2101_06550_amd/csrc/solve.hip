// solve.hip -- batched constant-coefficient banded solves on gfx950.
//
// Kernels (P = half bandwidth: 2 penta, 1 tri; T = FP64 or FP32 sweeps):
//  whole_sweep     one thread per system, any n, any strides: the thesis's
//                  own arrangement (Ch.4 "Implementation on GPU": one thread
//                  per system, factor once, forward + back sweep), with the
//                  bordering of the last P unknowns fused in (q^T f gathered
//                  in the forward sweep, Z x_tail applied in the back sweep).
//  chunk_sweep_il  interleaved layout, one thread per (system, chunk of 32):
//                  in-register sweep of the chunk interior, separator parts.
//  reduced_il      separator unknowns of every chunk from the reduced
//                  right-hand sides (block-circulant inverse, truncated).
//  correct_il      interior correction x = y - Zl s_prev - Zr s_own.
//  row_solve_lds   contiguous layout: whole rows staged through LDS (the
//                  transpose of the thesis, done in LDS), chunk sweeps in
//                  registers, reduced system and correction inside the
//                  workgroup, coalesced store.  Two HBM accesses per unknown.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "ens.hpp"
#include "launch.hpp"

namespace chx {

// ---------------------------------------------------------------------------
template <int P, typename T, bool ACC>
__global__ __launch_bounds__(256) void whole_sweep(double* work, long ss, long es, double* out,
                                                   long oss, long oes, int batch, int n,
                                                   int periodic,
                                                   const T* __restrict__ rec, BandT<T> bd,
                                                   T mi00, T mi01, T mi10, T mi11) {
  // work: right-hand sides on entry, forward-sweep scratch; out: solutions
  // (written, or added when ACC).  work == out is the in-place solve.
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= batch) return;
  double* xs = work + s * ss;
  double* os = out + s * oss;
  const int mi = periodic ? n - P : n;
  const T eps = bd.c[0];
  T g1 = 0, g2 = 0, q0 = 0, q1 = 0;
  for (int i = 0; i < mi; ++i) {
    const T f = (T)xs[(long)i * es];
    const T* r = rec + (long)i * 8;
    if (periodic) {
      q0 = q0 + r[4] * f;
      if (P == 2) q1 = q1 + r[5] * f;
    }
    T v = f;
    if (P == 2) v = v - eps * g2;
    v = v - r[1] * g1;
    v = v * r[0];
    xs[(long)i * es] = (double)v;
    g2 = g1;
    g1 = v;
  }
  T t0 = 0, t1 = 0;
  if (periodic) {
    const T r0 = (T)xs[(long)mi * es] - q0;
    const T r1 = (P == 2) ? (T)xs[(long)(mi + 1) * es] - q1 : T(0);
    t0 = mi00 * r0 + mi01 * r1;
    t1 = mi10 * r0 + mi11 * r1;
  }
  T y1 = 0, y2 = 0;
  for (int i = mi - 1; i >= 0; --i) {
    const T* r = rec + (long)i * 8;
    T v = (T)xs[(long)i * es];
    if (P == 2) v = v - r[3] * y2;
    v = v - r[2] * y1;
    y2 = y1;
    y1 = v;
    T o = v;
    if (periodic) {
      o = o - r[6] * t0;
      if (P == 2) o = o - r[7] * t1;
    }
    if (ACC) os[(long)i * oes] += (double)o;
    else os[(long)i * oes] = (double)o;
  }
  if (periodic) {
    if (ACC) {
      os[(long)mi * oes] += (double)t0;
      if (P == 2) os[(long)(mi + 1) * oes] += (double)t1;
    } else {
      os[(long)mi * oes] = (double)t0;
      if (P == 2) os[(long)(mi + 1) * oes] = (double)t1;
    }
  }
}

// ---------------------------------------------------------------------------
// Interleaved layout: element i of system s at i*ld + s.  Block = 64 systems
// (one wave, 512-byte coalesced rows) x 4 chunks (4 waves).
template <int P, int M, typename T, typename Ty, bool STORE_Y = true>
__global__ __launch_bounds__(256) void chunk_sweep_il(const double* src, long lds, Ty* y, long ldy,
                                                      int batch, int S, const T* __restrict__ rec,
                                                      BandT<T> bd, T* __restrict__ rho) {
  // src: right-hand sides (FP64); y: chunk-interior solutions (may alias src);
  // STORE_Y = false: only the separator parts are written
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long s = (long)blockIdx.x * 64 + lane;
  const int k = blockIdx.y * 4 + wave;
  if (s >= batch || k >= S) return;
  T f[M];
  const double* base = src + (long)k * M * lds + s;
#pragma unroll
  // the right-hand side streams in with non-temporal loads: measured on the
  // standalone solve of 131072 systems, both passes' loads so marked took it
  // from 0.675 to 0.605 ms (ordinary loads in this kernel alone: 0.633)
  for (int p = 0; p < M; ++p) f[p] = (T)__builtin_nontemporal_load(&base[(long)p * lds]);
  chunk_sweep<P, M, T>(f, rec, bd.c[0]);
  T pa[P], pb[P];
  chunk_parts<P, M, T>(f, bd, pa, pb);
  if (STORE_Y) {
    Ty* yb = y + (long)k * M * ldy + s;
#pragma unroll
    for (int p = 0; p < M - P; ++p) __builtin_nontemporal_store((Ty)f[p], &yb[(long)p * ldy]);
  }
#pragma unroll
  for (int a = 0; a < P; ++a) {
    rho[((long)k * 2 * P + a) * batch + s] = pa[a];
    rho[((long)k * 2 * P + P + a) * batch + s] = pb[a];
  }
}

// Second pass of a standalone solve: x holds the right-hand sides in the
// chunk interiors (untouched by the first pass) and the solved separators in
// the separator rows; each chunk is swept again (the same arithmetic as the
// first pass, recomputed instead of stored and re-read) and corrected,
// x = E_m^{-1} f - Zl s_prev - Zr s_own, in place.
template <int P, int M>
__global__ __launch_bounds__(256) void chunk_resolve_il(double* x, long ld, int batch, int S,
                                                        const double* __restrict__ rec,
                                                        BandT<double> bd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long s = (long)blockIdx.x * 64 + lane;
  const int k = blockIdx.y * 4 + wave;
  if (s >= batch || k >= S) return;
  constexpr int MI = M - P;
  const int kp = wrap_once(k - 1, S);
  double sp[P], so[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    sp[a] = x[((long)kp * M + MI + a) * ld + s];
    so[a] = x[((long)k * M + MI + a) * ld + s];
  }
  double f[M];
  double* base = x + (long)k * M * ld + s;
#pragma unroll
  for (int p = 0; p < MI; ++p) f[p] = __builtin_nontemporal_load(&base[(long)p * ld]);
#pragma unroll
  for (int p = MI; p < M; ++p) f[p] = 0.0;  // not read by the interior sweep
  chunk_sweep<P, M, double>(f, rec, bd.c[0]);
#pragma unroll
  for (int p = 0; p < MI; ++p) {
    double v = f[p];
#pragma unroll
    for (int a = 0; a < P; ++a) v = v - rec[p * 8 + 4 + a] * sp[a] - rec[p * 8 + 6 + a] * so[a];
    __builtin_nontemporal_store(v, &base[(long)p * ld]);
  }
}

// Reduced separator system: sep_k = sum_d B_d (pa_{k+d} - pb_{k+d+1}).
// Writes separator a of chunk k to dst row (k * drow_stride + drow_off + a).
template <int P, typename T, typename Td>
__global__ __launch_bounds__(256) void reduced_il(const T* __restrict__ rho, int batch, int S,
                                                  const T* __restrict__ blocks, int dlo,
                                                  int dcount, Td* __restrict__ dst, long ld,
                                                  int drow_stride, int drow_off) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long s = (long)blockIdx.x * 64 + lane;
  const int k = blockIdx.y * 4 + wave;
  if (s >= batch || k >= S) return;
  T acc[P];
#pragma unroll
  for (int a = 0; a < P; ++a) acc[a] = 0;
  for (int t = 0; t < dcount; ++t) {
    const int j = wrap_once(k + dlo + t, S);
    const int jn = wrap_once(j + 1, S);
    T r[P];
#pragma unroll
    for (int a = 0; a < P; ++a)
      r[a] = rho[((long)j * 2 * P + a) * batch + s] - rho[((long)jn * 2 * P + P + a) * batch + s];
    const T* B = blocks + (long)t * 4;
#pragma unroll
    for (int a = 0; a < P; ++a)
#pragma unroll
      for (int c = 0; c < P; ++c) acc[a] = acc[a] + B[a * 2 + c] * r[c];
  }
#pragma unroll
  for (int a = 0; a < P; ++a)
    dst[((long)k * drow_stride + drow_off + a) * ld + s] = (Td)acc[a];
}

template <int P, int M, typename T, typename Ty, bool ACC>
__global__ __launch_bounds__(256) void correct_il(const Ty* y, long ldy, double* out, long ldo,
                                                  int batch, int S, const T* __restrict__ rec) {
  // y: chunk-interior solutions with the separators in the separator rows;
  // out = y - Zl s_prev - Zr s_own (written, or added when ACC); y may be out.
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long s = (long)blockIdx.x * 64 + lane;
  const int k = blockIdx.y * 4 + wave;
  if (s >= batch || k >= S) return;
  constexpr int MI = M - P;
  const int kp = wrap_once(k - 1, S);
  T sp[P], so[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    sp[a] = (T)y[((long)kp * M + MI + a) * ldy + s];
    so[a] = (T)y[((long)k * M + MI + a) * ldy + s];
  }
  const Ty* yb = y + (long)k * M * ldy + s;
  double* ob = out + (long)k * M * ldo + s;
  // every row (and, when accumulating, every old output) is loaded before
  // the first store: y may be out, so a load placed after a store would
  // wait for it
  T yv[MI];
  double ov[M];
#pragma unroll
  for (int p = 0; p < MI; ++p) yv[p] = (T)yb[(long)p * ldy];
  if (ACC) {
#pragma unroll
    for (int p = 0; p < M; ++p) ov[p] = ob[(long)p * ldo];
  }
#pragma unroll
  for (int p = 0; p < MI; ++p) {
    T v = yv[p];
#pragma unroll
    for (int a = 0; a < P; ++a) v = v - rec[p * 8 + 4 + a] * sp[a] - rec[p * 8 + 6 + a] * so[a];
    if (ACC) ob[(long)p * ldo] = ov[p] + (double)v;
    else __builtin_nontemporal_store((double)v, &ob[(long)p * ldo]);
  }
  if (ACC || (const void*)y != (const void*)out) {
#pragma unroll
    for (int a = 0; a < P; ++a) {
      if (ACC) ob[(long)(MI + a) * ldo] = ov[MI + a] + (double)so[a];
      else ob[(long)(MI + a) * ldo] = (double)so[a];
    }
  }
}

// Residual r = f - A x of cyclic (or plain) banded systems along lines:
// element i of system s at s*ss + i*es for each of f, x, r.  sys_fast puts
// consecutive threads on consecutive systems (interleaved layout), otherwise
// on consecutive unknowns (contiguous layout).  FP64 throughout.
template <int P>
__global__ __launch_bounds__(256) void resid_lines(const double* __restrict__ f, long fss,
                                                   long fes, const double* __restrict__ x,
                                                   long xss, long xes, double* __restrict__ r,
                                                   long rss, long res, int batch, int n,
                                                   BandT<double> bd, int periodic, int sys_fast) {
  const long fast = (long)blockIdx.x * 256 + threadIdx.x;
  const long slow = blockIdx.y;
  const long s = sys_fast ? fast : slow;
  const int i = (int)(sys_fast ? slow : fast);
  if (s >= batch || i >= n) return;
  double v = f[s * fss + (long)i * fes];
#pragma unroll
  for (int o = -P; o <= P; ++o) {
    int ii = i + o;
    if (periodic) {
      ii += (ii < 0) ? n : 0;
      ii -= (ii >= n) ? n : 0;
    } else if (ii < 0 || ii >= n) {
      continue;
    }
    v = v - bd.c[o + P] * x[s * xss + (long)ii * xes];
  }
  r[s * rss + (long)i * res] = v;
}

// ---------------------------------------------------------------------------
// Contiguous layout, whole rows through LDS.  256 threads = 256 chunks of M;
// a workgroup holds R = 256 / S rows of n = S * M unknowns.  Element
// (row r, chunk k, position p) lives at tile[(r*S + k)*(M+1) + p]; the +1
// pad spreads the per-thread chunks over the LDS banks.  One workgroup per row
// group; two are resident per CU, so one's loads overlap the other's sweeps.
// Element e of a workgroup's tile is row e / n, column e % n of its row
// group; its LDS slot is e + e / M (the +1 pad per chunk).  Dense rows
// (ld == n) need no division: the group is one contiguous range, loaded with
// every load of a thread in flight before the first LDS store.  Strided rows
// (ld > n) take a compact loop.
// Which rows a row kernel solves: row q of its list is row map(q) of the
// array.  IdRows solves rows 0 .. rows-1; SubsetRows the separator rows (the
// last two of every column chunk of length Mc: per = 2, off = Mc - 2) or the
// interior rows (per = Mc - 2, off = 0), so that the two subsets can be
// solved on two streams, the interior rows while the separators are formed.
struct IdRows {
  static constexpr bool identity = true;
  __device__ long operator()(long q) const { return q; }
};
struct SubsetRows {
  static constexpr bool identity = false;
  int Mc, per, off;
  __device__ long operator()(long q) const { return (q / per) * Mc + off + q % per; }
};

template <int P, int M, typename T, typename Tin = double, class Map = IdRows>
__device__ __forceinline__ void row_group_stage(T* tile, const Tin* x, long ld, int rows, int n,
                                                long row0, int nel, int t, bool dense,
                                                const Map& map = Map()) {
  // dense: the group's rows are consecutive rows of a dense array
  if (dense) {
    const long nvalid = ((long)rows - row0) * n;
    const Tin* base = x + map(row0) * n;
    Tin vin[M];
    if (nel == 256 * M && nvalid >= nel) {  // a full group: 16-byte loads, no guards
      if constexpr (sizeof(Tin) == 4) {  // four values per load
        // non-temporal: the FP32 rows are read once (8192^2 refined step
        // 1.632 -> 1.611 ms with 3 passes)
        typedef float fv4 __attribute__((ext_vector_type(4)));
        const fv4* b4 = reinterpret_cast<const fv4*>(base);
#pragma unroll
        for (int u = 0; u < M / 4; ++u) {
          const fv4 v = __builtin_nontemporal_load(&b4[t + 256 * u]);
          vin[4 * u] = v.x;
          vin[4 * u + 1] = v.y;
          vin[4 * u + 2] = v.z;
          vin[4 * u + 3] = v.w;
        }
#pragma unroll
        for (int u = 0; u < M / 4; ++u) {
          const int e = 4 * t + 1024 * u;
#pragma unroll
          for (int q = 0; q < 4; ++q) tile[e + q + e / M] = (T)vin[4 * u + q];
        }
      } else {
        const double2* b2 = reinterpret_cast<const double2*>(base);
#pragma unroll
        for (int u = 0; u < M / 2; ++u) {
          const double2 v = b2[t + 256 * u];
          vin[2 * u] = v.x;
          vin[2 * u + 1] = v.y;
        }
#pragma unroll
        for (int u = 0; u < M / 2; ++u) {
          const int e = 2 * t + 512 * u;
          tile[e + e / M] = (T)vin[2 * u];
          tile[e + 1 + e / M] = (T)vin[2 * u + 1];
        }
      }
      return;
    } else {
#pragma unroll
      for (int u = 0; u < M; ++u) {
        const int e = t + 256 * u;
        vin[u] = (e < nel && e < nvalid) ? base[e] : Tin(0);
      }
    }
#pragma unroll
    for (int u = 0; u < M; ++u) {
      const int e = t + 256 * u;
      if (e < nel) tile[e + e / M] = (T)vin[u];
    }
  } else {
#pragma unroll 1
    for (int u = 0; u < M; ++u) {
      const int e = t + 256 * u;
      const int r = e / n;
      const int i = e - r * n;
      if (e < nel) tile[e + e / M] = (row0 + r < rows) ? (T)x[map(row0 + r) * ld + i] : T(0);
    }
  }
}

// LDS of one row group (the caller declares it, so a kernel that also runs
// other work can alias it).
template <int P, int M, typename T>
struct RowLds {
  T tile[256 * (M + 1)];
  T rhol[256 * 2 * P];
  T sepl[256 * P];
};

// Rows row0 .. row0 + R - 1 (R = 256 / S rows of n = S M unknowns each).
template <int P, int M, typename T, bool ACC, typename Tin = double, typename Tout = double,
          class Map = IdRows>
__device__ __forceinline__ void row_solve_body(const Tin* src, long lds, Tout* dst, long ldd,
                                               int rows, int n, int S, int R,
                                               const T* __restrict__ rec, const BandT<T>& bd,
                                               const T* __restrict__ blocks, int dlo, int dcount,
                                               long row0, RowLds<P, M, T>& sh,
                                               const Map& map = Map()) {
  T* tile = sh.tile;
  T* rhol = sh.rhol;
  T* sepl = sh.sepl;
  const int t = threadIdx.x;
  const int nel = R * n;  // <= 256 * M
  const int r = t / S, k = t - r * S;
  // the group's valid rows are consecutive rows of the array (always so for
  // IdRows): then dense arrays take the contiguous loads and stores
  bool contig = true;
  if constexpr (!Map::identity) {
    const long last = (row0 + R <= rows ? row0 + R : rows) - 1;
    contig = map(last) - map(row0) == last - row0;
  }
  {
    row_group_stage<P, M, T, Tin, Map>(tile, src, lds, rows, n, row0, nel, t, lds == n && contig,
                                       map);
    __syncthreads();
    const bool active = (r < R) && (row0 + r < rows);
    T f[M];
    if (active) {
#pragma unroll
      for (int p = 0; p < M; ++p) f[p] = tile[t * (M + 1) + p];
      chunk_sweep<P, M, T>(f, rec, bd.c[0]);
      T pa[P], pb[P];
      chunk_parts<P, M, T>(f, bd, pa, pb);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        rhol[a * 256 + t] = pa[a];
        rhol[(P + a) * 256 + t] = pb[a];
      }
    }
    __syncthreads();
    if (active) {
      // rho_j = pa_j - pb_{j+1} for the chunks j = k + dlo + u of this row;
      // struct-of-arrays LDS rows keep lanes on distinct banks, and the loop
      // is unrolled by four so LDS latency overlaps
      T acc[P];
#pragma unroll
      for (int a = 0; a < P; ++a) acc[a] = 0;
      const int rs = r * S;
      int u = 0;
      for (; u + 4 <= dcount; u += 4) {
        T rr2[4][P];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j = wrap_once(k + dlo + u + q, S);
          const int jn = wrap_once(j + 1, S);
#pragma unroll
          for (int a = 0; a < P; ++a)
            rr2[q][a] = rhol[a * 256 + rs + j] - rhol[(P + a) * 256 + rs + jn];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T* B = blocks + (u + q) * 4;
#pragma unroll
          for (int a = 0; a < P; ++a)
#pragma unroll
            for (int c = 0; c < P; ++c) acc[a] = acc[a] + B[a * 2 + c] * rr2[q][c];
        }
      }
      for (; u < dcount; ++u) {
        const int j = wrap_once(k + dlo + u, S);
        const int jn = wrap_once(j + 1, S);
        const T* B = blocks + u * 4;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int c = 0; c < P; ++c)
            acc[a] = acc[a] + B[a * 2 + c] * (rhol[c * 256 + rs + j] - rhol[(P + c) * 256 + rs + jn]);
      }
#pragma unroll
      for (int a = 0; a < P; ++a) sepl[a * 256 + t] = acc[a];
    }
    __syncthreads();
    if (active) {
      const int kp = wrap_once(k - 1, S);
      T sp[P], so[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        sp[a] = sepl[a * 256 + r * S + kp];
        so[a] = sepl[a * 256 + t];
      }
      chunk_correct<P, M, T>(f, rec, sp, so);
#pragma unroll
      for (int p = 0; p < M; ++p) tile[t * (M + 1) + p] = f[p];
    }
    __syncthreads();
    const bool dense_out = ldd == n && contig;
    const bool full = dense_out && nel == 256 * M && ((long)rows - row0) * n >= nel;
    if constexpr (sizeof(Tout) == 4) {
      static_assert(!ACC, "FP32 output does not accumulate");
      if (full) {  // four values per streamed 16-byte store
        float* b = dst + map(row0) * n;
#pragma unroll
        for (int u = 0; u < M / 4; ++u) {
          const int e = 4 * t + 1024 * u;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            __builtin_nontemporal_store((float)tile[e + q + e / M], &b[e + q]);
        }
      }
    } else {
      if (full) {
        double2* b2 = reinterpret_cast<double2*>(dst + map(row0) * n);
#pragma unroll
        for (int u = 0; u < M / 2; ++u) {
          const int e = 2 * t + 512 * u;
          double2 v;
          v.x = (double)tile[e + e / M];
          v.y = (double)tile[e + 1 + e / M];
          if (ACC) {
            const double2 o = b2[t + 256 * u];
            v.x += o.x;
            v.y += o.y;
          }
          store_stream(b2 + t + 256 * u, v);  // streamed: not re-read before the next pass
        }
      }
    }
    if (!full && dense_out) {
      const long nvalid = ((long)rows - row0) * n;
      Tout* base = dst + map(row0) * n;
#pragma unroll
      for (int u = 0; u < M; ++u) {
        const int e = t + 256 * u;
        if (e < nel && e < nvalid) {
          if (ACC) base[e] += (Tout)tile[e + e / M];
          else base[e] = (Tout)tile[e + e / M];
        }
      }
    } else if (!full) {
#pragma unroll 1
      for (int u = 0; u < M; ++u) {
        const int e = t + 256 * u;
        const int rr = e / n;
        const int i = e - rr * n;
        if (e < nel && row0 + rr < rows) {
          if (ACC) dst[map(row0 + rr) * ldd + i] += (Tout)tile[e + e / M];
          else dst[map(row0 + rr) * ldd + i] = (Tout)tile[e + e / M];
        }
      }
    }
    __syncthreads();
  }
}

template <int P, int M, typename T, bool ACC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void row_solve_lds(
    const double* src, long lds, double* dst, long ldd, int rows, int n, int S, int R,
    const T* __restrict__ rec, BandT<T> bd, const T* __restrict__ blocks, int dlo, int dcount) {
  __shared__ RowLds<P, M, T> sh;
  row_solve_body<P, M, T, ACC>(src, lds, dst, ldd, rows, n, S, R, rec, bd, blocks, dlo, dcount,
                               (long)blockIdx.x * R, sh);
}

// Dense rows in whole groups take the half-tile row kernels.
constexpr bool kRowsHalfTile = true;

// Dense rows in whole groups (R = 256 / S rows of n = S M points per
// workgroup, rows % R == 0, ld == n): the same solve as row_solve_body,
// staged through an LDS tile of HALF the group.  All of the group's loads
// are issued up front into registers; the first half of the group (chunks
// 0..127) goes through the tile to threads 0..127, then the second half to
// threads 128..255, and the output leaves the same way in two halves.  At
// M = 32, 46 KB of LDS instead of 80 KB: three groups per CU instead of two,
// so more of HBM's latency is covered (three more barriers per group).
// Arithmetic identical to row_solve_body (bitwise equal results).  NTL:
// the group streams in with non-temporal loads (the standalone solves; in
// the ADI step they slowed the row pass more than they sped up the column
// pass that follows it: 0.182 -> 0.216 and 0.216 -> 0.198 ms at 8192^2).
template <int P, int M, bool NTL = false>
__device__ __forceinline__ void row_half_body(double* xg, int S, const double* __restrict__ rec,
                                              const BandT<double>& bd,
                                              const double* __restrict__ blocks, int dlo,
                                              int dcount) {
  constexpr int H = 128;  // chunks per half
  __shared__ double tile[H * (M + 1)];
  __shared__ double rhol[256 * 2 * P];
  __shared__ double sepl[256 * P];
  const int t = threadIdx.x;
  const int r = t / S, k = t - r * S, rs = r * S;  // row in the group, chunk in the row
  double2* b2 = reinterpret_cast<double2*>(xg);
  double2 vin[M / 2];
#pragma unroll
  for (int u = 0; u < M / 2; ++u) {
    if constexpr (NTL) {
      typedef double dv2 __attribute__((ext_vector_type(2)));
      const dv2 w = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(b2 + t + 256 * u));
      vin[u].x = w.x;
      vin[u].y = w.y;
    } else {
      vin[u] = b2[t + 256 * u];
    }
  }
  // element e = 2t + 512u of the group lies in half u / (M/4); within its
  // half at e' = e - half NG/2, LDS slot e' + e' / M
  double f[M];
#pragma unroll
  for (int half = 0; half < 2; ++half) {
#pragma unroll
    for (int u = half * (M / 4); u < (half + 1) * (M / 4); ++u) {
      const int e = 2 * t + 512 * (u - half * (M / 4));
      tile[e + e / M] = vin[u].x;
      tile[e + 1 + e / M] = vin[u].y;
    }
    __syncthreads();
    if ((t >= H) == (half == 1)) {
      const int tl = t - half * H;
#pragma unroll
      for (int p = 0; p < M; ++p) f[p] = tile[tl * (M + 1) + p];
    }
    __syncthreads();
  }
  chunk_sweep<P, M, double>(f, rec, bd.c[0]);
  {
    double pa[P], pb[P];
    chunk_parts<P, M, double>(f, bd, pa, pb);
#pragma unroll
    for (int a = 0; a < P; ++a) {
      rhol[a * 256 + t] = pa[a];
      rhol[(P + a) * 256 + t] = pb[a];
    }
  }
  __syncthreads();
  {
    // rho_j = pa_j - pb_{j+1} for the chunks j = k + dlo + u of this row, in
    // the order of row_solve_body (four at a time, then the rest)
    double acc[P];
#pragma unroll
    for (int a = 0; a < P; ++a) acc[a] = 0;
    int u = 0;
    for (; u + 4 <= dcount; u += 4) {
      double rr2[4][P];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = wrap_once(k + dlo + u + q, S);
        const int jn = wrap_once(j + 1, S);
#pragma unroll
        for (int a = 0; a < P; ++a)
          rr2[q][a] = rhol[a * 256 + rs + j] - rhol[(P + a) * 256 + rs + jn];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double* B = blocks + (u + q) * 4;
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int c = 0; c < P; ++c) acc[a] = acc[a] + B[a * 2 + c] * rr2[q][c];
      }
    }
    for (; u < dcount; ++u) {
      const int j = wrap_once(k + dlo + u, S);
      const int jn = wrap_once(j + 1, S);
      const double* B = blocks + u * 4;
#pragma unroll
      for (int a = 0; a < P; ++a)
#pragma unroll
        for (int c = 0; c < P; ++c)
          acc[a] = acc[a] + B[a * 2 + c] * (rhol[c * 256 + rs + j] - rhol[(P + c) * 256 + rs + jn]);
    }
#pragma unroll
    for (int a = 0; a < P; ++a) sepl[a * 256 + t] = acc[a];
  }
  __syncthreads();
  {
    const int kp = wrap_once(k - 1, S);
    double sp[P], so[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      sp[a] = sepl[a * 256 + rs + kp];
      so[a] = sepl[a * 256 + t];
    }
    chunk_correct<P, M, double>(f, rec, sp, so);
  }
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    if ((t >= H) == (half == 1)) {
      const int tl = t - half * H;
#pragma unroll
      for (int p = 0; p < M; ++p) tile[tl * (M + 1) + p] = f[p];
    }
    __syncthreads();
#pragma unroll
    for (int u = half * (M / 4); u < (half + 1) * (M / 4); ++u) {
      const int e = 2 * t + 512 * (u - half * (M / 4));
      double2 v;
      v.x = tile[e + e / M];
      v.y = tile[e + 1 + e / M];
      store_stream(b2 + t + 256 * u, v);  // streamed: not re-read before the next pass
    }
    if (half == 0) __syncthreads();
  }
}

template <int P, int M, bool NTL = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void row_solve_half(
    double* x, int S, const double* __restrict__ rec, BandT<double> bd,
    const double* __restrict__ blocks, int dlo, int dcount) {
  row_half_body<P, M, NTL>(x + (long)blockIdx.x * (256 * M), S, rec, bd, blocks, dlo, dcount);
}

// FP32 rows in, FP32 rows out (the refined step's row solves of its FP32
// chunk-solved columns).
template <int P, int M>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void row_solve_lds_f32(
    const float* src, long lds, float* dst, long ldd, int rows, int n, int S, int R,
    const float* __restrict__ rec, BandT<float> bd, const float* __restrict__ blocks, int dlo,
    int dcount) {
  __shared__ RowLds<P, M, float> sh;
  row_solve_body<P, M, float, false, float, float>(src, lds, dst, ldd, rows, n, S, R, rec, bd,
                                                   blocks, dlo, dcount, (long)blockIdx.x * R, sh);
}

// Fixed-order sum of dnparts (mass, energy) partial pairs by one block of at
// least 256 threads: a 256-way split and tree whatever the block size, so the
// order (and rounding) of the sum never depends on the kernel's tile shape.
__device__ __forceinline__ void diag_tail_sum(const double* __restrict__ dpart, long dnparts,
                                              double dscale, double* __restrict__ dout,
                                              double* sm2) {
  __syncthreads();
  constexpr int nt = 256;
  if ((int)threadIdx.x < nt) {
    const long per = (dnparts + nt - 1) / nt;
    const long b0 = (long)threadIdx.x * per;
    const long b1 = (b0 + per < dnparts) ? b0 + per : dnparts;
    double m = 0.0, e = 0.0;
    long b = b0;
    // batches of 32 (a 8192^2 step's whole share) and then of 8 pairs,
    // every batch's loads issued before its adds; the adds keep their
    // order, so the sum does not depend on the batching
    for (; b + 32 <= b1; b += 32) {
      double2 q[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) q[u] = reinterpret_cast<const double2*>(dpart)[b + u];
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        m += q[u].x;
        e += q[u].y;
      }
    }
    for (; b + 8 <= b1; b += 8) {
      double2 q[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) q[u] = reinterpret_cast<const double2*>(dpart)[b + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        m += q[u].x;
        e += q[u].y;
      }
    }
    for (; b < b1; ++b) {
      m += dpart[2 * b];
      e += dpart[2 * b + 1];
    }
    sm2[threadIdx.x] = m;
    sm2[nt + threadIdx.x] = e;
  }
  __syncthreads();
  for (int h = nt / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sm2[threadIdx.x] += sm2[threadIdx.x + h];
      sm2[nt + threadIdx.x] += sm2[nt + threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dout[0] = sm2[0] * dscale;
    dout[1] = sm2[nt] * dscale;
  }
}

// Reduced separator system with an LDS window: a block (W waves) owns 64
// systems and KB = W G consecutive chunks; it stages rho_j = pa_j - pb_{j+1}
// for the KB + dcount - 1 chunks its convolutions touch (U window entries
// per wave in flight at once), then each wave computes G consecutive chunks
// at once, reading every window entry from LDS a single time (register
// blocking).  Every output sums its dcount terms in the same order whatever
// (W, G, U), so all shapes give bitwise identical results.  Block (0,0) can
// also finish a fixed-order sum of per-block (mass, energy) partials
// (dout != nullptr).
template <int P, typename T, typename Td, int W, int G, int U>
__device__ __forceinline__ void reduced_body(const T* __restrict__ rho, int batch, int S,
                                             const T* __restrict__ blocks, int dlo, int dcount,
                                             Td* __restrict__ dst, long ld, int drow_stride,
                                             int drow_off, const double* __restrict__ dpart,
                                             long dnparts, double dscale,
                                             double* __restrict__ dout, int bx, int by,
                                             unsigned char* smraw) {
  constexpr int KB = W * G;
  T* sm = reinterpret_cast<T*>(smraw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long s = (long)bx * 64 + lane;
  const int k0 = by * KB;
  const int nwin = KB + dcount - 1;
  const bool sv = s < batch;
  // Every load of a pass is issued before any result is used: an entry past
  // the window re-reads the last one and a system past the batch re-reads the
  // last system (both in bounds, neither stored), so no load sits behind a
  // branch and the U * 2P loads of a lane are in flight together.
  const long sl = sv ? s : (long)batch - 1;
  for (int w0 = wave; w0 < nwin; w0 += W * U) {
    T v[U][P];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int w = min(w0 + W * u, nwin - 1);
      int j = (k0 + dlo + w) % S;
      j += (j < 0) ? S : 0;
      const int jn = (j + 1 == S) ? 0 : j + 1;
#pragma unroll
      for (int a = 0; a < P; ++a)
        v[u][a] = rho[((long)j * 2 * P + a) * batch + sl] -
                  rho[((long)jn * 2 * P + P + a) * batch + sl];
    }
    // keeps the compiler from sinking an entry's loads into the branch of
    // its LDS store below, which would wait on them one entry at a time
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int a = 0; a < P; ++a) asm volatile("" : "+v"(v[u][a]));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int w = w0 + W * u;
      if (w < nwin) {
#pragma unroll
        for (int a = 0; a < P; ++a) sm[(w * P + a) * 64 + lane] = v[u][a];
      }
    }
  }
  __syncthreads();
  const int kk0 = wave * G;  // first chunk (within the block) of this wave
  if (sv && k0 + kk0 < S) {
    T acc[G][P];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int a = 0; a < P; ++a) acc[g][a] = 0;
    // Output g takes block t against window entry kk0 + g + t, t ascending;
    // win[g] holds that entry, so the G entries slide one place per block and
    // every entry is read from LDS once.
    T win[G][P];
#pragma unroll
    for (int g = 0; g + 1 < G; ++g)
#pragma unroll
      for (int c = 0; c < P; ++c) win[g + 1][c] = sm[((kk0 + g) * P + c) * 64 + lane];
#pragma unroll 4
    for (int t = 0; t < dcount; ++t) {
#pragma unroll
      for (int g = 0; g + 1 < G; ++g)
#pragma unroll
        for (int c = 0; c < P; ++c) win[g][c] = win[g + 1][c];
#pragma unroll
      for (int c = 0; c < P; ++c) win[G - 1][c] = sm[((kk0 + t + G - 1) * P + c) * 64 + lane];
      const T* B = blocks + t * 4;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int c = 0; c < P; ++c) acc[g][a] = acc[g][a] + B[a * 2 + c] * win[g][c];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k = k0 + kk0 + g;
      if (k < S) {
#pragma unroll
        for (int a = 0; a < P; ++a)
          dst[((long)k * drow_stride + drow_off + a) * ld + s] = (Td)acc[g][a];
      }
    }
  }
  if (dout != nullptr) diag_tail_sum(dpart, dnparts, dscale, dout, reinterpret_cast<double*>(smraw));
}

template <int P, typename T, typename Td, int W, int G, int U>
__global__ __launch_bounds__(64 * W) void reduced_il_lds(const T* __restrict__ rho, int batch,
                                                         int S, const T* __restrict__ blocks,
                                                         int dlo, int dcount, Td* __restrict__ dst,
                                                         long ld, int drow_stride, int drow_off,
                                                         const double* __restrict__ dpart,
                                                         long dnparts, double dscale,
                                                         double* __restrict__ dout) {
  extern __shared__ unsigned char smraw[];
  const bool first = blockIdx.x == 0 && blockIdx.y == 0;
  reduced_body<P, T, Td, W, G, U>(rho, batch, S, blocks, dlo, dcount, dst, ld, drow_stride,
                                  drow_off, dpart, dnparts, dscale, first ? dout : nullptr,
                                  blockIdx.x, blockIdx.y, smraw);
}

// Whole-column form of the same convolution: a block owns L systems and all
// S chunks of them, so every rho_j is loaded once (the windowed form loads
// each KB + dcount - 1 times per KB chunks) and the periodic window wraps
// inside LDS.  Thread (c, q) = (threadIdx.x % L, threadIdx.x / L) stages
// entries q, q + NQ, ... and computes chunks q G .. q G + G - 1 of system c,
// each summing its dcount terms in the windowed form's order (bitwise equal).
template <int P, typename T, typename Td, int L, int G>
__global__ __launch_bounds__(1024) void reduced_whole(const T* __restrict__ rho, int batch, int S,
                                                      const T* __restrict__ blocks, int dlo,
                                                      int dcount, Td* __restrict__ dst, long ld,
                                                      int drow_stride, int drow_off,
                                                      const double* __restrict__ dpart,
                                                      long dnparts, double dscale,
                                                      double* __restrict__ dout) {
  extern __shared__ unsigned char smraw[];
  T* sm = reinterpret_cast<T*>(smraw);
  const int NQ = (S + G - 1) / G;  // chunk groups, one per L threads
  const int c = threadIdx.x % L, q = threadIdx.x / L;
  const long s = (long)blockIdx.x * L + c;
  const bool sv = s < batch;
  const long sl = sv ? s : (long)batch - 1;
  if (q < NQ) {
    // G passes of NQ entries cover the S chunks; an entry past S re-reads
    // chunk S - 1 (not stored), so all loads issue before any is used
    T v[G][P];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int j = min(q + NQ * u, S - 1);
      const int jn = (j + 1 == S) ? 0 : j + 1;
#pragma unroll
      for (int a = 0; a < P; ++a)
        v[u][a] = rho[((long)j * 2 * P + a) * batch + sl] -
                  rho[((long)jn * 2 * P + P + a) * batch + sl];
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
      for (int a = 0; a < P; ++a) asm volatile("" : "+v"(v[u][a]));
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int j = q + NQ * u;
      if (j < S) {
#pragma unroll
        for (int a = 0; a < P; ++a) sm[(j * P + a) * L + c] = v[u][a];
      }
    }
  }
  __syncthreads();
  const int k0 = q * G;
  if (sv && k0 < S) {
    T acc[G][P];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int a = 0; a < P; ++a) acc[g][a] = 0;
    // output g takes block t against chunk (k0 + g + dlo + t) mod S; win[g]
    // holds that entry and idx is the chunk entering the window next
    int idx = (k0 + dlo) % S;
    idx += (idx < 0) ? S : 0;
    T win[G][P];
#pragma unroll
    for (int g = 0; g + 1 < G; ++g) {
#pragma unroll
      for (int a = 0; a < P; ++a) win[g + 1][a] = sm[(idx * P + a) * L + c];
      idx = (idx + 1 == S) ? 0 : idx + 1;
    }
#pragma unroll 4
    for (int t = 0; t < dcount; ++t) {
#pragma unroll
      for (int g = 0; g + 1 < G; ++g)
#pragma unroll
        for (int a = 0; a < P; ++a) win[g][a] = win[g + 1][a];
#pragma unroll
      for (int a = 0; a < P; ++a) win[G - 1][a] = sm[(idx * P + a) * L + c];
      idx = (idx + 1 == S) ? 0 : idx + 1;
      const T* B = blocks + t * 4;
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int a = 0; a < P; ++a)
#pragma unroll
          for (int b = 0; b < P; ++b) acc[g][a] = acc[g][a] + B[a * 2 + b] * win[g][b];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int k = k0 + g;
      if (k < S) {
#pragma unroll
        for (int a = 0; a < P; ++a)
          dst[((long)k * drow_stride + drow_off + a) * ld + s] = (Td)acc[g][a];
      }
    }
  }
  if (dout != nullptr && blockIdx.x == 0)
    diag_tail_sum(dpart, dnparts, dscale, dout, reinterpret_cast<double*>(smraw));
}

template <typename T>
static BandT<T> band_of(const double* coef) {
  BandT<T> bd;
  for (int i = 0; i < 5; ++i) bd.c[i] = (T)coef[i];
  return bd;
}

// ---------------------------------------------------------------------------
// Batched 1D periodic schemes (Ch.4 eq. disc, Ch.5 eq. 5:1ddiffscheme,
// Ch.6 eq. 6:1Dnumerical): the right-hand side of each step is a 3- or
// 5-point stencil of the state, so the first pass of the chunked solve forms
// it on the fly from the interleaved state (rows k M - 2 .. k M + M + 1 of
// each 64-system segment) and sweeps the chunk interior in registers.
template <int KIND>
__device__ __forceinline__ double b1d_rhs(const double* X, int q, double s, double al) {
  if (KIND == 0)
    return -s * X[q - 2] + 4.0 * s * X[q - 1] + (1.0 - 6.0 * s) * X[q] + 4.0 * s * X[q + 1] -
           s * X[q + 2];
  if (KIND == 1) return s * X[q - 1] + (1.0 - 2.0 * s) * X[q] + s * X[q + 1];
  const double ml = X[q - 1] * X[q - 1] * X[q - 1] - X[q - 1];
  const double mc = X[q] * X[q] * X[q] - X[q];
  const double mr = X[q + 1] * X[q + 1] * X[q + 1] - X[q + 1];
  return X[q] + al * (ml - 2.0 * mc + mr);
}

// RECON: src is the previous step's half-solved buffer (chunk interiors
// uncorrected, separator rows final) and each value is corrected as it is
// loaded, x = y - Zl s_prev - Zr s_own, so no separate correction pass runs
// between steps.
template <int P, int M>
__device__ __forceinline__ double b1d_recon(double v, int p, const double* __restrict__ rec,
                                            const double (&sp)[2], const double (&so)[2]) {
  if (p >= M - P) return v;
#pragma unroll
  for (int a = 0; a < P; ++a) v = v - rec[p * 8 + 4 + a] * sp[a] - rec[p * 8 + 6 + a] * so[a];
  return v;
}

template <int KIND, int P, int M, bool RECON>
__global__ __launch_bounds__(256) void batch1d_sweep(const double* __restrict__ x, long ld,
                                                     double* __restrict__ y, long ldy, int batch,
                                                     int n, int S, const double* __restrict__ rec,
                                                     BandT<double> bd, double* __restrict__ rho,
                                                     double s, double al) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long sys = (long)blockIdx.x * 64 + lane;
  const int k = blockIdx.y * 4 + wave;
  if (sys >= batch || k >= S) return;
  constexpr int MI = M - P;
  double sm[2] = {0, 0}, sk[2] = {0, 0}, skp[2] = {0, 0};  // separators of chunks k-1, k, k+1
  if (RECON) {
    const int km = (k == 0) ? S - 1 : k - 1, kp = (k + 1 == S) ? 0 : k + 1;
#pragma unroll
    for (int a = 0; a < P; ++a) {
      sm[a] = x[((long)km * M + MI + a) * ld + sys];
      sk[a] = x[((long)k * M + MI + a) * ld + sys];
      skp[a] = x[((long)kp * M + MI + a) * ld + sys];
    }
  }
  double X[M + 4];
#pragma unroll
  for (int q = 0; q < M + 4; ++q) {
    int row = k * M - 2 + q;
    row += (row < 0) ? n : 0;
    row -= (row >= n) ? n : 0;
    // non-temporal, as in the standalone solve's passes (measured: the
    // 65536 x 1024 hyperdiffusion batch 0.236 -> 0.224 ms per step)
    double v = __builtin_nontemporal_load(&x[(long)row * ld + sys]);
    if (RECON) {
      // q = 0, 1: the last two rows of chunk k-1 (separators for P = 2; for
      // P = 1 the first of them is never used); q = 2 .. M+1: chunk k;
      // q = M+2, M+3: rows 0, 1 of chunk k+1
      if (q >= 2 && q < M + 2) v = b1d_recon<P, M>(v, q - 2, rec, sm, sk);
      else if (q >= M + 2) v = b1d_recon<P, M>(v, q - M - 2, rec, sk, skp);
    }
    X[q] = v;
  }
  double f[M];
#pragma unroll
  for (int p = 0; p < M; ++p) f[p] = b1d_rhs<KIND>(X, p + 2, s, al);
  chunk_sweep<P, M, double>(f, rec, bd.c[0]);
  double pa[P], pb[P];
  chunk_parts<P, M, double>(f, bd, pa, pb);
  double* yb = y + (long)k * M * ldy + sys;
#pragma unroll
  for (int p = 0; p < M - P; ++p) __builtin_nontemporal_store(f[p], &yb[(long)p * ldy]);
#pragma unroll
  for (int a = 0; a < P; ++a) {
    rho[((long)k * 2 * P + a) * batch + sys] = pa[a];
    rho[((long)k * 2 * P + P + a) * batch + sys] = pb[a];
  }
}

// Lengths without the chunked plan: the right-hand side alone, one thread
// per (system, unknown), into y (pitch ldy).
template <int KIND>
__global__ __launch_bounds__(256) void batch1d_rhs(const double* __restrict__ x, long ld,
                                                   double* __restrict__ y, long ldy, int batch,
                                                   int n, double s, double al) {
  const long sys = (long)blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (sys >= batch) return;
  double X[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    int row = i - 2 + q;
    row = (row % n + n) % n;
    X[q] = x[(long)row * ld + sys];
  }
  y[(long)i * ldy + sys] = b1d_rhs<KIND>(X, 2, s, al);
}

hipError_t launch_batch1d_rhs(int kind, const double* x, long ld, double* y, long ldy, int batch,
                              int n, double s, double al, hipStream_t st) {
  dim3 grid((batch + 255) / 256, n);
  if (kind == 0)
    hipLaunchKernelGGL(batch1d_rhs<0>, grid, dim3(256), 0, st, x, ld, y, ldy, batch, n, s, al);
  else if (kind == 1)
    hipLaunchKernelGGL(batch1d_rhs<1>, grid, dim3(256), 0, st, x, ld, y, ldy, batch, n, s, al);
  else
    hipLaunchKernelGGL(batch1d_rhs<2>, grid, dim3(256), 0, st, x, ld, y, ldy, batch, n, s, al);
  return hipGetLastError();
}

hipError_t launch_batch1d_steps(int kind, bool chunked, const DevChunk& c, const DevWhole& w,
                                double* x, long ld, int batch, int n, double s, double al,
                                int nsteps, double* y0, double* y1, double* rho, hipStream_t st) {
  const int P = kind == 1 ? 1 : 2;
  hipError_t e = hipSuccess;
  if (chunked) {
    // step j sweeps buf[j & 1] from x (j = 0) or from buf[(j-1) & 1] with
    // the deferred correction; the last buffer is corrected into x at the end
    dim3 grid((batch + 63) / 64, (c.S + 3) / 4);
    const BandT<double> bd = band_of<double>(c.coef);
    double* buf[2] = {y0, y1};
    for (int j = 0; j < nsteps && e == hipSuccess; ++j) {
      const double* src = j == 0 ? x : buf[(j - 1) & 1];
      const long lsrc = j == 0 ? ld : (long)batch;
      double* dst = buf[j & 1];
#define CHX_B1D(K_, P_, R_)                                                                      \
  hipLaunchKernelGGL((batch1d_sweep<K_, P_, kChunk, R_>), grid, dim3(256), 0, st, src, lsrc, dst, \
                     (long)batch, batch, n, c.S, c.rec, bd, rho, s, al)
      if (j == 0) {
        if (kind == 0) CHX_B1D(0, 2, false);
        else if (kind == 1) CHX_B1D(1, 1, false);
        else CHX_B1D(2, 2, false);
      } else {
        if (kind == 0) CHX_B1D(0, 2, true);
        else if (kind == 1) CHX_B1D(1, 1, true);
        else CHX_B1D(2, 2, true);
      }
#undef CHX_B1D
      e = hipGetLastError();
      if (e == hipSuccess)
        e = P == 2 ? launch_reduced_il<2>(c, rho, batch, dst, batch, kChunk, kChunk - 2, st)
                   : launch_reduced_il<1>(c, rho, batch, dst, batch, kChunk, kChunk - 1, st);
    }
    if (e != hipSuccess) return e;
    const double* last = buf[(nsteps - 1) & 1];
    if (P == 2)
      hipLaunchKernelGGL((correct_il<2, kChunk, double, double, false>), grid, dim3(256), 0, st,
                         last, (long)batch, x, ld, batch, c.S, c.rec);
    else
      hipLaunchKernelGGL((correct_il<1, kChunk, double, double, false>), grid, dim3(256), 0, st,
                         last, (long)batch, x, ld, batch, c.S, c.rec);
    return hipGetLastError();
  }
  dim3 grid((batch + 255) / 256, n);
  for (int j = 0; j < nsteps && e == hipSuccess; ++j) {
    if (kind == 0)
      hipLaunchKernelGGL(batch1d_rhs<0>, grid, dim3(256), 0, st, x, ld, y0, (long)batch, batch, n, s, al);
    else if (kind == 1)
      hipLaunchKernelGGL(batch1d_rhs<1>, grid, dim3(256), 0, st, x, ld, y0, (long)batch, batch, n, s, al);
    else
      hipLaunchKernelGGL(batch1d_rhs<2>, grid, dim3(256), 0, st, x, ld, y0, (long)batch, batch, n, s, al);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = P == 2 ? launch_whole<2>(w, y0, 1, batch, batch, st)
                 : launch_whole<1>(w, y0, 1, batch, batch, st);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(x, ld * sizeof(double), y0, (size_t)batch * sizeof(double),
                           (size_t)batch * sizeof(double), n, hipMemcpyDeviceToDevice, st);
  }
  return e;
}

// ---------------------------------------------------------------------------
// Split row pass, for rows of 4096 or 8192 points (R = 2 or 1 rows per
// group).  Only the separator rows (the last P rows of every 32-row column
// chunk) need the column separators; every other row can be row-solved while
// the separators are being computed.  rows_split_fused does both in one
// launch: blocks [0, nred) run the separator convolution (4 waves, the row
// group's LDS tile reused as the window), the others solve interior row
// groups; rows_sep then solves the separator rows.  The two sets of rows are
// disjoint, and each row is solved by the same code as in the plain pass, so
// results are bitwise identical to it.
__device__ __forceinline__ long split_row0(long g, int R, bool sep) {
  const int gper = (sep ? 2 : kChunk - 2) / R;
  return kChunk * (g / gper) + (sep ? kChunk - 2 : 0) + R * (g % gper);
}

template <int G, int U>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void rows_split_fused(
    const double* __restrict__ rho, DevChunk cy, double* x, int nx, int ny, DevChunk cx,
    BandT<double> bdx, int nred, int nbx, const double* __restrict__ dpart, long dnparts,
    double dscale, double* __restrict__ dout) {
  __shared__ RowLds<2, kChunk, double> sh;
  const int b = blockIdx.x;
  if (b < nred) {
    reduced_body<2, double, double, 4, G, U>(rho, nx, cy.S, cy.blocks, cy.dlo, cy.dcount, x, nx,
                                             kChunk, kChunk - 2, dpart, dnparts, dscale,
                                             b == 0 ? dout : nullptr, b % nbx, b / nbx,
                                             reinterpret_cast<unsigned char*>(sh.tile));
  } else {
    const int R = 256 / cx.S;
    row_solve_body<2, kChunk, double, false>(x, nx, x, nx, ny, nx, cx.S, R, cx.rec, bdx,
                                             cx.blocks, cx.dlo, cx.dcount,
                                             split_row0(b - nred, R, false), sh);
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void rows_sep(
    double* x, int nx, int ny, DevChunk cx, BandT<double> bdx) {
  __shared__ RowLds<2, kChunk, double> sh;
  const int R = 256 / cx.S;
  row_solve_body<2, kChunk, double, false>(x, nx, x, nx, ny, nx, cx.S, R, cx.rec, bdx, cx.blocks,
                                           cx.dlo, cx.dcount, split_row0(blockIdx.x, R, true),
                                           sh);
}


// The separator rows (SEP) or the interior rows of a step whose columns are
// chunked by Mc rows, for any row plan: groups of R = 256 / S consecutive
// rows of the subset (a group may span two column chunks; rows are
// independent).  Used by the overlapped row order: the interior rows need no
// column separator, so they are solved on one stream while the separators
// and then the separator rows are formed on another.
template <bool SEP, int M>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void rows_subset(
    double* x, int nx, int ny, int Mc, DevChunk cx, BandT<double> bdx) {
  __shared__ RowLds<2, M, double> sh;
  const int R = 256 / cx.S;
  const int per = SEP ? 2 : Mc - 2;
  const SubsetRows map{Mc, per, SEP ? Mc - 2 : 0};
  const int count = (ny / Mc) * per;
  row_solve_body<2, M, double, false, double, double, SubsetRows>(
      x, nx, x, nx, count, nx, cx.S, R, cx.rec, bdx, cx.blocks, cx.dlo, cx.dcount,
      (long)blockIdx.x * R, sh, map);
}

hipError_t launch_rows_subset(bool sep, double* x, int nx, int ny, int Mc, const DevChunk& cx,
                              hipStream_t st) {
  if (cx.S > 256 || ny % Mc != 0 || (cx.M != kChunk && cx.M != 16)) return hipErrorInvalidValue;
  const int R = 256 / cx.S;
  const long count = (long)(ny / Mc) * (sep ? 2 : Mc - 2);
  const dim3 grid((unsigned)((count + R - 1) / R));
  const BandT<double> bd = band_of<double>(cx.coef);
#define CHX_SUB(S_, M_) \
  hipLaunchKernelGGL((rows_subset<S_, M_>), grid, dim3(256), 0, st, x, nx, ny, Mc, cx, bd)
  if (sep) {
    if (cx.M == 16) CHX_SUB(true, 16);
    else CHX_SUB(true, kChunk);
  } else {
    if (cx.M == 16) CHX_SUB(false, 16);
    else CHX_SUB(false, kChunk);
  }
#undef CHX_SUB
  return hipGetLastError();
}

// (chunks per wave, window entries staged at once) of the fused kernel's
// separator part.
constexpr int kSplitG[kNumSplitShapes] = {8, 8, 4};

bool split_fits(const DevChunk& cy, const DevChunk& cx, int shape) {
  if (shape < 0 || shape >= kNumSplitShapes) return false;
  if (cx.S != 128 && cx.S != 256) return false;
  const size_t win = (size_t)(4 * kSplitG[shape] + cy.dcount - 1) * 2 * 64 * sizeof(double);
  return win <= sizeof(RowLds<2, kChunk, double>::tile) && cy.dcount <= cy.S;
}

hipError_t launch_rows_split_fused(int shape, const DevChunk& cy, const double* rho, double* x,
                                   int nx, int ny, const DevChunk& cx, const double* dpart,
                                   long dnparts, double dscale, double* dout, hipStream_t st) {
  if (!split_fits(cy, cx, shape)) return hipErrorInvalidValue;
  const int R = 256 / cx.S;
  const int nbx = (nx + 63) / 64;
  const int kb = 4 * kSplitG[shape];
  const int nred = nbx * ((cy.S + kb - 1) / kb);
  const long nint = (long)(ny / kChunk) * ((kChunk - 2) / R);
  const BandT<double> bdx = band_of<double>(cx.coef);
  const dim3 grid((unsigned)(nred + nint));
#define CHX_SPLIT(G_, U_)                                                                        \
  hipLaunchKernelGGL((rows_split_fused<G_, U_>), grid, dim3(256), 0, st, rho, cy, x, nx, ny, cx, \
                     bdx, nred, nbx, dpart, dnparts, dscale, dout)
  switch (shape) {
    case 0: CHX_SPLIT(8, 4); break;
    case 1: CHX_SPLIT(8, 8); break;
    default: CHX_SPLIT(4, 4); break;
  }
#undef CHX_SPLIT
  return hipGetLastError();
}


hipError_t launch_rows_sep(double* x, int nx, int ny, const DevChunk& cx, hipStream_t st) {
  const int R = 256 / cx.S;
  const dim3 grid((unsigned)((ny / kChunk) * (2 / R)));
  hipLaunchKernelGGL(rows_sep, grid, dim3(256), 0, st, x, nx, ny, cx, band_of<double>(cx.coef));
  return hipGetLastError();
}

// The ensemble's separator kernel uses one fixed shape (runs of several
// classes share the launch).
constexpr int kRedWaves = 8;
constexpr int kRedG = 4;
constexpr int kRedKB = kRedWaves * kRedG;

// ---------------------------------------------------------------------------
// Ensemble kernels: block = work item {run, a, b}; buffers by step parity.
// Tile shapes (waves per block, chunks per wave) of the FP64 ensemble's
// separator kernel; ch_ensemble_create times them on the ensemble's runs.
struct EnsRedShape {
  int W, G;
};
constexpr EnsRedShape kEnsRedShapes[kNumEnsRedShapes] = {{8, 4}, {8, 1}, {4, 2}, {4, 4}};

int ens_red_chunks_per_block(int shape) {
  const EnsRedShape& r = kEnsRedShapes[(shape < 0 || shape >= kNumEnsRedShapes) ? 0 : shape];
  return r.W * r.G;
}

template <int W, int G>
__global__ __launch_bounds__(64 * W) void ens_reduced_k(const EnsRun* __restrict__ runs,
                                                        EnsClasses cls,
                                                        const int4* __restrict__ items,
                                                        unsigned char* ws, int step,
                                                        double* diag_out, long diag_stride) {
  const int4 it = items[blockIdx.x];
  const EnsRun& R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].py;
  double* dst = reinterpret_cast<double*>(ws + ((step & 1) ? R.off_b1 : R.off_b0));
  const double* rho = reinterpret_cast<const double*>(ws + R.off_rho);
  const double* part = reinterpret_cast<const double*>(ws + R.off_part);
  double* dout = (diag_out != nullptr && it.y == 0 && it.z == 0)
                     ? diag_out + it.x * diag_stride + 2 * (long)step
                     : nullptr;
  extern __shared__ unsigned char smraw[];
  reduced_body<2, double, double, W, G, 4>(rho, R.nx, R.Sc, c.blocks, c.dlo, c.dcount, dst, R.nx,
                                           kChunk, kChunk - 2, part, R.ncolblocks,
                                           cls.c[R.cls].K.dxdy, dout, it.y, it.z, smraw);
}

__global__ __launch_bounds__(512) void ens_reduced(const EnsRun* __restrict__ runs,
                                                   EnsClasses cls,
                                                   const int4* __restrict__ items,
                                                   unsigned char* ws, int step, double* diag_out,
                                                   long diag_stride) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].py;
  double* dst = reinterpret_cast<double*>(ws + ((step & 1) ? R.off_b1 : R.off_b0));
  const double* rho = reinterpret_cast<const double*>(ws + R.off_rho);
  const double* part = reinterpret_cast<const double*>(ws + R.off_part);
  double* dout = (diag_out != nullptr && it.y == 0 && it.z == 0)
                     ? diag_out + it.x * diag_stride + 2 * (long)step
                     : nullptr;
  extern __shared__ unsigned char smraw[];
  reduced_body<2, double, double, kRedWaves, kRedG, 4>(rho, R.nx, R.Sc, c.blocks, c.dlo, c.dcount,
                                                      dst, R.nx, kChunk, kChunk - 2, part,
                                                      R.ncolblocks, cls.c[R.cls].K.dxdy, dout,
                                                      it.y, it.z, smraw);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ens_rows(
    const EnsRun* __restrict__ runs, EnsClasses cls,
    const int4* __restrict__ items, unsigned char* ws, int step) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].px;
  BandT<double> bd;
#pragma unroll
  for (int k = 0; k < 5; ++k) bd.c[k] = c.coef[k];
  double* x = reinterpret_cast<double*>(ws + ((step & 1) ? R.off_b1 : R.off_b0));
  __shared__ RowLds<2, kChunk, double> sh;
  row_solve_body<2, kChunk, double, false>(x, R.nx, x, R.nx, R.ny, R.nx, c.S, 256 / c.S, c.rec,
                                           bd, c.blocks, c.dlo, c.dcount,
                                           (long)it.y * (256 / c.S), sh);
}

// The same with the half-tile body, for ensembles whose every run has dense
// rows in whole groups (bitwise equal to ens_rows).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void ens_rows_half(
    const EnsRun* __restrict__ runs, EnsClasses cls, const int4* __restrict__ items,
    unsigned char* ws, int step) {
  const int4 it = items[blockIdx.x];
  const EnsRun& R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].px;
  BandT<double> bd;
#pragma unroll
  for (int k = 0; k < 5; ++k) bd.c[k] = c.coef[k];
  double* x = reinterpret_cast<double*>(ws + ((step & 1) ? R.off_b1 : R.off_b0));
  row_half_body<2, kChunk>(x + (long)it.y * (256 * kChunk), c.S, c.rec, bd, c.blocks, c.dlo,
                           c.dcount);
}

// FP32-refined ensembles: separators of the FP32 column buffer (dout: the
// pass-0 diagnostics of the run's state at `step`), and FP32 row solves of it
// into the run's V_pass.
template <int W, int G>
__global__ __launch_bounds__(64 * W) void ens_reduced32_k(const EnsRun* __restrict__ runs,
                                                          EnsClasses cls,
                                                          const int4* __restrict__ items,
                                                          unsigned char* ws, int step,
                                                          double* diag_out, long diag_stride) {
  const int4 it = items[blockIdx.x];
  const EnsRun& R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].py;
  float* dst = reinterpret_cast<float*>(ws + R.off_y32);
  const float* rho = reinterpret_cast<const float*>(ws + R.off_rho32);
  const double* part = reinterpret_cast<const double*>(ws + R.off_part);
  double* dout = (diag_out != nullptr && it.y == 0 && it.z == 0)
                     ? diag_out + it.x * diag_stride + 2 * (long)step
                     : nullptr;
  extern __shared__ unsigned char smraw[];
  reduced_body<2, float, float, W, G, 4>(rho, R.nx, R.Sc, c.blocks32, c.dlo, c.dcount, dst, R.nx,
                                         kChunk, kChunk - 2, part, R.ncolblocks,
                                         cls.c[R.cls].K.dxdy, dout, it.y, it.z, smraw);
}

__global__ __launch_bounds__(512) void ens_reduced32(const EnsRun* __restrict__ runs,
                                                     EnsClasses cls,
                                                     const int4* __restrict__ items,
                                                     unsigned char* ws, int step, double* diag_out,
                                                     long diag_stride) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].py;
  float* dst = reinterpret_cast<float*>(ws + R.off_y32);
  const float* rho = reinterpret_cast<const float*>(ws + R.off_rho32);
  const double* part = reinterpret_cast<const double*>(ws + R.off_part);
  double* dout = (diag_out != nullptr && it.y == 0 && it.z == 0)
                     ? diag_out + it.x * diag_stride + 2 * (long)step
                     : nullptr;
  extern __shared__ unsigned char smraw[];
  reduced_body<2, float, float, kRedWaves, kRedG, 4>(rho, R.nx, R.Sc, c.blocks32, c.dlo, c.dcount,
                                                    dst, R.nx, kChunk, kChunk - 2, part,
                                                    R.ncolblocks, cls.c[R.cls].K.dxdy, dout,
                                                    it.y, it.z, smraw);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ens_rows32(
    const EnsRun* __restrict__ runs, EnsClasses cls, const int4* __restrict__ items,
    unsigned char* ws, int pass) {
  const int4 it = items[blockIdx.x];
  const EnsRun R = runs[it.x];
  const DevChunk& c = cls.c[R.cls].px;
  BandT<float> bd;
#pragma unroll
  for (int k = 0; k < 5; ++k) bd.c[k] = (float)c.coef[k];
  const float* src = reinterpret_cast<const float*>(ws + R.off_y32);
  // read from the run table, not from the copy R: an index known only at
  // run time would place the whole copy in scratch memory (176 bytes stored
  // and reloaded per thread, more than the thread's share of the rows)
  float* dst = reinterpret_cast<float*>(ws + runs[it.x].off_v[pass]);
  __shared__ RowLds<2, kChunk, float> sh;
  row_solve_body<2, kChunk, float, false, float, float>(src, R.nx, dst, R.nx, R.ny, R.nx, c.S,
                                                        256 / c.S, c.rec32, bd, c.blocks32, c.dlo,
                                                        c.dcount, (long)it.y * (256 / c.S), sh);
}

hipError_t launch_ens_reduced32(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                                int nitems, unsigned char* ws, int step, double* diag_out,
                                long diag_stride, size_t lds_bytes, hipStream_t st, int shape) {
  if (nitems <= 0) return hipSuccess;
#define CHX_ENSRED32(W_, G_)                                                                   \
  hipLaunchKernelGGL((ens_reduced32_k<W_, G_>), dim3(nitems), dim3(64 * W_), lds_bytes, st, \
                     runs, cls, items, ws, step, diag_out, diag_stride)
  switch (shape) {
    case 1: CHX_ENSRED32(8, 1); break;
    case 2: CHX_ENSRED32(4, 2); break;
    case 3: CHX_ENSRED32(4, 4); break;
    default:
      hipLaunchKernelGGL(ens_reduced32, dim3(nitems), dim3(64 * kRedWaves), lds_bytes, st, runs,
                         cls, items, ws, step, diag_out, diag_stride);
  }
#undef CHX_ENSRED32
  return hipGetLastError();
}

hipError_t launch_ens_rows32(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                             int nitems, unsigned char* ws, int pass, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(ens_rows32, dim3(nitems), dim3(256), 0, st, runs, cls, items, ws, pass);
  return hipGetLastError();
}

hipError_t launch_ens_reduced(const EnsRun* runs, const EnsClasses& cls, const int4* items,
                              int nitems, unsigned char* ws, int step, double* diag_out,
                              long diag_stride, size_t lds_bytes, hipStream_t st, int shape) {
#define CHX_ENSRED(W_, G_)                                                                       \
  hipLaunchKernelGGL((ens_reduced_k<W_, G_>), dim3(nitems), dim3(64 * W_), lds_bytes, st, runs, \
                     cls, items, ws, step, diag_out, diag_stride)
  switch (shape) {
    case 1: CHX_ENSRED(8, 1); break;
    case 2: CHX_ENSRED(4, 2); break;
    case 3: CHX_ENSRED(4, 4); break;
    default:
      hipLaunchKernelGGL(ens_reduced, dim3(nitems), dim3(64 * kRedWaves), lds_bytes, st, runs,
                         cls, items, ws, step, diag_out, diag_stride);
  }
#undef CHX_ENSRED
  return hipGetLastError();
}

hipError_t launch_ens_rows(const EnsRun* runs, const EnsClasses& cls, const int4* items, int nitems,
                           unsigned char* ws, int step, hipStream_t st, bool half) {
  if (half && kRowsHalfTile)
    hipLaunchKernelGGL(ens_rows_half, dim3(nitems), dim3(256), 0, st, runs, cls, items, ws, step);
  else
    hipLaunchKernelGGL(ens_rows, dim3(nitems), dim3(256), 0, st, runs, cls, items, ws, step);
  return hipGetLastError();
}

size_t ens_reduced_lds_bytes(int dcount, int shape) {
  const int kb = shape == 0 ? kRedKB : ens_red_chunks_per_block(shape);
  const int threads = 64 * kEnsRedShapes[(shape < 0 || shape >= kNumEnsRedShapes) ? 0 : shape].W;
  size_t lds = (size_t)(kb + dcount - 1) * 2 * 64 * sizeof(double);
  if (lds < 2 * (size_t)threads * sizeof(double)) lds = 2 * (size_t)threads * sizeof(double);
  return lds;
}

// ---------------------------------------------------------------------------
// Launchers


template <int P>
hipError_t launch_whole(const DevWhole& w, double* x, long ss, long es, int batch,
                        hipStream_t st) {
  dim3 grid((batch + 255) / 256);
  hipLaunchKernelGGL((whole_sweep<P, double, false>), grid, dim3(256), 0, st, x, ss, es, x, ss, es,
                     batch, w.n, w.periodic, w.rec, band_of<double>(w.coef), w.minv[0], w.minv[1],
                     w.minv[2], w.minv[3]);
  return hipGetLastError();
}

template <int P>
hipError_t launch_whole32(const DevWhole& w, double* work, long ss, long es, double* out, long oss,
                          long oes, int batch, bool acc, hipStream_t st) {
  dim3 grid((batch + 255) / 256);
  const float m0 = (float)w.minv[0], m1 = (float)w.minv[1], m2 = (float)w.minv[2],
              m3 = (float)w.minv[3];
  if (acc)
    hipLaunchKernelGGL((whole_sweep<P, float, true>), grid, dim3(256), 0, st, work, ss, es, out, oss,
                       oes, batch, w.n, w.periodic, w.rec32, band_of<float>(w.coef), m0, m1, m2,
                       m3);
  else
    hipLaunchKernelGGL((whole_sweep<P, float, false>), grid, dim3(256), 0, st, work, ss, es, out,
                       oss, oes, batch, w.n, w.periodic, w.rec32, band_of<float>(w.coef), m0, m1,
                       m2, m3);
  return hipGetLastError();
}

// Candidate tile shapes of the separator kernel: (waves per block, chunks
// per wave, window entries staged per wave at once), or for the
// whole-column form (L > 0) L systems per block and G chunks per thread.
struct RedShape {
  int W, G, U, L;
};
// (7, 8: larger windows, whose LDS only gfx950's 160 KB holds at the decay
// windows of large grids; 9 .. 11: few chunks per block, for small grids
// where the chunk count is too low to fill the chip with the others;
// 12 .. 14: whole columns, S P L elements of LDS)
constexpr RedShape kRedShapes[kNumRedShapes] = {
    {8, 4, 4, 0},  {8, 4, 8, 0},  {8, 2, 4, 0}, {4, 8, 4, 0},  {4, 8, 8, 0},
    {4, 4, 4, 0},  {16, 2, 4, 0}, {16, 3, 4, 0}, {16, 4, 4, 0}, {4, 1, 8, 0},
    {4, 2, 8, 0},  {8, 1, 8, 0},  {0, 8, 0, 32}, {0, 4, 0, 16}, {0, 8, 0, 16}};

// threads of a whole-column launch (at least 256 for the diagnostics sum)
static int whole_threads(const RedShape& r, int S) {
  const int t = ((r.L * ((S + r.G - 1) / r.G) + 63) / 64) * 64;
  return t < 256 ? 256 : t;
}

bool reduced_shape_whole(int shape) {
  return shape >= 0 && shape < kNumRedShapes && kRedShapes[shape].L > 0;
}

size_t reduced_lds_bytes(int shape, int P, size_t elem, int S, int dcount, bool diag) {
  const RedShape& r = kRedShapes[shape];
  if (r.L > 0 && whole_threads(r, S) > 1024) return ~(size_t)0;
  size_t lds = r.L > 0 ? (size_t)S * P * r.L * elem
                       : (size_t)(r.W * r.G + dcount - 1) * P * 64 * elem;
  const size_t dmin = 2 * (size_t)256 * sizeof(double);
  if (diag && lds < dmin) lds = dmin;
  return lds;
}

template <int P, typename T, typename Td, int W, int G, int U>
static void reduced_launch(dim3 grid, size_t lds, hipStream_t st, const T* rho, int batch,
                           const DevChunk& c, const T* blocks, Td* dst, long ld, int drow_stride,
                           int drow_off, const double* dpart, long dnparts, double dscale,
                           double* dout) {
  hipLaunchKernelGGL((reduced_il_lds<P, T, Td, W, G, U>), grid, dim3(64 * W), lds, st, rho, batch,
                     c.S, blocks, c.dlo, c.dcount, dst, ld, drow_stride, drow_off, dpart, dnparts,
                     dscale, dout);
}

template <int P, typename T, typename Td>
static hipError_t reduced_any(const DevChunk& c, const T* rho, const T* blocks, int batch, Td* dst,
                              long ld, int drow_stride, int drow_off, hipStream_t st,
                              const double* dpart, long dnparts, double dscale, double* dout,
                              int shape) {
  if (shape < 0 || shape >= kNumRedShapes) shape = 0;
  size_t lds = reduced_lds_bytes(shape, P, sizeof(T), c.S, c.dcount, dout != nullptr);
  if (lds > kMaxLdsBytes && shape != 0) {
    shape = 0;
    lds = reduced_lds_bytes(0, P, sizeof(T), c.S, c.dcount, dout != nullptr);
  }
  if (lds <= kMaxLdsBytes && kRedShapes[shape].L > 0) {
    const RedShape& r = kRedShapes[shape];
    const dim3 grid((batch + r.L - 1) / r.L), block(whole_threads(r, c.S));
#define CHX_WHOLE(L_, G_)                                                                   \
  hipLaunchKernelGGL((reduced_whole<P, T, Td, L_, G_>), grid, block, lds, st, rho, batch, c.S, \
                     blocks, c.dlo, c.dcount, dst, ld, drow_stride, drow_off, dpart, dnparts,  \
                     dscale, dout)
    switch (shape) {
      case 12: CHX_WHOLE(32, 8); break;
      case 13: CHX_WHOLE(16, 4); break;
      default: CHX_WHOLE(16, 8); break;
    }
#undef CHX_WHOLE
  } else if (lds <= kMaxLdsBytes) {
    const RedShape& r = kRedShapes[shape];
    const int kb = r.W * r.G;
    dim3 grid((batch + 63) / 64, (c.S + kb - 1) / kb);
#define CHX_RED(W_, G_, U_)                                                                   \
  reduced_launch<P, T, Td, W_, G_, U_>(grid, lds, st, rho, batch, c, blocks, dst, ld,         \
                                       drow_stride, drow_off, dpart, dnparts, dscale, dout)
    switch (shape) {
      case 0: CHX_RED(8, 4, 4); break;
      case 1: CHX_RED(8, 4, 8); break;
      case 2: CHX_RED(8, 2, 4); break;
      case 3: CHX_RED(4, 8, 4); break;
      case 4: CHX_RED(4, 8, 8); break;
      case 5: CHX_RED(4, 4, 4); break;
      case 6: CHX_RED(16, 2, 4); break;
      case 7: CHX_RED(16, 3, 4); break;
      case 8: CHX_RED(16, 4, 4); break;
      case 9: CHX_RED(4, 1, 8); break;
      case 10: CHX_RED(4, 2, 8); break;
      default: CHX_RED(8, 1, 8); break;
    }
#undef CHX_RED
  } else {
    if (dout) return hipErrorInvalidValue;
    dim3 grid((batch + 63) / 64, (c.S + 3) / 4);
    hipLaunchKernelGGL((reduced_il<P, T, Td>), grid, dim3(256), 0, st, rho, batch, c.S, blocks,
                       c.dlo, c.dcount, dst, ld, drow_stride, drow_off);
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_reduced_il(const DevChunk& c, const double* rho, int batch, double* dst, long ld,
                             int drow_stride, int drow_off, hipStream_t st, const double* dpart,
                             long dnparts, double dscale, double* dout) {
  return reduced_any<P, double, double>(c, rho, c.blocks, batch, dst, ld, drow_stride, drow_off,
                                        st, dpart, dnparts, dscale, dout, c.red_shape);
}

template <int P>
hipError_t launch_chunked_il(const DevChunk& c, double* x, long ld, int batch, double* rho,
                             hipStream_t st, bool correct) {
  dim3 grid((batch + 63) / 64, (c.S + 3) / 4);
  if (!correct) {  // the chunk interiors y stay for the caller to correct later
    hipLaunchKernelGGL((chunk_sweep_il<P, kChunk, double, double>), grid, dim3(256), 0, st, x, ld,
                       x, ld, batch, c.S, c.rec, band_of<double>(c.coef), rho);
    return launch_reduced_il<P>(c, rho, batch, x, ld, kChunk, kChunk - P, st, nullptr, 0, 0.0,
                                nullptr);
  }
  // separator parts only; separators into the separator rows; then every
  // chunk swept again from its right-hand side and corrected
  hipLaunchKernelGGL((chunk_sweep_il<P, kChunk, double, double, false>), grid, dim3(256), 0, st,
                     x, ld, x, ld, batch, c.S, c.rec, band_of<double>(c.coef), rho);
  hipError_t e = launch_reduced_il<P>(c, rho, batch, x, ld, kChunk, kChunk - P, st, nullptr, 0,
                                      0.0, nullptr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((chunk_resolve_il<P, kChunk>), grid, dim3(256), 0, st, x, ld, batch, c.S,
                     c.rec, band_of<double>(c.coef));
  return hipGetLastError();
}

template <int P>
hipError_t launch_chunked_il32(const DevChunk& c, const double* src, long lds, float* y32,
                               float* rho32, double* out, long ldo, int batch, bool acc,
                               hipStream_t st) {
  dim3 grid((batch + 63) / 64, (c.S + 3) / 4);
  hipLaunchKernelGGL((chunk_sweep_il<P, kChunk, float, float>), grid, dim3(256), 0, st, src, lds,
                     y32, (long)batch, batch, c.S, c.rec32, band_of<float>(c.coef), rho32);
  hipError_t e = reduced_any<P, float, float>(c, rho32, c.blocks32, batch, y32, (long)batch,
                                              kChunk, kChunk - P, st, nullptr, 0, 0.0, nullptr,
                                              c.red_shape);
  if (e != hipSuccess) return e;
  if (acc)
    hipLaunchKernelGGL((correct_il<P, kChunk, float, float, true>), grid, dim3(256), 0, st, y32,
                       (long)batch, out, ldo, batch, c.S, c.rec32);
  else
    hipLaunchKernelGGL((correct_il<P, kChunk, float, float, false>), grid, dim3(256), 0, st, y32,
                       (long)batch, out, ldo, batch, c.S, c.rec32);
  return hipGetLastError();
}

template <int P>
hipError_t launch_rows_lds(const DevChunk& c, double* x, long ld, int rows, hipStream_t st,
                           bool stream_in) {
  const int R = 256 / c.S;
  const long ngroups = ((long)rows + R - 1) / R;
  // dense rows in whole groups of 256 chunks: the half-tile kernel
  const bool half = kRowsHalfTile && P == 2 && ld == c.n && 256 % c.S == 0 && rows % R == 0;
  if (half && c.M == kChunk && stream_in)
    hipLaunchKernelGGL((row_solve_half<2, kChunk, true>), dim3((unsigned)ngroups), dim3(256), 0,
                       st, x, c.S, c.rec, band_of<double>(c.coef), c.blocks, c.dlo, c.dcount);
  else if (half && c.M == kChunk)
    hipLaunchKernelGGL((row_solve_half<2, kChunk>), dim3((unsigned)ngroups), dim3(256), 0, st, x,
                       c.S, c.rec, band_of<double>(c.coef), c.blocks, c.dlo, c.dcount);
  else if (half && c.M == 16)
    hipLaunchKernelGGL((row_solve_half<2, 16>), dim3((unsigned)ngroups), dim3(256), 0, st, x,
                       c.S, c.rec, band_of<double>(c.coef), c.blocks, c.dlo, c.dcount);
  else if (P == 2 && c.M == 16)
    hipLaunchKernelGGL((row_solve_lds<P, 16, double, false>), dim3((unsigned)ngroups), dim3(256),
                       0, st, x, ld, x, ld, rows, c.n, c.S, R, c.rec, band_of<double>(c.coef),
                       c.blocks, c.dlo, c.dcount);
  else
    hipLaunchKernelGGL((row_solve_lds<P, kChunk, double, false>), dim3((unsigned)ngroups),
                       dim3(256), 0, st, x, ld, x, ld, rows, c.n, c.S, R, c.rec,
                       band_of<double>(c.coef), c.blocks, c.dlo, c.dcount);
  return hipGetLastError();
}

template <int P>
hipError_t launch_rows_lds32(const DevChunk& c, const double* src, long lds, double* dst, long ldd,
                             int rows, bool acc, hipStream_t st) {
  const int R = 256 / c.S;
  const long ngroups = ((long)rows + R - 1) / R;
  if (acc)
    hipLaunchKernelGGL((row_solve_lds<P, kChunk, float, true>), dim3((unsigned)ngroups), dim3(256),
                       0, st, src, lds, dst, ldd, rows, c.n, c.S, R, c.rec32,
                       band_of<float>(c.coef), c.blocks32, c.dlo, c.dcount);
  else
    hipLaunchKernelGGL((row_solve_lds<P, kChunk, float, false>), dim3((unsigned)ngroups),
                       dim3(256), 0, st, src, lds, dst, ldd, rows, c.n, c.S, R, c.rec32,
                       band_of<float>(c.coef), c.blocks32, c.dlo, c.dcount);
  return hipGetLastError();
}

hipError_t launch_rows_lds_f32(const DevChunk& c, const float* src, float* dst, int rows,
                               hipStream_t st) {
  const int R = 256 / c.S;
  const long ngroups = ((long)rows + R - 1) / R;
  hipLaunchKernelGGL((row_solve_lds_f32<2, kChunk>), dim3((unsigned)ngroups), dim3(256), 0, st,
                     src, (long)c.n, dst, (long)c.n, rows, c.n, c.S, R, c.rec32,
                     band_of<float>(c.coef), c.blocks32, c.dlo, c.dcount);
  return hipGetLastError();
}

hipError_t launch_reduced_il32(const DevChunk& c, const float* rho, int batch, float* dst,
                               long ld, hipStream_t st, const double* dpart, long dnparts,
                               double dscale, double* dout) {
  return reduced_any<2, float, float>(c, rho, c.blocks32, batch, dst, ld, kChunk, kChunk - 2, st,
                                      dpart, dnparts, dscale, dout, c.red_shape);
}

template <int P>
hipError_t launch_resid_lines(const double* coef, int periodic, int n, const double* f, long fss,
                              long fes, const double* x, long xss, long xes, double* r, long rss,
                              long res, int batch, bool sys_fast, hipStream_t st) {
  const long fast = sys_fast ? batch : n, slow = sys_fast ? n : batch;
  dim3 grid((unsigned)((fast + 255) / 256), (unsigned)slow);
  hipLaunchKernelGGL((resid_lines<P>), grid, dim3(256), 0, st, f, fss, fes, x, xss, xes, r, rss,
                     res, batch, n, band_of<double>(coef), periodic, sys_fast ? 1 : 0);
  return hipGetLastError();
}

#define CHX_INST(P)                                                                             \
  template hipError_t launch_whole<P>(const DevWhole&, double*, long, long, int, hipStream_t);  \
  template hipError_t launch_whole32<P>(const DevWhole&, double*, long, long, double*, long,    \
                                        long, int, bool, hipStream_t);                           \
  template hipError_t launch_chunked_il<P>(const DevChunk&, double*, long, int, double*,        \
                                           hipStream_t, bool);                                   \
  template hipError_t launch_chunked_il32<P>(const DevChunk&, const double*, long, float*,      \
                                             float*, double*, long, int, bool, hipStream_t);     \
  template hipError_t launch_reduced_il<P>(const DevChunk&, const double*, int, double*, long,  \
                                           int, int, hipStream_t, const double*, long, double,   \
                                           double*);                                             \
  template hipError_t launch_rows_lds<P>(const DevChunk&, double*, long, int, hipStream_t, bool); \
  template hipError_t launch_rows_lds32<P>(const DevChunk&, const double*, long, double*, long, \
                                           int, bool, hipStream_t);                              \
  template hipError_t launch_resid_lines<P>(const double*, int, int, const double*, long, long, \
                                            const double*, long, long, double*, long, long, int, \
                                            bool, hipStream_t);
CHX_INST(1)
CHX_INST(2)
#undef CHX_INST

}  // namespace chx
