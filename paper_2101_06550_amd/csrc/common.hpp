// common.hpp -- small device/host helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chx {

// Constant band coefficients handed to kernels by value: coef[o + P] is the
// coefficient of x[i + o].
template <typename T>
struct BandT {
  T c[5];
};

// Chunk length of the chunked kernels (unknowns per thread-chunk).
constexpr int kChunk = 32;

// Pointers typed by address space.  A pointer that a kernel reads out of
// memory (a run record, a plan passed inside a struct) is generic: the
// compiler can neither place it in device memory (it emits flat accesses,
// which also count against the scalar loads' wait counter) nor prove that
// the kernel's own stores, LDS ones included, leave the data alone (it reads
// plan tables with vector loads and waits on each sweep row's coefficients).
// Plan tables are never written while a kernel runs: read through the
// constant space they go through scalar loads, as they do where the pointer
// is a restrict kernel argument; fields go through the global space.
using TabD = const __attribute__((address_space(4))) double*;
using TabF = const __attribute__((address_space(4))) float*;
using GD = __attribute__((address_space(1))) double*;
using GCD = const __attribute__((address_space(1))) double*;
using GCF = const __attribute__((address_space(1))) float*;

// SplitMix64 finaliser (Steele, Lea and Flood 2014): the mixing function of
// the counter-based generator of the Cahn-Hilliard-Cook forcing.
__host__ __device__ __forceinline__ unsigned long long chx_sm_mix(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int wrap_once(int j, int S) {
  j += (j < 0) ? S : 0;
  j -= (j >= S) ? S : 0;
  return j;
}

// Streaming 16-byte global accesses (non-temporal: the data is touched once
// per pass).  On gfx950 a plain copy moves 6.5 TB/s with non-temporal loads
// and stores against 5.6 TB/s with ordinary ones; in the step's passes the
// stores alone pay (measured per pass).
__device__ __forceinline__ double2 load_stream(const double2* p) {
  double2 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}
__device__ __forceinline__ void store_stream(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// Lane l receives the value of lane l-1 (wave_shr:1); lane 0 keeps `edge`.
__device__ __forceinline__ double dpp_from_left(double v, double edge) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  int elo = __double2loint(edge), ehi = __double2hiint(edge);
  lo = __builtin_amdgcn_update_dpp(elo, lo, 0x138, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(ehi, hi, 0x138, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Lane l receives the value of lane l+1 (wave_shl:1); lane 63 keeps `edge`.
__device__ __forceinline__ double dpp_from_right(double v, double edge) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  int elo = __double2loint(edge), ehi = __double2hiint(edge);
  lo = __builtin_amdgcn_update_dpp(elo, lo, 0x130, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(ehi, hi, 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Forward + back sweep of one chunk held in registers (compile-time
// unrolled).  On entry f[0..M) holds the chunk's right-hand side; on exit
// f[0..M-P) holds y = E_m^{-1} f_interior and the separator values f[M-P..M)
// are untouched.  rec: kRec values per interior position (1/alpha, L(i,i-1),
// R(i,i+1), R(i,i+2), ...).  eps = L(i,i-2) = the band's outermost
// sub-diagonal (P = 2 only).
template <int P, int M, typename T, typename RP = const T*>
__device__ __forceinline__ void chunk_sweep(T (&f)[M], RP __restrict__ rec, T eps) {
  constexpr int MI = M - P;
#pragma unroll
  for (int p = 0; p < MI; ++p) {
    T v = f[p];
    if (P == 2 && p >= 2) v = v - eps * f[p - 2];
    if (p >= 1) v = v - rec[p * 8 + 1] * f[p - 1];
    f[p] = v * rec[p * 8 + 0];
  }
#pragma unroll
  for (int p = MI - 1; p >= 0; --p) {
    T v = f[p];
    if (P == 2 && p + 2 < MI) v = v - rec[p * 8 + 3] * f[p + 2];
    if (p + 1 < MI) v = v - rec[p * 8 + 2] * f[p + 1];
    f[p] = v;
  }
}

// Separator right-hand-side parts of one chunk after its sweep:
//   pa[a] = f_sep[a] - (coupling of separator a to this chunk's interior) y
//   pb[a] = (coupling of the previous chunk's separator a to this interior) y
// so that the reduced right-hand side of chunk k is pa_k - pb_{k+1}.
template <int P, int M, typename T>
__device__ __forceinline__ void chunk_parts(const T (&f)[M], const BandT<T>& bd, T (&pa)[P],
                                            T (&pb)[P]) {
  constexpr int MI = M - P;
#pragma unroll
  for (int a = 0; a < P; ++a) {
    T v = f[MI + a];
#pragma unroll
    for (int p = MI + a - P; p < MI; ++p) v = v - bd.c[(p - MI - a) + P] * f[p];
    pa[a] = v;
    T w = T(0);
#pragma unroll
    for (int q = 0; q <= a; ++q) w = w + bd.c[(q + P - a) + P] * f[q];
    pb[a] = w;
  }
}

// Interior correction x = y - Zl s_prev - Zr s_own (rec[4..5] = Zl, rec[6..7] = Zr),
// separators set to s_own.
template <int P, int M, typename T, typename RP = const T*>
__device__ __forceinline__ void chunk_correct(T (&f)[M], RP __restrict__ rec,
                                              const T (&sp)[P], const T (&so)[P]) {
  constexpr int MI = M - P;
#pragma unroll
  for (int p = 0; p < MI; ++p) {
    T v = f[p];
#pragma unroll
    for (int a = 0; a < P; ++a) v = v - rec[p * 8 + 4 + a] * sp[a] - rec[p * 8 + 6 + a] * so[a];
    f[p] = v;
  }
#pragma unroll
  for (int a = 0; a < P; ++a) f[MI + a] = so[a];
}

}  // namespace chx
