// plan.hpp -- host-side factorisation tables for constant-coefficient banded
// systems (bandwidth P = 1 tridiagonal, P = 2 pentadiagonal).
//
// Two table families are built, both once per (n, coefficients):
//
//  * "whole" tables: the thesis's own arrangement (Ch.4 "The pentadiagonal
//    matrix system"): the last P unknowns are bordered off (Navon for P = 2;
//    for P = 1 the same bordering is the Schur-complement form of the
//    Sherman-Morrison correction of Ch.5), the leading (n-P) block E is
//    LR-factored (Ch.4 "Solution of the pentadiagonal system"), and
//    q = E^{-T} h, Z = E^{-1} k and [C22 - h^T E^{-1} k]^{-1} are stored so a
//    single forward sweep can accumulate q^T f and a single back sweep can
//    apply the correction.  Used by the one-thread-per-system kernels.
//
//  * "chunk" tables: the same bordering applied to every chunk of m
//    consecutive unknowns (the last P of each chunk are separators).  All
//    chunks share one interior matrix E_m, so the tables are per position in
//    a chunk, independent of n.  The separators solve a small block-cyclic
//    system whose inverse is the separator-separator block of A^{-1}; its
//    blocks are read off the first column of the circulant A^{-1} and kept
//    down to 2^-60 of the largest block.  Used by the chunked kernels that
//    give one system many threads.
//
// All arithmetic here is long double; the device receives FP64 and FP32
// roundings of the results.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

namespace chx {

// Record of 8 values per position used by every sweep kernel:
//   [0] 1/alpha_i   [1] L(i,i-1)   [2] R(i,i+1)   [3] R(i,i+2)
//   [4..7] kernel-specific correction vectors (see ChunkTables / WholeTables)
constexpr int kRec = 8;

struct Band {
  int P = 2;            // half bandwidth
  double coef[5] = {};  // coefficient of x[i+o] at coef[o + P], o = -P..P
  bool periodic = true;
};

struct WholeTables {
  int n = 0, P = 2, mi = 0;   // mi = n - P (periodic) or n (not periodic)
  std::vector<double> rec;    // mi * kRec: [4,5] = q_0,q_1 ; [6,7] = Z_0,Z_1
  std::vector<float> rec32;
  double minv[4] = {1, 0, 0, 1};  // [C22 - h^T E^{-1} k]^{-1}, row-major PxP
  float minv32[4] = {1, 0, 0, 1};
};

struct ChunkTables {
  int n = 0, P = 2, m = 0, S = 0, mi = 0;  // chunk length, chunk count, interior
  std::vector<double> rec;    // mi * kRec: [4,5] = Zl(:,0..1), [6,7] = Zr(:,0..1)
  std::vector<float> rec32;
  int dlo = 0, dcount = 0;    // reduced-system offsets d = dlo .. dlo+dcount-1
  std::vector<double> blocks; // dcount * 4: block B_d (PxP row-major, padded to 2x2)
  std::vector<float> blocks32;
  double max_dropped = 0.0;   // largest |entry| of a dropped block (0 if none)
};

// Status codes mirror chx.h.
int build_whole(const Band& band, int n, WholeTables* out);
int build_chunk(const Band& band, int n, int m, ChunkTables* out);

// First column of A^{-1} for the cyclic band matrix (long double solve).
int circulant_inverse_column(const Band& band, int n, std::vector<long double>* g);

}  // namespace chx
