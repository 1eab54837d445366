// abi.cpp -- the extern "C" boundary declared in include/chx.h: argument
// checks, plan construction and upload, kernel dispatch.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <string>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "ch_launch.hpp"
#include "chx.h"
#include "common.hpp"
#include "ens.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace chx;

namespace {

// A factored constant-coefficient band matrix and its device tables.
struct BandPlan {
  int P = 2, n = 0, periodic = 1;
  double coef[5] = {};
  double kappa = 1.0;  // 2-norm condition number (exact when periodic)
  WholeTables whole;
  ChunkTables chunk;
  bool has_chunk = false;
  DevWhole dwhole;
  DevChunk dchunk;
  // 16-point chunks as well (the ADI step's plans, when n allows): twice the
  // parallelism and half the serial sweep of the 32-point chunks, for grids
  // whose passes are too small to fill the chip
  ChunkTables chunk16;
  bool has_chunk16 = false;
  DevChunk dchunk16;
  void* dmem = nullptr;
  int device = 0;

  ~BandPlan() {
    if (dmem) (void)hipFree(dmem);
  }
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int upload(BandPlan* p) {
  size_t off = 0;
  const size_t o_w = off; off = align256(off + p->whole.rec.size() * sizeof(double));
  const size_t o_w32 = off; off = align256(off + p->whole.rec32.size() * sizeof(float));
  const size_t o_c = off; off = align256(off + p->chunk.rec.size() * sizeof(double));
  const size_t o_c32 = off; off = align256(off + p->chunk.rec32.size() * sizeof(float));
  const size_t o_b = off; off = align256(off + p->chunk.blocks.size() * sizeof(double));
  const size_t o_b32 = off; off = align256(off + p->chunk.blocks32.size() * sizeof(float));
  const size_t o_h = off; off = align256(off + p->chunk16.rec.size() * sizeof(double));
  const size_t o_h32 = off; off = align256(off + p->chunk16.rec32.size() * sizeof(float));
  const size_t o_hb = off; off = align256(off + p->chunk16.blocks.size() * sizeof(double));
  const size_t o_hb32 = off; off = align256(off + p->chunk16.blocks32.size() * sizeof(float));
  if (hipGetDevice(&p->device) != hipSuccess) return CHX_EHIP;
  if (hipMalloc(&p->dmem, off > 0 ? off : 256) != hipSuccess) {
    p->dmem = nullptr;
    return CHX_EHIP;
  }
  std::vector<unsigned char> host(off > 0 ? off : 256, 0);
  auto put = [&](size_t o, const void* src, size_t bytes) {
    if (bytes) std::memcpy(host.data() + o, src, bytes);
  };
  put(o_w, p->whole.rec.data(), p->whole.rec.size() * sizeof(double));
  put(o_w32, p->whole.rec32.data(), p->whole.rec32.size() * sizeof(float));
  put(o_c, p->chunk.rec.data(), p->chunk.rec.size() * sizeof(double));
  put(o_c32, p->chunk.rec32.data(), p->chunk.rec32.size() * sizeof(float));
  put(o_b, p->chunk.blocks.data(), p->chunk.blocks.size() * sizeof(double));
  put(o_b32, p->chunk.blocks32.data(), p->chunk.blocks32.size() * sizeof(float));
  put(o_h, p->chunk16.rec.data(), p->chunk16.rec.size() * sizeof(double));
  put(o_h32, p->chunk16.rec32.data(), p->chunk16.rec32.size() * sizeof(float));
  put(o_hb, p->chunk16.blocks.data(), p->chunk16.blocks.size() * sizeof(double));
  put(o_hb32, p->chunk16.blocks32.data(), p->chunk16.blocks32.size() * sizeof(float));
  if (hipMemcpy(p->dmem, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
    return CHX_EHIP;
  auto* base = static_cast<unsigned char*>(p->dmem);
  p->dwhole.n = p->n;
  p->dwhole.P = p->P;
  p->dwhole.periodic = p->periodic;
  for (int k = 0; k < 5; ++k) p->dwhole.coef[k] = p->coef[k];
  for (int k = 0; k < 4; ++k) p->dwhole.minv[k] = p->whole.minv[k];
  p->dwhole.rec = reinterpret_cast<const double*>(base + o_w);
  p->dwhole.rec32 = reinterpret_cast<const float*>(base + o_w32);
  if (p->has_chunk) {
    p->dchunk.n = p->n;
    p->dchunk.P = p->P;
    p->dchunk.S = p->chunk.S;
    p->dchunk.dlo = p->chunk.dlo;
    p->dchunk.dcount = p->chunk.dcount;
    for (int k = 0; k < 5; ++k) p->dchunk.coef[k] = p->coef[k];
    p->dchunk.rec = reinterpret_cast<const double*>(base + o_c);
    p->dchunk.rec32 = reinterpret_cast<const float*>(base + o_c32);
    p->dchunk.blocks = reinterpret_cast<const double*>(base + o_b);
    p->dchunk.blocks32 = reinterpret_cast<const float*>(base + o_b32);
    p->dchunk.M = p->chunk.m;
  }
  if (p->has_chunk16) {
    DevChunk& d = p->dchunk16;
    d.n = p->n;
    d.P = p->P;
    d.S = p->chunk16.S;
    d.dlo = p->chunk16.dlo;
    d.dcount = p->chunk16.dcount;
    d.M = p->chunk16.m;
    for (int k = 0; k < 5; ++k) d.coef[k] = p->coef[k];
    d.rec = reinterpret_cast<const double*>(base + o_h);
    d.rec32 = reinterpret_cast<const float*>(base + o_h32);
    d.blocks = reinterpret_cast<const double*>(base + o_hb);
    d.blocks32 = reinterpret_cast<const float*>(base + o_hb32);
  }
  return CHX_OK;
}

// Condition number of the constant-coefficient band matrix.  Periodic: the
// matrix is circulant (normal), its eigenvalues are the symbol
// f(theta) = sum_k coef[k + P] e^{i k theta} at theta = 2 pi m / n, and
// kappa_2 = max |f| / min |f| exactly.  Non-periodic (banded Toeplitz): the
// same ratio over a fine sampling of theta, the spectrum's envelope (exact in
// the limit for symmetric matrices, an estimate otherwise).
double band_kappa(int P, int n, const double* coef, bool periodic) {
  const int m = periodic ? n : 8 * n;
  double lo = INFINITY, hi = 0.0;
  for (int q = 0; q < m; ++q) {
    const double th = 2.0 * M_PI * (double)q / (double)m;
    double re = 0.0, im = 0.0;
    for (int k = -P; k <= P; ++k) {
      re += coef[k + P] * std::cos(k * th);
      im += coef[k + P] * std::sin(k * th);
    }
    const double a = std::hypot(re, im);
    lo = std::min(lo, a);
    hi = std::max(hi, a);
  }
  return lo > 0.0 ? hi / lo : INFINITY;
}

// Iterative refinement with FP32 sweeps contracts the error by about
// c kappa 2^-24 per pass (c a small growth constant of the FP32 LR
// factorisation and sweeps, taken as 4); at or above 1 it need not converge.
bool refinement_fails(double kappa) { return !(4.0 * kappa * 0x1.0p-24 < 1.0); }

bool finite_all(const double* v, int n) {
  for (int k = 0; k < n; ++k)
    if (!std::isfinite(v[k])) return false;
  return true;
}

// Build (host) and upload (device) a band plan.
template <class PlanT>
int make_plan(int P, int n, const double* coef, int periodic, PlanT** out,
              bool chunk16 = false) {
  if (!out) return CHX_EINVAL;
  *out = nullptr;
  const int nmin = (P == 2) ? 5 : 3;
  if (n < nmin) return CHX_EUNSUPPORTED_N;
  if (!finite_all(coef, 2 * P + 1)) return CHX_EINVAL;
  PlanT* p = new (std::nothrow) PlanT();
  if (!p) return CHX_ENOMEM;
  p->P = P;
  p->n = n;
  p->periodic = periodic ? 1 : 0;
  for (int k = 0; k < 2 * P + 1; ++k) p->coef[k] = coef[k];
  p->kappa = band_kappa(P, n, coef, p->periodic != 0);
  Band band;
  band.P = P;
  band.periodic = p->periodic != 0;
  for (int k = 0; k < 2 * P + 1; ++k) band.coef[k] = coef[k];
  int rc = build_whole(band, n, &p->whole);
  if (rc == CHX_OK && p->periodic && n % kChunk == 0) {
    rc = build_chunk(band, n, kChunk, &p->chunk);
    p->has_chunk = (rc == CHX_OK);
    if (rc == CHX_EINVAL) rc = CHX_OK;  // shape not eligible: keep the whole-system path
  }
  if (rc == CHX_OK && chunk16 && p->has_chunk && n % 16 == 0) {
    const int rc16 = build_chunk(band, n, 16, &p->chunk16);
    p->has_chunk16 = (rc16 == CHX_OK);
    if (rc16 != CHX_OK && rc16 != CHX_EINVAL) rc = rc16;
  }
  if (rc == CHX_OK) rc = upload(p);
  if (rc != CHX_OK) {
    delete p;
    return rc;
  }
  *out = p;
  return CHX_OK;
}

// Workspace of one batched solve.  FP64: the separator partials of the
// chunked interleaved path.  FP32-refined: a compact copy of the right-hand
// sides, a compact residual buffer, and (chunked interleaved) FP32 chunk
// solutions and FP32 separator partials.
struct SolveWs {
  size_t f = 0, r = 0, y32 = 0, rho32 = 0, total = 0;
};

SolveWs solve_ws_layout(const BandPlan* p, int batch, int layout, int dtype) {
  SolveWs w;
  if (!p || batch <= 0) return w;
  const bool chunk_il = layout == CHX_INTERLEAVED && p->has_chunk;
  if (dtype == CHX_F64) {
    if (chunk_il) w.total = align256((size_t)p->chunk.S * 2 * p->P * (size_t)batch * sizeof(double));
    return w;
  }
  size_t off = 0;
  const size_t nb = (size_t)p->n * batch;
  w.f = off; off += align256(nb * sizeof(double));
  w.r = off; off += align256(nb * sizeof(double));
  if (chunk_il) {
    w.y32 = off; off += align256(nb * sizeof(float));
    w.rho32 = off; off += align256((size_t)p->chunk.S * 2 * p->P * (size_t)batch * sizeof(float));
  }
  w.total = off;
  return w;
}

size_t solve_ws(const BandPlan* p, int batch, int layout, int dtype) {
  return solve_ws_layout(p, batch, layout, dtype).total;
}

// One FP32-sweep solve of the batch: out (strides of x) = A32^{-1} src,
// written or added (acc).  src is either x itself (in place, strides of x)
// or the compact residual buffer.
template <int P>
hipError_t solve32(const BandPlan* p, int batch, int layout, double* src, bool src_is_x, double* x,
                   long ld, unsigned char* ws, const SolveWs& w, bool acc, hipStream_t st) {
  const int n = p->n;
  const long lds = src_is_x ? ld : (layout == CHX_INTERLEAVED ? (long)batch : (long)n);
  if (layout == CHX_INTERLEAVED) {
    if (p->has_chunk)
      return launch_chunked_il32<P>(p->dchunk, src, lds, reinterpret_cast<float*>(ws + w.y32),
                                    reinterpret_cast<float*>(ws + w.rho32), x, ld, batch, acc, st);
    return launch_whole32<P>(p->dwhole, src, 1, lds, x, 1, ld, batch, acc, st);
  }
  if (p->has_chunk && p->chunk.S <= 256)
    return launch_rows_lds32<P>(p->dchunk, src, lds, x, ld, batch, acc, st);
  return launch_whole32<P>(p->dwhole, src, lds, 1, x, ld, 1, batch, acc, st);
}

template <int P>
hipError_t solve_refined(const BandPlan* p, int batch, double* x, long ld, int layout, int refine,
                         unsigned char* ws, const SolveWs& w, hipStream_t st) {
  const int n = p->n;
  const bool il = layout == CHX_INTERLEAVED;
  double* fcopy = reinterpret_cast<double*>(ws + w.f);
  double* rbuf = reinterpret_cast<double*>(ws + w.r);
  const long pc = il ? batch : n;  // compact pitch
  hipError_t e = il ? hipMemcpy2DAsync(fcopy, pc * sizeof(double), x, ld * sizeof(double),
                                       (size_t)batch * sizeof(double), n, hipMemcpyDeviceToDevice,
                                       st)
                    : hipMemcpy2DAsync(fcopy, pc * sizeof(double), x, ld * sizeof(double),
                                       (size_t)n * sizeof(double), batch, hipMemcpyDeviceToDevice,
                                       st);
  if (e == hipSuccess) e = solve32<P>(p, batch, layout, x, true, x, ld, ws, w, false, st);
  for (int k = 0; k < refine && e == hipSuccess; ++k) {
    if (il)
      e = launch_resid_lines<P>(p->coef, p->periodic, n, fcopy, 1, pc, x, 1, ld, rbuf, 1, pc,
                                batch, true, st);
    else
      e = launch_resid_lines<P>(p->coef, p->periodic, n, fcopy, pc, 1, x, ld, 1, rbuf, pc, 1,
                                batch, false, st);
    if (e == hipSuccess) e = solve32<P>(p, batch, layout, rbuf, false, x, ld, ws, w, true, st);
  }
  return e;
}

int solve(const BandPlan* p, int batch, void* x, long ld, int layout, int dtype, int refine,
          void* ws, size_t ws_bytes, chx_stream s) {
  if (!p) return CHX_EINVAL;
  if (batch < 0) return CHX_EINVAL;
  if (batch == 0) return CHX_OK;
  if (!x) return CHX_EINVAL;
  if (layout != CHX_INTERLEAVED && layout != CHX_CONTIGUOUS) return CHX_EINVAL;
  if (dtype != CHX_F64 && dtype != CHX_F32_REFINED) return CHX_EINVAL;
  if (dtype == CHX_F32_REFINED && (refine < 1 || refine > 3)) return CHX_EINVAL;
  if (layout == CHX_INTERLEAVED && ld < batch) return CHX_EINVAL;
  if (layout == CHX_CONTIGUOUS && ld < p->n) return CHX_EINVAL;
  if (dtype == CHX_F32_REFINED && refinement_fails(p->kappa)) return CHX_EREFINE;
  const SolveWs w = solve_ws_layout(p, batch, layout, dtype);
  if (w.total > 0 && (!ws || ws_bytes < w.total)) return CHX_ENOMEM;
  if (w.total > 0 && (reinterpret_cast<uintptr_t>(ws) & 255)) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* xd = static_cast<double*>(x);
  auto* wsb = static_cast<unsigned char*>(ws);
  hipError_t e = hipSuccess;
  if (dtype == CHX_F32_REFINED) {
    e = (p->P == 2) ? solve_refined<2>(p, batch, xd, ld, layout, refine, wsb, w, st)
                    : solve_refined<1>(p, batch, xd, ld, layout, refine, wsb, w, st);
  } else if (layout == CHX_INTERLEAVED) {
    if (p->has_chunk) {
      e = (p->P == 2) ? launch_chunked_il<2>(p->dchunk, xd, ld, batch, static_cast<double*>(ws), st)
                      : launch_chunked_il<1>(p->dchunk, xd, ld, batch, static_cast<double*>(ws), st);
    } else {
      e = (p->P == 2) ? launch_whole<2>(p->dwhole, xd, 1, ld, batch, st)
                      : launch_whole<1>(p->dwhole, xd, 1, ld, batch, st);
    }
  } else {
    if (p->has_chunk && p->chunk.S <= 256) {
      e = (p->P == 2) ? launch_rows_lds<2>(p->dchunk, xd, ld, batch, st, true)
                      : launch_rows_lds<1>(p->dchunk, xd, ld, batch, st, true);
    } else {
      e = (p->P == 2) ? launch_whole<2>(p->dwhole, xd, ld, 1, batch, st)
                      : launch_whole<1>(p->dwhole, xd, ld, 1, batch, st);
    }
  }
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

}  // namespace

struct chx_penta_plan_s : BandPlan {};
struct chx_tri_plan_s : BandPlan {};

// ---------------------------------------------------------------------------
// Cahn-Hilliard handle
struct chx_ch_s {
  chx_ch_params prm{};
  BandPlan* px = nullptr;  // rows: length nx, sigma_x
  BandPlan* py = nullptr;  // columns: length ny, sigma_y
  bool fast = false;
  bool small_ok = false;  // the single-workgroup LDS-resident path fits
  bool small = false;     // ... and is in use
  int split = -1;         // split row pass shape (-1: plain separators + rows,
                          // kSplitOverlap: separators beside the interior rows)
  int col_order = 0;      // tile order of the column pass (CHX_TUNE_COLUMN_ORDER)
  int mcol = kChunk;      // chunk length of the column solves (32, or 16: CHX_TUNE_COLUMN_CHUNK)
  int mrow = kChunk;      // chunk length of the row solves (CHX_TUNE_ROW_CHUNK)
  // the second stream of the overlapped schedule and its fork / join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double sigma = 0.0;     // Cahn-Hilliard-Cook forcing intensity (0: off)
  unsigned long long noise_seed = 0, noise_step = 0;
  ChCoef K{};
  Ch2Coef K2{};           // the thesis's delta-form scheme (CHX_SCHEME_P2)
  size_t off_b0 = 0, off_b1 = 0, off_rho = 0, off_part = 0, off_r = 0, ws_total = 0;
  // FP32-sweep refined path: residual buffer, FP32 chunk solutions and partials
  size_t off_y32 = 0, off_rho32 = 0, off_v32[4] = {};  // FP32-refined step
  double cxs[5] = {}, cys[5] = {};
  long part_count = 0;
  double* dscratch = nullptr;  // ch_diagnostics: partials + 2 outputs
  // ch_k1: transform plan and buffers, made on first use
  bool fft_ready = false;
  hipfftHandle fft{};
  void* fft_mem = nullptr;
  long dscratch_parts = 0;
  // CHX_TUNE_GRAPH: ch_adi_step replays a captured hipGraph of the whole call
  // (re-captured when the field, ld, nsteps, diag_out or ws change)
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  double* g_c = nullptr;
  long g_ld = 0;
  int g_nsteps = -1;
  double* g_diag = nullptr;
  void* g_ws = nullptr;
  hipEvent_t g_done = nullptr;  // recorded after every replay
  void drop_graph() {
    if (gexec && g_done) (void)hipEventSynchronize(g_done);  // no replay still running
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
  ~chx_ch_s() {
    drop_graph();
    if (g_done) (void)hipEventDestroy(g_done);
    if (cap) (void)hipStreamDestroy(cap);
    delete px;
    delete py;
    if (dscratch) (void)hipFree(dscratch);
    if (fft_ready) (void)hipfftDestroy(fft);
    if (fft_mem) (void)hipFree(fft_mem);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};

// ---------------------------------------------------------------------------
// Uneven ensemble handle
struct chx_ens_s {
  int nruns = 0;
  std::vector<chx_ch_params> prm;
  std::vector<BandPlan*> px, py;  // per size class
  std::vector<EnsRun> runs;       // host copy of the run table
  std::vector<EnsClass> classes;
  void* dmem = nullptr;           // run table, class table, work items
  EnsRun* druns = nullptr;
  EnsClasses hcls{};              // class tables passed by value to the kernels
  int4* ditems = nullptr;
  int* dsmall = nullptr;          // runs on the single-workgroup LDS path
  int* dbig = nullptr;            // the other runs
  int nsmall = 0, nbig = 0, small_threads = 0;
  size_t small_lds = 0;
  hipStream_t side = nullptr;     // small runs overlap the big runs' phases
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int n_col = 0, n_red = 0, n_row = 0;
  long o_col = 0, o_red = 0, o_row = 0;
  bool rows_half = false;  // every row item a dense whole group: half-tile row kernel
  int red_shape = 0;       // FP64 separator kernel shape (timed at creation)
  std::vector<int> red_order;  // the runs whose separator items follow o_red
  size_t ws_total = 0, red_lds = 0;
  long max_points = 0;
  // cached hipGraph of a whole call (nsteps, diag, ws)
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;
  int g_nsteps = -1;
  double* g_diag = nullptr;
  void* g_ws = nullptr;
  // FP32-refined ensembles: work items ordered by refine passes (most
  // first); rn_*[k] = the items of the runs that make pass k (a prefix)
  bool refined = false;
  int max_passes = 0;
  int rn_col[4] = {}, rn_red[4] = {}, rn_row[4] = {};
  // Cahn-Hilliard-Cook forcing: counter on the device (so graph replays
  // advance it) and its host mirror
  bool noise = false;
  unsigned long long* dnoise = nullptr;
  unsigned long long noise_step = 0;

  // per-run coarsening measures: Simpson partials, and a batched real-to-
  // complex transform per grid size (made on first use)
  void* mom_mem = nullptr;
  std::vector<long> mom_off;  // per run: offset (doubles) of its partials
  void* k1_mem = nullptr;
  struct FftGroup {
    int nx, ny;
    std::vector<int> runs;
    hipfftHandle plan;
  };
  std::vector<FftGroup> k1_groups;
  size_t k1_real_off = 0, k1_spec_off = 0, k1_part_off = 0;
  std::vector<long> k1_poff;  // per run: offset (doubles) of its partials
  ~chx_ens_s() {
    for (auto& g : k1_groups)
      if (g.plan) (void)hipfftDestroy(g.plan);
    if (mom_mem) (void)hipFree(mom_mem);
    if (dnoise) (void)hipFree(dnoise);

    if (k1_mem) (void)hipFree(k1_mem);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (side) (void)hipStreamDestroy(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (auto* p : px) delete p;
    for (auto* p : py) delete p;
    if (dmem) (void)hipFree(dmem);
  }
};

namespace {

bool same_grid(const chx_ch_params& a, const chx_ch_params& b) {
  return a.nx == b.nx && a.ny == b.ny && a.lx == b.lx && a.ly == b.ly && a.D == b.D &&
         a.gamma == b.gamma && a.dt == b.dt;
}

ChCoef make_coef(const chx_ch_params& q) {
  const double dx = q.lx / q.nx, dy = q.ly / q.ny;
  ChCoef K;
  K.cx = q.D * q.dt / (dx * dx);
  K.cy = q.D * q.dt / (dy * dy);
  K.ccross = 2.0 * q.D * q.gamma * q.dt / (dx * dx * dy * dy);
  K.inv_dx = 1.0 / dx;
  K.inv_dy = 1.0 / dy;
  K.half_gamma = 0.5 * q.gamma;
  K.dxdy = dx * dy;
  return K;
}

int ens_launch_refined(chx_ens_s* E, int nsteps, double* diag_out, unsigned char* ws,
                       hipStream_t st);

int ens_launch_all(chx_ens_s* E, int nsteps, double* diag_out, unsigned char* ws,
                   hipStream_t st) {
  if (E->refined) return ens_launch_refined(E, nsteps, diag_out, ws, st);
  hipError_t e = hipSuccess;
  const long dstride = 2L * (nsteps + 1);
  const int4* it = E->ditems;
  // small runs: one launch for all steps, on the side stream when big runs
  // run beside them (fork / join by events, also under graph capture)
  const bool fork = E->nsmall > 0 && E->nbig > 0;
  if (E->nsmall > 0) {
    hipStream_t ss = st;
    if (fork) {
      e = hipEventRecord(E->ev_fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(E->side, E->ev_fork, 0);
      ss = E->side;
    }
    if (e == hipSuccess)
      e = launch_ens_small_steps(E->druns, E->hcls, E->dsmall, E->nsmall, E->small_threads,
                                 E->small_lds, nsteps, diag_out, dstride,
                                 E->noise ? E->dnoise : nullptr, ss);
    if (e == hipSuccess && fork) e = hipEventRecord(E->ev_join, E->side);
  }
  for (int n = 0; E->nbig > 0 && n < nsteps && e == hipSuccess; ++n) {
    e = launch_ens_column_pass(n > 0, diag_out != nullptr, E->noise ? E->dnoise : nullptr,
                               E->druns, E->hcls, it + E->o_col, E->n_col, ws, n, st);
    if (e == hipSuccess)
      e = launch_ens_reduced(E->druns, E->hcls, it + E->o_red, E->n_red, ws, n, diag_out, dstride,
                             E->red_lds, st, E->red_shape);
    if (e == hipSuccess) e = launch_ens_rows(E->druns, E->hcls, it + E->o_row, E->n_row, ws, n, st,
                                             E->rows_half);
  }
  // the states written out with their final diagnostics in the same pass
  if (e == hipSuccess && E->nbig > 0)
    e = launch_ens_column_final(E->druns, E->hcls, it + E->o_col, E->n_col, E->dbig, E->nbig, ws,
                                nsteps - 1, diag_out, dstride, nsteps, st);
  if (fork) {  // join even after a failure, so no capture is left open
    const hipError_t j = hipStreamWaitEvent(st, E->ev_join, 0);
    if (e == hipSuccess) e = j;
  }
  // every run has read the counter: move it on by this call's steps
  if (e == hipSuccess && E->noise) e = launch_ens_noise_advance(E->dnoise, nsteps, st);
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

}  // namespace

extern "C" {

int chx_version(void) { return 100; }

const char* chx_status_string(int status) {
  switch (status) {
    case CHX_OK: return "ok";
    case CHX_EINVAL: return "invalid argument";
    case CHX_EUNSUPPORTED_N: return "system size below the minimum";
    case CHX_EPIVOT: return "zero, negative or non-finite pivot";
    case CHX_EHIP: return "HIP runtime or launch failure";
    case CHX_ENONFINITE: return "non-finite diagnostic";
    case CHX_ENOMEM: return "workspace too small or allocation failed";
    case CHX_EREFINE: return "iterative refinement did not converge";
    case CHX_ESCRATCH: return "workspace needed exceeds the static scratch";
    default: return "unknown status";
  }
}

int penta_factor(int n, double a, double b, double c, double d, double e, int periodic,
                 chx_penta_plan* out) {
  if (!out) return CHX_EINVAL;
  const double coef[5] = {a, b, c, d, e};
  return make_plan(2, n, coef, periodic, out);
}

int penta_plan_destroy(chx_penta_plan p) {
  delete p;
  return CHX_OK;
}

size_t penta_solve_ws_bytes(chx_penta_plan p, int batch, int layout, int dtype,
                            int refine_passes) {
  (void)refine_passes;  // the refined workspace does not grow with the pass count
  return solve_ws(p, batch, layout, dtype);
}

int penta_solve_batch(chx_penta_plan p, int batch, void* x_inout, long ld, int layout, int dtype,
                      int refine_passes, void* ws, size_t ws_bytes, chx_stream s) {
  if (p && p->P != 2) return CHX_EINVAL;
  return solve(p, batch, x_inout, ld, layout, dtype, refine_passes, ws, ws_bytes, s);
}

}  // extern "C"

// Static device scratch of penta_solve_batch_noalloc.  In host code the
// name `scratch` is only a host-side stand-in for the device array: its
// device address (one per GPU) comes from hipGetSymbolAddress, looked up once
// per device and kept here; only that address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[CHX_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch (looked up on first use).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return CHX_EHIP;
  if (dev >= kMaxScratchDevices) return CHX_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CHX_EHIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CHX_OK;
}
}  // namespace

extern "C" {

int penta_solve_batch_noalloc(chx_penta_plan p, int batch, void* x_inout, long ld, int layout,
                              int dtype, int refine_passes, chx_stream s) {
  if (!p) return CHX_EINVAL;
  if (p->P != 2) return CHX_EINVAL;
  if (layout != CHX_INTERLEAVED && layout != CHX_CONTIGUOUS) return CHX_EINVAL;
  if (dtype != CHX_F64 && dtype != CHX_F32_REFINED) return CHX_EINVAL;
  const size_t need = solve_ws(p, batch, layout, dtype);
  if (need > (size_t)CHX_NOALLOC_SCRATCH_BYTES) return CHX_ESCRATCH;
  void* ptr = nullptr;
  if (need > 0) {
    const int rc = scratch_address(&ptr);
    if (rc != CHX_OK) return rc;
  }
  return solve(p, batch, x_inout, ld, layout, dtype, refine_passes, ptr,
               need > 0 ? (size_t)CHX_NOALLOC_SCRATCH_BYTES : 0, s);
}

int tri_factor(int n, double a, double b, double c, int periodic, chx_tri_plan* out) {
  if (!out) return CHX_EINVAL;
  const double coef[3] = {a, b, c};
  return make_plan(1, n, coef, periodic, out);
}

int tri_plan_destroy(chx_tri_plan p) {
  delete p;
  return CHX_OK;
}

size_t tri_solve_ws_bytes(chx_tri_plan p, int batch, int layout, int dtype, int refine_passes) {
  (void)refine_passes;
  return solve_ws(p, batch, layout, dtype);
}

int tri_solve_batch(chx_tri_plan p, int batch, void* x_inout, long ld, int layout, int dtype,
                    int refine_passes, void* ws, size_t ws_bytes, chx_stream s) {
  if (p && p->P != 1) return CHX_EINVAL;
  return solve(p, batch, x_inout, ld, layout, dtype, refine_passes, ws, ws_bytes, s);
}

}  // extern "C"

struct chx_batch1d_s {
  int kind = 0, n = 0;
  double s = 0.0, al = 0.0;
  BandPlan* plan = nullptr;
  ~chx_batch1d_s() { delete plan; }
};

extern "C" {

int batch1d_create(int kind, int n, double L, double dt, double a, double D, chx_batch1d* out) {
  if (!out) return CHX_EINVAL;
  *out = nullptr;
  if (kind < CHX_1D_HYPERDIFFUSION_CN || kind > CHX_1D_CAHN_HILLIARD) return CHX_EINVAL;
  if (!(L > 0) || !(dt > 0) || !(a >= 0) || !(D >= 0) || !std::isfinite(L) ||
      !std::isfinite(dt) || !std::isfinite(a) || !std::isfinite(D))
    return CHX_EINVAL;
  const int P = kind == CHX_1D_DIFFUSION_CN ? 1 : 2;
  if (n < (P == 1 ? 3 : 5)) return CHX_EUNSUPPORTED_N;
  chx_batch1d_s* b = new (std::nothrow) chx_batch1d_s();
  if (!b) return CHX_ENOMEM;
  b->kind = kind;
  b->n = n;
  const double dx = L / n;
  int rc;
  if (kind == CHX_1D_HYPERDIFFUSION_CN) {
    b->s = a * dt / (2.0 * dx * dx * dx * dx);
  } else if (kind == CHX_1D_DIFFUSION_CN) {
    b->s = a * dt / (2.0 * dx * dx);
  } else {
    b->s = a * D * dt / (dx * dx * dx * dx);
    b->al = D * dt / (dx * dx);
  }
  if (P == 1) {
    const double co[3] = {-b->s, 1.0 + 2.0 * b->s, -b->s};
    rc = make_plan(1, n, co, 1, &b->plan);
  } else {
    const double co[5] = {b->s, -4.0 * b->s, 1.0 + 6.0 * b->s, -4.0 * b->s, b->s};
    rc = make_plan(2, n, co, 1, &b->plan);
  }
  if (rc != CHX_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return CHX_OK;
}

int batch1d_destroy(chx_batch1d b) {
  delete b;
  return CHX_OK;
}

size_t batch1d_ws_bytes(chx_batch1d b, int batch) {
  if (!b || batch <= 0) return 0;
  const size_t field = align256((size_t)b->n * batch * sizeof(double));
  if (!b->plan->has_chunk) return field;
  return 2 * field +
         align256((size_t)b->plan->chunk.S * 2 * b->plan->P * (size_t)batch * sizeof(double));
}

int batch1d_step(chx_batch1d b, int batch, double* x, long ld, int nsteps, void* ws,
                 size_t ws_bytes, chx_stream s) {
  if (!b || !x || batch < 0 || nsteps < 1) return CHX_EINVAL;
  if (batch == 0) return CHX_OK;
  if (ld < batch) return CHX_EINVAL;
  if (!ws || ws_bytes < batch1d_ws_bytes(b, batch)) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  auto* base = static_cast<unsigned char*>(ws);
  const size_t field = align256((size_t)b->n * batch * sizeof(double));
  double* y0 = reinterpret_cast<double*>(base);
  double* y1 = reinterpret_cast<double*>(base + field);
  double* rho = reinterpret_cast<double*>(base + 2 * field);
  const hipError_t e =
      launch_batch1d_steps(b->kind, b->plan->has_chunk, b->plan->dchunk, b->plan->dwhole, x, ld,
                           batch, b->n, b->s, b->al, nsteps, y0, y1, rho,
                           static_cast<hipStream_t>(s));
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

// Rewrite mode (the thesis's cuPentBatchRewrite benchmark): per step the
// right-hand side, every system's diagonals written afresh, then a fused
// factor-and-solve of each system; the state ping-pongs between two fields of
// the workspace (pitch batch) and lands in x at the end.
static size_t b1d_field(const chx_batch1d_s* b, int batch) {
  return align256((size_t)b->n * batch * sizeof(double));
}

size_t batch1d_rewrite_ws_bytes(chx_batch1d b, int batch) {
  if (!b || batch <= 0) return 0;
  const int P = b->plan->P;
  return (2 + (2 * P + 1)) * b1d_field(b, batch) + align256(vb_rewrite_ws_bytes(P, b->n, batch));
}

int batch1d_step_rewrite(chx_batch1d b, int batch, double* x, long ld, int nsteps, void* ws,
                         size_t ws_bytes, chx_stream s) {
  if (!b || !x || batch < 0 || nsteps < 1) return CHX_EINVAL;
  if (batch == 0) return CHX_OK;
  if (ld < batch) return CHX_EINVAL;
  if (!ws || ws_bytes < batch1d_rewrite_ws_bytes(b, batch)) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  auto* base = static_cast<unsigned char*>(ws);
  const size_t field = b1d_field(b, batch);
  const int P = b->plan->P, nb = 2 * P + 1, n = b->n;
  double* f[2] = {reinterpret_cast<double*>(base), reinterpret_cast<double*>(base + field)};
  double* bands[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < nb; ++k) bands[k] = reinterpret_cast<double*>(base + (2 + k) * field);
  double* rw = reinterpret_cast<double*>(base + (2 + nb) * field);
  hipError_t e = hipSuccess;
  for (int j = 0; j < nsteps && e == hipSuccess; ++j) {
    const double* src = j == 0 ? x : f[(j - 1) & 1];
    const long lsrc = j == 0 ? ld : (long)batch;
    double* dst = f[j & 1];
    e = launch_batch1d_rhs(b->kind, src, lsrc, dst, batch, batch, n, b->s, b->al, st);
    if (e == hipSuccess) e = vb_fill_bands(nb, bands, b->plan->coef, n, batch, batch, st);
    if (e == hipSuccess)
      e = P == 2 ? vb_penta_rewrite_periodic(n, batch, bands, batch, dst, rw, st)
                 : vb_tri_rewrite_periodic(n, batch, bands, batch, dst, rw, st);
  }
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(x, ld * sizeof(double), f[(nsteps - 1) & 1],
                         (size_t)batch * sizeof(double), (size_t)batch * sizeof(double), n,
                         hipMemcpyDeviceToDevice, st);
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

int stencil2d_apply(const void* in, void* out, int nx, int ny, long ld, int dtype,
                    const double* weights, int left, int right, int top, int bottom, int periodic,
                    int premap, chx_stream s) {
  if (!in || !out || !weights) return CHX_EINVAL;
  if (dtype != CHX_F64 && dtype != CHX_F32) return CHX_EINVAL;
  if (nx < 1 || ny < 1 || ld < nx) return CHX_EINVAL;
  if (left < 0 || right < 0 || top < 0 || bottom < 0) return CHX_EINVAL;
  if (left > 4 || right > 4 || top > 4 || bottom > 4) return CHX_EINVAL;
  if (premap != 0 && premap != 1) return CHX_EINVAL;
  const char* a0 = reinterpret_cast<const char*>(in);
  const char* b0 = reinterpret_cast<const char*>(out);
  const size_t elem = dtype == CHX_F32 ? sizeof(float) : sizeof(double);
  const size_t span = ((size_t)(ny - 1) * ld + nx) * elem;
  if (a0 < b0 + span && b0 < a0 + span) return CHX_EINVAL;  // buffers overlap
  const int nw = (left + right + 1) * (top + bottom + 1);
  if (!finite_all(weights, nw)) return CHX_EINVAL;
  const hipStream_t st = static_cast<hipStream_t>(s);
  hipError_t e =
      dtype == CHX_F32
          ? launch_stencil2d_f32(static_cast<const float*>(in), static_cast<float*>(out), nx, ny,
                                 ld, weights, left, right, top, bottom, periodic ? 1 : 0, premap,
                                 st)
          : launch_stencil2d(static_cast<const double*>(in), static_cast<double*>(out), nx, ny,
                             ld, weights, left, right, top, bottom, periodic ? 1 : 0, premap, st);
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

}  // extern "C"

namespace {

// Autotuning of the multi-kernel step's separator stage: every candidate is
// launched on zeroed scratch buffers of the real size (five rounds captured
// into a graph, replayed once to warm up and once timed with events on a
// private stream): the separator kernel in
// each tile shape whose LDS fits, followed by the row pass, and the split row
// pass in each of its shapes (fused separators + interior rows, then the
// separator rows).  The fastest combination is kept.  Results are cached per
// (grid, chunks, window) for the process, so handles of the same size are
// tuned once.
struct Tuned {
  int red_shape = 0;
  int split = -1;
  int col_order = 0;
  int mcol = kChunk, mrow = kChunk;  // chunk lengths of the column and row solves
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int>, Tuned> g_tune_cache;

size_t device_max_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 64 * 1024;
  }
  return (size_t)v;
}

// Row-split value of the overlapped schedule: the column separator kernel and
// then the separator rows on a second stream, the interior rows beside them.
constexpr int kSplitOverlap = -2;

// Rows of the row plan solved in 16-point chunks: tables built and a row of
// at most 256 chunks (one workgroup per row group).
bool rows16_fit(const BandPlan* px) { return px->has_chunk16 && px->dchunk16.S <= 256; }

// Persistent tuning cache: a text file with one line per tuned size,
//   chx-tune-3 <arch> <nx> <ny> <column plan S dlo dcount> <row plan S dlo dcount>
//       <separator shape> <row split> <column order> <column chunk> <row chunk>
// at $CHX_TUNE_CACHE, else $XDG_CACHE_HOME/chx/tuning.txt, else
// $HOME/.cache/chx/tuning.txt; CHX_TUNE_CACHE=0 turns it off.  Lines are only
// appended; the last line of a key wins; unreadable lines are skipped.
std::string tune_cache_path() {
  const char* env = std::getenv("CHX_TUNE_CACHE");
  if (env) return (env[0] == '\0' || (env[0] == '0' && env[1] == '\0')) ? std::string() : env;
  std::string dir;
  if (const char* x = std::getenv("XDG_CACHE_HOME"); x && x[0]) dir = x;
  else if (const char* hm = std::getenv("HOME"); hm && hm[0]) dir = std::string(hm) + "/.cache";
  else return std::string();
  (void)mkdir(dir.c_str(), 0755);
  dir += "/chx";
  (void)mkdir(dir.c_str(), 0755);
  return dir + "/tuning.txt";
}

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

std::string tune_key_text(const std::string& arch, int nx, int ny, const DevChunk& cy,
                          const DevChunk& cx) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "chx-tune-3 %s %d %d %d %d %d %d %d %d", arch.c_str(), nx, ny,
                cy.S, cy.dlo, cy.dcount, cx.S, cx.dlo, cx.dcount);
  return buf;
}

bool tune_cache_lookup(const std::string& path, const std::string& key, Tuned* out) {
  if (path.empty()) return false;
  std::ifstream in(path);
  std::string line;
  bool found = false;
  while (std::getline(in, line)) {
    if (line.compare(0, key.size(), key) != 0 || line.size() <= key.size() ||
        line[key.size()] != ' ')
      continue;
    Tuned t;
    if (std::sscanf(line.c_str() + key.size(), " %d %d %d %d %d", &t.red_shape, &t.split,
                    &t.col_order, &t.mcol, &t.mrow) != 5)
      continue;
    if (t.red_shape < 0 || t.red_shape >= kNumRedShapes || t.col_order < 0 ||
        t.col_order >= CHX_NUM_COLUMN_ORDERS || t.split < -2 || t.split >= kNumSplitShapes ||
        (t.mcol != 16 && t.mcol != kChunk) || (t.mrow != 16 && t.mrow != kChunk))
      continue;
    *out = t;
    found = true;
  }
  return found;
}

void tune_cache_store(const std::string& path, const std::string& key, const Tuned& t) {
  if (path.empty()) return;
  std::ofstream outf(path, std::ios::app);
  if (outf)
    outf << key << ' ' << t.red_shape << ' ' << t.split << ' ' << t.col_order << ' ' << t.mcol
         << ' ' << t.mrow << '\n';
}

// Times a launch sequence from a captured graph: reps repetitions of run()
// captured once, replayed once to warm up and twice between events, the
// faster replay kept.  On small grids the kernels finish faster than the
// host can launch them one by one, and a timing of eager launches would
// measure the host instead; small grids take more repetitions, so that a
// replay lasts long enough to rank candidates a few per cent apart.
struct GraphTimer {
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = false;
  int reps = 5;
  GraphTimer(long points) {
    reps = points <= (4L << 20) ? 20 : 5;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  }
  ~GraphTimer() {
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
  }
  template <typename F>
  float time(F&& run) {
    float best = -1.f;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    ok = ok && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      bool launched = true;
      for (int k = 0; launched && k < reps; ++k) launched = run() == hipSuccess;
      ok = hipStreamEndCapture(st, &g) == hipSuccess && launched && g != nullptr;
    }
    ok = ok && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess &&
         hipGraphLaunch(ge, st) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k) {
      float ms = -1.f;
      ok = hipEventRecord(e0, st) == hipSuccess && hipGraphLaunch(ge, st) == hipSuccess &&
           hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
           hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      if (ok && (best < 0.f || ms < best)) best = ms;
    }
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    return best;
  }
};

Tuned tune_step(const BandPlan* py, const BandPlan* px, int nx, int ny) {
  const DevChunk& c = py->dchunk;
  const auto key = std::make_tuple(nx, ny, c.S, c.dlo, c.dcount);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end()) return it->second;
  Tuned best;
  const char* env = std::getenv("CHX_AUTOTUNE");
  if (env && env[0] == '0') return best;
  const std::string cache_path = tune_cache_path();
  const std::string cache_key = tune_key_text(device_arch(), nx, ny, c, px->dchunk);
  if (tune_cache_lookup(cache_path, cache_key, &best)) {
    // a split or overlap choice needs the handle's shapes to allow it
    if (best.split >= 0 && !split_fits(c, px->dchunk, best.split)) best.split = -1;
    if (best.mcol == 16 && !py->has_chunk16) best.mcol = kChunk;
    if (best.mrow == 16 && !rows16_fit(px)) best.mrow = kChunk;
    g_tune_cache[key] = best;
    return best;
  }
  // buffers sized for the shorter chunks where the plans have them
  const int Smax = py->has_chunk16 ? py->dchunk16.S : c.S;
  const size_t rho_bytes = (size_t)Smax * 4 * nx * sizeof(double);
  const size_t dst_bytes = (size_t)ny * nx * sizeof(double);
  double *rho = nullptr, *dst = nullptr;
  GraphTimer timer((long)nx * ny);
  hipStream_t st = timer.st;
  bool& ok = timer.ok;
  ok = ok && hipMalloc(&rho, rho_bytes) == hipSuccess && hipMalloc(&dst, dst_bytes) == hipSuccess &&
       hipMemsetAsync(rho, 0, rho_bytes, st) == hipSuccess &&
       hipMemsetAsync(dst, 0, dst_bytes, st) == hipSuccess;
  auto time_it = [&](auto&& run) { return timer.time(run); };
  DevChunk trial = c;
  float best_ms = -1.f;
  const size_t max_lds = std::min(device_max_lds(), kMaxLdsBytes);
  for (int shape = 0; ok && shape < kNumRedShapes; ++shape) {
    if (reduced_lds_bytes(shape, 2, sizeof(double), c.S, c.dcount, true) > max_lds) continue;
    trial.red_shape = shape;
    const float ms = time_it([&]() {
      hipError_t e = launch_reduced_il<2>(trial, rho, nx, dst, nx, kChunk, kChunk - 2, st);
      return e == hipSuccess ? launch_rows_lds<2>(px->dchunk, dst, nx, ny, st) : e;
    });
    if (ok && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      best.red_shape = shape;
    }
  }
  for (int shape = 0; ok && shape < kNumSplitShapes; ++shape) {
    if (!split_fits(c, px->dchunk, shape)) continue;
    const float ms = time_it([&]() {
      hipError_t e = launch_rows_split_fused(shape, c, rho, dst, nx, ny, px->dchunk, nullptr, 0,
                                             0.0, nullptr, st);
      return e == hipSuccess ? launch_rows_sep(dst, nx, ny, px->dchunk, st) : e;
    });
    if (ok && ms < best_ms) {
      best_ms = ms;
      best.split = shape;
    }
  }
  // tile order of the column pass: the pass with its diagnostics, reading
  // the zeroed field as a previous step's buffer (a second field buffer
  // takes its output)
  double *ybuf = nullptr, *part = nullptr;
  const long nparts = ch_column_pass_blocks(nx, Smax);
  // (one more pair: the separator kernel's diagnostics output)
  if (ok && hipMalloc(&ybuf, dst_bytes) == hipSuccess &&
      hipMalloc(&part, (size_t)(nparts + 1) * 2 * sizeof(double)) == hipSuccess) {
    ChCoef K{};
    float best_col = -1.f;
    for (int order = 0; ok && order < CHX_NUM_COLUMN_ORDERS; ++order) {
      const float ms = time_it([&]() {
        return launch_ch_column_pass(true, true, dst, nx, ybuf, nx, nx, ny, c, rho, K, part, st,
                                     nullptr, order);
      });
      if (ok && (best_col < 0.f || ms < best_col)) {
        best_col = ms;
        best.col_order = order;
      }
    }
    // whole steps (column pass, separators, rows) for the separator shape,
    // the chunk lengths (32 or 16 points in each direction where the plans
    // allow them) and the overlapped row order: timed alone on warm
    // buffers, the separator kernel reads its parts from L2, while in a step
    // it reads what the column pass has just written on other XCDs, so
    // shapes rank differently there.  The overlapped order (separators and
    // then the separator rows on a second stream beside the interior rows)
    // is timed with each length pair's best shape.  The fused split forms
    // are 32-point forms, kept only where the plain 32-point step wins.
    hipStream_t side = nullptr;
    hipEvent_t ef = nullptr, ej = nullptr;
    const bool ok2 = hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreateWithFlags(&ef, hipEventDisableTiming) == hipSuccess &&
                     hipEventCreateWithFlags(&ej, hipEventDisableTiming) == hipSuccess;
    const Tuned keep = best;
    // one whole step of a candidate (chunk lengths, separator shape, order),
    // with the diagnostics every step of the benchmark computes: the
    // separator kernel's first block then also finishes their sum, which
    // lengthens shapes that run in a single round of blocks
    double* dout = part + 2 * nparts;
    struct Cand {
      float ms;
      int mc, mr, shape;
      bool overlap;
    };
    auto step_of = [&](const Cand& cd) {
      DevChunk cy = cd.mc == 16 ? py->dchunk16 : py->dchunk;
      const DevChunk& cx = cd.mr == 16 ? px->dchunk16 : px->dchunk;
      cy.red_shape = cd.shape;
      const long colblocks = ch_column_pass_blocks(nx, cy.S);
      return time_it([&]() {
        hipError_t e = launch_ch_column_pass(true, true, dst, nx, ybuf, nx, nx, ny, cy, rho, K,
                                             part, st, nullptr, keep.col_order);
        if (!cd.overlap) {
          if (e == hipSuccess)
            e = launch_reduced_il<2>(cy, rho, nx, ybuf, nx, cy.M, cy.M - 2, st, part, colblocks,
                                     K.dxdy, dout);
          return e == hipSuccess ? launch_rows_lds<2>(cx, ybuf, nx, ny, st) : e;
        }
        if (e == hipSuccess) e = hipEventRecord(ef, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, ef, 0);
        if (e == hipSuccess)
          e = launch_reduced_il<2>(cy, rho, nx, ybuf, nx, cy.M, cy.M - 2, side, part, colblocks,
                                   K.dxdy, dout);
        if (e == hipSuccess) e = launch_rows_subset(true, ybuf, nx, ny, cy.M, cx, side);
        if (e == hipSuccess) e = hipEventRecord(ej, side);
        if (e == hipSuccess) e = launch_rows_subset(false, ybuf, nx, ny, cy.M, cx, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ej, 0);
        return e;
      });
    };
    std::vector<Cand> cands;
    for (int mc : {kChunk, 16}) {
      for (int mr : {kChunk, 16}) {
        if ((mc == 16 && !py->has_chunk16) || (mr == 16 && !rows16_fit(px))) continue;
        const DevChunk& cy = mc == 16 ? py->dchunk16 : py->dchunk;
        Cand pair{-1.f, mc, mr, 0, false};
        for (int shape = 0; ok && shape < kNumRedShapes; ++shape) {
          if (reduced_lds_bytes(shape, 2, sizeof(double), cy.S, cy.dcount, true) > max_lds) continue;
          const Cand cd{step_of(Cand{0.f, mc, mr, shape, false}), mc, mr, shape, false};
          if (!ok) break;
          cands.push_back(cd);
          if (pair.ms < 0.f || cd.ms < pair.ms) pair = cd;
        }
        if (!ok || !ok2 || pair.ms < 0.f) continue;
        const Cand ov{0.f, mc, mr, pair.shape, true};
        const float ms = step_of(ov);
        if (ok) cands.push_back(Cand{ms, mc, mr, pair.shape, true});
      }
    }
    // the closest candidates differ by about the run-to-run spread of one
    // timing: the three fastest (and the fastest whole-column separator
    // shape, if none of them is one) are timed again, in turn, from longer
    // graphs, and the fastest of those rounds decides -- a windowed shape
    // only if it beats the whole-column one by more than 1 %, since it moves
    // more bytes and its lead there has not held up in longer runs
    std::sort(cands.begin(), cands.end(),
              [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
    const Cand* whole = nullptr;
    for (const Cand& cd : cands)
      if (reduced_shape_whole(cd.shape) && (!whole || cd.ms < whole->ms)) whole = &cd;
    const Cand whole_cand = whole ? *whole : Cand{};
    if (cands.size() > 3) cands.resize(3);
    bool have_whole = false;
    for (const Cand& cd : cands) have_whole = have_whole || reduced_shape_whole(cd.shape);
    if (whole && !have_whole) cands.push_back(whole_cand);
    timer.reps *= 4;
    for (Cand& cd : cands) cd.ms = -1.f;
    for (int round = 0; ok && round < 2; ++round) {
      for (Cand& cd : cands) {
        const float ms = step_of(cd);
        if (ok && (cd.ms < 0.f || ms < cd.ms)) cd.ms = ms;
      }
    }
    timer.reps /= 4;
    bool overlap = false;
    if (ok && !cands.empty()) {
      const Cand* win = &cands[0];
      for (const Cand& cd : cands)
        if (cd.ms < win->ms) win = &cd;
      const Cand* wf = nullptr;  // the fastest whole-column finalist
      for (const Cand& cd : cands)
        if (reduced_shape_whole(cd.shape) && (!wf || cd.ms < wf->ms)) wf = &cd;
      if (wf && !reduced_shape_whole(win->shape) && wf->ms <= 1.01f * win->ms) win = wf;
      best.mcol = win->mc;
      best.mrow = win->mr;
      best.red_shape = win->shape;
      overlap = win->overlap;
    }
    if (side) (void)hipStreamSynchronize(side);
    if (ef) (void)hipEventDestroy(ef);
    if (ej) (void)hipEventDestroy(ej);
    if (side) (void)hipStreamDestroy(side);
    if (overlap) best.split = kSplitOverlap;
    else if (best.mcol != kChunk || best.mrow != kChunk) best.split = -1;
  }
  if (st) (void)hipStreamSynchronize(st);
  if (rho) (void)hipFree(rho);
  if (dst) (void)hipFree(dst);
  if (ybuf) (void)hipFree(ybuf);
  if (part) (void)hipFree(part);
  if (!ok) {
    (void)hipGetLastError();  // a failed trial leaves the defaults
    return Tuned{};
  }
  g_tune_cache[key] = best;
  tune_cache_store(cache_path, cache_key, best);
  return best;
}

// The FP32 separator kernel's tile shape for refined handles, timed inside a
// refinement pass (residual and column sweep, separators, row solves) on
// zeroed buffers; cached like tune_step's choices (key "chx-tune-3r ...").
int tune_refined(const BandPlan* py, const BandPlan* px, int nx, int ny, const double* cxs,
                 const double* cys) {
  const DevChunk& c = py->dchunk;
  static std::map<std::tuple<int, int, int, int, int>, int> cache;
  const auto key = std::make_tuple(nx, ny, c.S, c.dlo, c.dcount);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const char* env = std::getenv("CHX_AUTOTUNE");
  if (env && env[0] == '0') return 0;
  const std::string cache_path = tune_cache_path();
  std::string cache_key = tune_key_text(device_arch(), nx, ny, c, px->dchunk);
  cache_key.replace(0, 10, "chx-tune-3r");
  Tuned t;
  if (tune_cache_lookup(cache_path, cache_key, &t)) {
    cache[key] = t.red_shape;
    return t.red_shape;
  }
  const size_t pts = (size_t)nx * ny;
  const size_t b_r = pts * sizeof(double), b_f = pts * sizeof(float);
  const size_t b_rho = (size_t)c.S * 4 * nx * sizeof(float);
  double* r = nullptr;
  float *y32 = nullptr, *rho = nullptr, *v0 = nullptr, *v1 = nullptr;
  GraphTimer timer((long)pts);
  bool& ok = timer.ok;
  ok = ok && hipMalloc(&r, b_r) == hipSuccess && hipMalloc(&y32, b_f) == hipSuccess &&
       hipMalloc(&rho, b_rho) == hipSuccess && hipMalloc(&v0, b_f) == hipSuccess &&
       hipMalloc(&v1, b_f) == hipSuccess && hipMemsetAsync(r, 0, b_r, timer.st) == hipSuccess &&
       hipMemsetAsync(y32, 0, b_f, timer.st) == hipSuccess &&
       hipMemsetAsync(rho, 0, b_rho, timer.st) == hipSuccess &&
       hipMemsetAsync(v0, 0, b_f, timer.st) == hipSuccess &&
       hipMemsetAsync(v1, 0, b_f, timer.st) == hipSuccess;
  const float* V[2] = {v0, v1};
  DevChunk trial = c;
  float best_ms = -1.f;
  const size_t max_lds = std::min(device_max_lds(), kMaxLdsBytes);
  for (int shape = 0; ok && shape < kNumRedShapes; ++shape) {
    if (reduced_lds_bytes(shape, 2, sizeof(float), c.S, c.dcount, false) > max_lds) continue;
    trial.red_shape = shape;
    const float ms = timer.time([&]() {
      hipError_t e = launch_rstep_resid(r, V, 1, y32, rho, nx, ny, c, cxs, cys, timer.st);
      if (e == hipSuccess) e = launch_reduced_il32(trial, rho, nx, y32, nx, timer.st);
      return e == hipSuccess ? launch_rows_lds_f32(px->dchunk, y32, v1, ny, timer.st) : e;
    });
    if (ok && (best_ms < 0.f || ms < best_ms)) {
      best_ms = ms;
      t.red_shape = shape;
    }
  }
  if (timer.st) (void)hipStreamSynchronize(timer.st);
  for (void* p : {(void*)r, (void*)y32, (void*)rho, (void*)v0, (void*)v1})
    if (p) (void)hipFree(p);
  if (!ok) {
    (void)hipGetLastError();
    return 0;
  }
  cache[key] = t.red_shape;
  tune_cache_store(cache_path, cache_key, t);
  return t.red_shape;
}

// Separator work items of the runs in `order` for tile shape `shape`: per
// run, blocks of 64 columns x (the shape's chunks per block) column chunks.
std::vector<int4> ens_red_items(const chx_ens_s* E, const std::vector<int>& order, int shape) {
  const int kb = ens_red_chunks_per_block(shape);
  std::vector<int4> out;
  for (int r : order) {
    const int nby = (E->runs[r].Sc + kb - 1) / kb, nbx = (E->runs[r].nx + 63) / 64;
    for (int by = 0; by < nby; ++by)
      for (int bx = 0; bx < nbx; ++bx) out.push_back(make_int4(r, bx, by, 0));
  }
  return out;
}

// Separator items, LDS and shape of the FP64 ensemble set to shape sh
// (CHX_EINVAL if its LDS does not fit).
int ens_set_red_shape(chx_ens_s* E, int sh) {
  if (sh < 0 || sh >= kNumEnsRedShapes) return CHX_EINVAL;
  size_t lds = 0;
  for (const EnsClass& c : E->classes) lds = std::max(lds, ens_reduced_lds_bytes(c.py.dcount, sh));
  if (lds > std::min(device_max_lds(), kMaxLdsBytes)) return CHX_EINVAL;
  const auto red = ens_red_items(E, E->red_order, sh);
  if (!red.empty() && hipMemcpy(E->ditems + E->o_red, red.data(), sizeof(int4) * red.size(),
                                hipMemcpyHostToDevice) != hipSuccess)
    return CHX_EHIP;
  E->red_shape = sh;
  E->n_red = (int)red.size();
  E->red_lds = lds;
  if (E->refined) {  // items of the runs that make refinement pass k (a prefix)
    for (int k = 0; k < 4; ++k) E->rn_red[k] = 0;
    for (const int4& it : red)
      for (int k = 0; k <= E->prm[it.x].refine_passes; ++k) ++E->rn_red[k];
  }
  return CHX_OK;
}

// Times every separator tile shape on the ensemble's own runs (column pass
// then separators, from a captured graph, on a scratch workspace of the
// ensemble's size) and keeps the fastest; the items are rewritten in place.
// CHX_AUTOTUNE=0 keeps shape 0.  Every shape sums the same terms in the same
// order, so the choice never changes a result.
int ens_tune_red(chx_ens_s* E, const std::vector<int>& order) {
  const char* env = std::getenv("CHX_AUTOTUNE");
  if (env && env[0] == '0') return CHX_OK;
  long points = 0;
  for (int r : order) points += (long)E->runs[r].nx * E->runs[r].ny;
  unsigned char* ws = nullptr;
  GraphTimer timer(points);
  bool& ok = timer.ok;
  ok = ok && hipMalloc(&ws, E->ws_total) == hipSuccess &&
       hipMemsetAsync(ws, 0, E->ws_total, timer.st) == hipSuccess;
  const size_t max_lds = std::min(device_max_lds(), kMaxLdsBytes);
  float best = -1.f;
  int best_shape = 0;
  for (int sh = 0; ok && sh < kNumEnsRedShapes; ++sh) {
    size_t lds = 0;
    for (const EnsClass& c : E->classes)
      lds = std::max(lds, ens_reduced_lds_bytes(c.py.dcount, sh));
    if (lds > max_lds) continue;
    const auto red = ens_red_items(E, order, sh);
    ok = hipMemcpy(E->ditems + E->o_red, red.data(), sizeof(int4) * red.size(),
                   hipMemcpyHostToDevice) == hipSuccess;
    const int n = (int)red.size();
    // FP64: step 1 of a call, the column pass reads the scratch workspace's
    // first buffer (step 0 would read the runs' own fields, which no call has
    // set yet: null pointers here) and writes the second, which the
    // separators then complete.  Refined: refinement pass 1 (its residual
    // reads only workspace buffers) and its FP32 separators.
    const float ms = timer.time([&]() {
      if (E->refined) {
        hipError_t e = launch_ens_rstep_column(1, false, E->druns, E->hcls, E->ditems + E->o_col,
                                               E->rn_col[1], ws, timer.st);
        return e == hipSuccess
                   ? launch_ens_reduced32(E->druns, E->hcls, E->ditems + E->o_red, n, ws, 1,
                                          nullptr, 0, lds, timer.st, sh)
                   : e;
      }
      hipError_t e = launch_ens_column_pass(true, false, nullptr, E->druns, E->hcls,
                                            E->ditems + E->o_col, E->n_col, ws, 1, timer.st);
      return e == hipSuccess ? launch_ens_reduced(E->druns, E->hcls, E->ditems + E->o_red, n, ws,
                                                  1, nullptr, 0, lds, timer.st, sh)
                             : e;
    });
    if (ok && (best < 0.f || ms < best)) {
      best = ms;
      best_shape = sh;
    }
  }
  if (timer.st) (void)hipStreamSynchronize(timer.st);
  if (ws) (void)hipFree(ws);
  if (!ok) (void)hipGetLastError();  // a failed trial leaves shape 0
  return ens_set_red_shape(E, ok ? best_shape : 0);
}

}  // namespace

extern "C" {

static_assert(kNumRedShapes == CHX_NUM_REDUCED_SHAPES, "shape count mismatch");
static_assert(kNumSplitShapes == CHX_NUM_SPLIT_SHAPES, "shape count mismatch");

int ch_create(const chx_ch_params* prm, chx_ch* out) {
  if (!prm || !out) return CHX_EINVAL;
  *out = nullptr;
  const chx_ch_params& q = *prm;
  if (q.nx < 5 || q.ny < 5) return CHX_EUNSUPPORTED_N;
  if (!(q.lx > 0) || !(q.ly > 0) || !(q.dt > 0) || !(q.D >= 0) || !(q.gamma >= 0) ||
      !std::isfinite(q.lx) || !std::isfinite(q.ly) || !std::isfinite(q.dt) ||
      !std::isfinite(q.D) || !std::isfinite(q.gamma))
    return CHX_EINVAL;
  if (q.dtype != CHX_F64 && q.dtype != CHX_F32_REFINED) return CHX_EINVAL;
  if (q.dtype == CHX_F32_REFINED && (q.refine_passes < 1 || q.refine_passes > 3)) return CHX_EINVAL;
  if (q.scheme != CHX_SCHEME_P1 && q.scheme != CHX_SCHEME_P2) return CHX_EINVAL;
  if (q.scheme == CHX_SCHEME_P2 && q.dtype != CHX_F64) return CHX_EINVAL;
  chx_ch_s* h = new (std::nothrow) chx_ch_s();
  if (!h) return CHX_ENOMEM;
  h->prm = q;
  const double dx = q.lx / q.nx, dy = q.ly / q.ny;
  // P2 (the thesis's delta form) factors I + 2/3 D gamma dt d4 per direction
  const double wgt = q.scheme == CHX_SCHEME_P2 ? 2.0 / 3.0 : 1.0;
  const double sx = wgt * q.D * q.gamma * q.dt / (dx * dx * dx * dx);
  const double sy = wgt * q.D * q.gamma * q.dt / (dy * dy * dy * dy);
  const double cxs[5] = {sx, -4 * sx, 1 + 6 * sx, -4 * sx, sx};
  const double cys[5] = {sy, -4 * sy, 1 + 6 * sy, -4 * sy, sy};
  // FP64 P1 handles also carry 16-point chunk tables: on small grids the
  // shorter serial sweeps may beat the 32-point ones (the tuner decides)
  const bool c16 = q.scheme == CHX_SCHEME_P1 && q.dtype == CHX_F64;
  int rc = make_plan(2, q.nx, cxs, 1, &h->px, c16);
  if (rc == CHX_OK) rc = make_plan(2, q.ny, cys, 1, &h->py, c16);
  if (rc != CHX_OK) {
    delete h;
    return rc;
  }
  h->K.cx = q.D * q.dt / (dx * dx);
  h->K.cy = q.D * q.dt / (dy * dy);
  h->K.ccross = 2.0 * q.D * q.gamma * q.dt / (dx * dx * dy * dy);
  h->K.inv_dx = 1.0 / dx;
  h->K.inv_dy = 1.0 / dy;
  h->K.half_gamma = 0.5 * q.gamma;
  h->K.dxdy = dx * dy;
  for (int k = 0; k < 5; ++k) {
    h->cxs[k] = cxs[k];
    h->cys[k] = cys[k];
  }
  h->K2.a = (2.0 / 3.0) * q.D * q.gamma * q.dt;
  h->K2.b = (2.0 / 3.0) * q.D * q.dt;
  h->K2.inv_dx4 = 1.0 / (dx * dx * dx * dx);
  h->K2.inv_dy4 = 1.0 / (dy * dy * dy * dy);
  h->K2.inv_dx2dy2 = 1.0 / (dx * dx * dy * dy);
  h->K2.inv_dx2 = 1.0 / (dx * dx);
  h->K2.inv_dy2 = 1.0 / (dy * dy);
  h->fast = q.scheme == CHX_SCHEME_P1 && (q.nx % 64 == 0) && (q.ny % kChunk == 0) &&
            h->px->has_chunk && h->py->has_chunk && h->px->chunk.S <= 256;
  if (q.dtype == CHX_F32_REFINED && !h->fast) {  // the refined path uses the chunked kernels
    delete h;
    return CHX_EINVAL;
  }
  // FP32 sweeps in each direction: the error of one refined pass is about
  // (kappa_x + kappa_y) 2^-24, the two 1D solves' errors adding
  if (q.dtype == CHX_F32_REFINED && refinement_fails(h->px->kappa + h->py->kappa)) {
    delete h;
    return CHX_EREFINE;
  }
  const size_t field = align256((size_t)q.nx * q.ny * sizeof(double));
  const long diag_parts = ch_diag_partial_blocks(q.nx, q.ny);
  size_t off = 0;
  if (q.dtype == CHX_F32_REFINED) {
    // r (FP64), the FP32 chunk-solved columns, their separator parts, and
    // one FP32 buffer per solve of the step (the deferred solutions V_k)
    const size_t field32 = align256((size_t)q.nx * q.ny * sizeof(float));
    h->off_r = off; off += field;
    h->off_y32 = off; off += field32;
    h->off_rho32 = off;
    off += align256((size_t)h->py->chunk.S * 4 * q.nx * sizeof(float));
    for (int k = 0; k <= q.refine_passes; ++k) {
      h->off_v32[k] = off;
      off += field32;
    }
    h->part_count = std::max(rstep_parts(q.nx, q.ny), diag_parts);
  } else if (h->fast) {
    // separator parts and column-pass partials sized for the shorter chunks
    // where the column plan has them
    const int S = h->py->has_chunk16 ? h->py->chunk16.S : h->py->chunk.S;
    h->off_b0 = off; off += field;
    h->off_b1 = off; off += field;
    h->off_rho = off;
    off += align256((size_t)S * 4 * q.nx * sizeof(double));
    h->part_count = std::max(ch_column_pass_blocks(q.nx, S), diag_parts);
  } else {
    h->off_r = off; off += field;
    if (q.scheme == CHX_SCHEME_P2) {  // a second right-hand side, a third state
      h->off_b0 = off; off += field;
      h->off_b1 = off; off += field;
    }
    if (q.scheme == CHX_SCHEME_P2 && h->py->has_chunk) {  // column solve partials
      h->off_rho = off;
      off += align256((size_t)h->py->chunk.S * 4 * q.nx * sizeof(double));
    }
    h->part_count = diag_parts;
  }
  h->off_part = off;
  off += align256((size_t)h->part_count * 2 * sizeof(double));
  h->ws_total = off;
  h->dscratch_parts = diag_parts;
  if (hipMalloc(&h->dscratch, (size_t)(diag_parts * 2 + 2) * sizeof(double)) != hipSuccess) {
    h->dscratch = nullptr;
    delete h;
    return CHX_EHIP;
  }
  h->small_ok = h->fast && q.dtype == CHX_F64 && ch_small_fits(q.nx, q.ny, device_max_lds());
  h->small = h->small_ok;
  if (h->fast && q.dtype == CHX_F64) {
    if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
      delete h;
      return CHX_EHIP;
    }
  }
  if (q.dtype == CHX_F32_REFINED)
    h->py->dchunk.red_shape = tune_refined(h->py, h->px, q.nx, q.ny, h->cxs, h->cys);
  // the thesis scheme's separators and rows are the same kernels as the P1
  // step's: its separator shape is tuned by the same whole-step timing (on
  // its own plans; 32-point chunks, the only length it takes)
  if (q.scheme == CHX_SCHEME_P2 && h->py->has_chunk && h->px->has_chunk && q.nx % 64 == 0 &&
      h->px->chunk.S <= 256)
    h->py->dchunk.red_shape = tune_step(h->py, h->px, q.nx, q.ny).red_shape;
  if (h->fast && q.dtype == CHX_F64 && !h->small) {
    const Tuned t = tune_step(h->py, h->px, q.nx, q.ny);
    h->py->dchunk.red_shape = t.red_shape;
    h->split = t.split;
    h->col_order = t.col_order;
    h->mcol = t.mcol;
    h->mrow = t.mrow;
  }
  *out = h;
  return CHX_OK;
}

int ch_get_tuning(chx_ch h, int what, int* value) {
  if (!h || !value) return CHX_EINVAL;
  switch (what) {
    case CHX_TUNE_REDUCED_SHAPE: *value = h->py->dchunk.red_shape; return CHX_OK;
    case CHX_TUNE_SMALL_PATH: *value = h->small ? 1 : 0; return CHX_OK;
    case CHX_TUNE_ROW_SPLIT: *value = h->split; return CHX_OK;
    case CHX_TUNE_COLUMN_ORDER: *value = h->col_order; return CHX_OK;
    case CHX_TUNE_GRAPH: *value = h->use_graph ? 1 : 0; return CHX_OK;
    case CHX_TUNE_COLUMN_CHUNK: *value = h->mcol; return CHX_OK;
    case CHX_TUNE_ROW_CHUNK: *value = h->mrow; return CHX_OK;
    default: return CHX_EINVAL;
  }
}

int ch_set_tuning(chx_ch h, int what, int value) {
  if (!h) return CHX_EINVAL;
  h->drop_graph();  // a captured call holds the old choices
  switch (what) {
    case CHX_TUNE_GRAPH:
      if (value != 0 && value != 1) return CHX_EINVAL;
      h->use_graph = value == 1;
      return CHX_OK;
    case CHX_TUNE_REDUCED_SHAPE:
      if (value < 0 || value >= kNumRedShapes) return CHX_EINVAL;
      h->py->dchunk.red_shape = value;
      return CHX_OK;
    case CHX_TUNE_SMALL_PATH:
      if (value != 0 && (value != 1 || !h->small_ok)) return CHX_EINVAL;
      h->small = value == 1;
      return CHX_OK;
    case CHX_TUNE_ROW_SPLIT:
      // the fused split forms are forms of the 32-point chunks; the
      // overlapped order takes either length
      if (value >= 0 && (h->mcol != kChunk || h->mrow != kChunk)) return CHX_EINVAL;
      if (value == kSplitOverlap) {
        if (!h->side) return CHX_EINVAL;
      } else if (value != -1 && !(h->fast && h->prm.dtype == CHX_F64 &&
                                  split_fits(h->py->dchunk, h->px->dchunk, value))) {
        return CHX_EINVAL;
      }
      h->split = value;
      return CHX_OK;
    case CHX_TUNE_COLUMN_CHUNK:
      if (value != kChunk && !(value == 16 && h->fast && h->py->has_chunk16)) return CHX_EINVAL;
      if (value != kChunk && h->split >= 0) return CHX_EINVAL;
      h->mcol = value;
      return CHX_OK;
    case CHX_TUNE_ROW_CHUNK:
      if (value != kChunk && !(value == 16 && h->fast && rows16_fit(h->px))) return CHX_EINVAL;
      if (value != kChunk && h->split >= 0) return CHX_EINVAL;
      h->mrow = value;
      return CHX_OK;
    case CHX_TUNE_COLUMN_ORDER:
      if (value < 0 || value >= CHX_NUM_COLUMN_ORDERS) return CHX_EINVAL;
      h->col_order = value;
      return CHX_OK;
    default: return CHX_EINVAL;
  }
}

int ch_destroy(chx_ch h) {
  delete h;
  return CHX_OK;
}

// The Cook forcing is drawn inside the kernels: no extra workspace.
static size_t ws_need(const chx_ch_s* h) { return h->ws_total; }

size_t ch_ws_bytes(chx_ch h) { return h ? ws_need(h) : 0; }

int ch_set_noise(chx_ch h, double sigma, unsigned long long seed, unsigned long long step0) {
  if (!h || !(sigma >= 0) || !std::isfinite(sigma)) return CHX_EINVAL;
  if (sigma > 0 && !(h->fast && h->prm.dtype == CHX_F64 && h->prm.scheme == CHX_SCHEME_P1))
    return CHX_EINVAL;
  h->sigma = sigma;
  h->noise_seed = seed;
  h->noise_step = step0;
  return CHX_OK;
}

int ch_get_noise_step(chx_ch h, unsigned long long* step) {
  if (!h || !step) return CHX_EINVAL;
  *step = h->noise_step;
  return CHX_OK;
}

// Per-phase event timing of ch_adi_step (phase 0 column pass, 1 column
// separators, 2 row pass, 3 finalize + diagnostics reductions).  Every event
// is created before the first launch (reserve), so the launch sequence only
// records events: no event creation between kernels.
struct PhaseTimer {
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev;  // created up front
  size_t used = 0;
  std::vector<int> phase;
  bool failed = false;
  int every = 1;    // time the kernels of every `every`-th step (and the last launches)
  bool on = true;   // timing the current step
  bool reserve(size_t n) {
    ev.reserve(n);
    for (size_t k = 0; k < n; ++k) {
      hipEvent_t a;
      if (hipEventCreate(&a) != hipSuccess) return false;
      ev.push_back(a);
    }
    phase.reserve(n / 2);
    return true;
  }
  void step(int n) { on = (n % every) == 0; }
  void record() {
    if (used >= ev.size()) { failed = true; return; }
    if (hipEventRecord(ev[used++], st) != hipSuccess) failed = true;
  }
  void begin() { record(); }
  void end(int ph) {
    phase.push_back(ph);
    record();
  }
  ~PhaseTimer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

static int run_steps(chx_ch h, double* c, long ld, int nsteps, double* diag_out, void* ws,
                     size_t ws_bytes, hipStream_t st, PhaseTimer* tm) {
  if (!h || !c) return CHX_EINVAL;
  if (h->prm.scheme != CHX_SCHEME_P1) return CHX_EINVAL;  // P2 handles: ch_adi_step_p2
  const int nx = h->prm.nx, ny = h->prm.ny;
  if (ld < nx || nsteps < 1) return CHX_EINVAL;
  if (!ws || ws_bytes < ws_need(h)) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  auto* base = static_cast<unsigned char*>(ws);
  double* part = reinterpret_cast<double*>(base + h->off_part);
  const bool noise = h->sigma > 0;
  // the forcing's draw parameters of step k of this call
  auto noise_of = [&](int k) {
    const double dx = h->prm.lx / nx, dy = h->prm.ly / ny;
    return SmallNoise{chx_sm_mix(h->noise_seed), h->noise_step + (unsigned long long)k,
                      h->prm.dt * std::sqrt(h->sigma / (dx * dy * h->prm.dt)), 1.0 / dx, 1.0 / dy};
  };
  hipError_t e = hipSuccess;
  auto ok = [&]() { return e == hipSuccess; };
  auto B = [&]() { if (tm && tm->on) tm->begin(); };
  auto E = [&](int ph) { if (tm && tm->on) tm->end(ph); };
  if (h->prm.dtype == CHX_F32_REFINED) {
    // pass 0: r = RHS(c) (FP64, kept) swept in FP32 down the columns, the
    // FP32 separators, FP32 row solves into V_0; pass k: R = r - A x_{k-1}
    // (x_{k-1} rebuilt from V_0 .. V_{k-1}) swept the same way into V_k;
    // then c = x_p, with the final state's diagnostics on the last step
    double* r = reinterpret_cast<double*>(base + h->off_r);
    float* y32 = reinterpret_cast<float*>(base + h->off_y32);
    float* rho32 = reinterpret_cast<float*>(base + h->off_rho32);
    const int np = h->prm.refine_passes;
    float* V[4] = {};
    for (int k = 0; k <= np; ++k) V[k] = reinterpret_cast<float*>(base + h->off_v32[k]);
    const long rparts = rstep_parts(nx, ny);
    for (int n = 0; n < nsteps && ok(); ++n) {
      if (tm) tm->step(n);
      const bool diag = diag_out != nullptr;
      // every step after the first rebuilds its state from the previous
      // step's solutions, which stay in the workspace (c is written once,
      // after the last step)
      B();
      e = launch_rstep_first(c, ld, r, y32, rho32, nx, ny, h->py->dchunk, h->K,
                             diag ? part : nullptr, st, V, n > 0 ? np + 1 : 0);
      E(0);
      if (ok()) {
        B();
        e = launch_reduced_il32(h->py->dchunk, rho32, nx, y32, nx, st, diag ? part : nullptr,
                                diag ? rparts : 0, h->K.dxdy, diag ? diag_out + 2 * n : nullptr);
        E(1);
      }
      if (ok()) {
        B();
        e = launch_rows_lds_f32(h->px->dchunk, y32, V[0], ny, st);
        E(2);
      }
      for (int k = 1; k <= np && ok(); ++k) {
        B();
        e = launch_rstep_resid(r, V, k, y32, rho32, nx, ny, h->py->dchunk, h->cxs, h->cys, st);
        E(0);
        if (ok()) {
          B();
          e = launch_reduced_il32(h->py->dchunk, rho32, nx, y32, nx, st);
          E(1);
        }
        if (ok()) {
          B();
          e = launch_rows_lds_f32(h->px->dchunk, y32, V[k], ny, st);
          E(2);
        }
      }
      if (ok() && n + 1 == nsteps) {
        if (tm) tm->on = true;
        B();
        e = launch_rstep_final(V, np + 1, c, ld, nx, ny, h->py->dchunk, h->K, part,
                               diag ? diag_out + 2 * nsteps : nullptr, st);
        E(3);
      }
    }
    if (tm && tm->failed) return CHX_EHIP;
    return ok() ? CHX_OK : CHX_EHIP;
  } else if (h->small) {
    // one workgroup, field resident in LDS for all steps; it also writes the
    // diagnostics of every state, the final one included
    B();
    const SmallNoise nz = noise_of(0);
    e = launch_ch_small_steps(c, ld, nx, ny, nsteps, h->py->dchunk, h->px->dchunk, h->K, diag_out,
                              noise ? &nz : nullptr, st);
    E(0);
    if (ok() && noise) h->noise_step += (unsigned long long)nsteps;
    if (tm && tm->failed) return CHX_EHIP;
    return ok() ? CHX_OK : CHX_EHIP;
  } else if (h->fast) {
    double* buf[2] = {reinterpret_cast<double*>(base + h->off_b0),
                      reinterpret_cast<double*>(base + h->off_b1)};
    double* rho = reinterpret_cast<double*>(base + h->off_rho);
    const double* src = c;
    long lds = ld;
    bool recon = false;
    // the chunk plans of the two directions (the separator shape is chosen
    // on the 32-point plan and applies to either)
    DevChunk cy = h->mcol == 16 ? h->py->dchunk16 : h->py->dchunk;
    cy.red_shape = h->py->dchunk.red_shape;
    const DevChunk& cx = h->mrow == 16 ? h->px->dchunk16 : h->px->dchunk;
    const long colblocks = ch_column_pass_blocks(nx, cy.S);
    for (int n = 0; n < nsteps && ok(); ++n) {
      if (tm) tm->step(n);
      double* dst = buf[n & 1];
      const bool diag = diag_out != nullptr;
      if (ok()) {
        B();
        const SmallNoise nz = noise_of(n);  // Cahn-Hilliard-Cook draws of this step
        e = launch_ch_column_pass(recon, diag, src, lds, dst, nx, nx, ny, cy, rho,
                                  h->K, part, st, noise ? &nz : nullptr, h->col_order);
        E(0);
      }
      if (ok() && h->split == kSplitOverlap && !(tm && tm->on)) {
        // separators, then the separator rows, on the second stream; the
        // interior rows (which need no separator) beside them on st
        e = hipEventRecord(h->ev_fork, st);
        if (ok()) e = hipStreamWaitEvent(h->side, h->ev_fork, 0);
        if (ok()) {
          e = launch_reduced_il<2>(cy, rho, nx, dst, nx, cy.M, cy.M - 2, h->side,
                                   diag ? part : nullptr, diag ? colblocks : 0, h->K.dxdy,
                                   diag ? diag_out + 2 * n : nullptr);
          if (e == hipSuccess) e = launch_rows_subset(true, dst, nx, ny, cy.M, cx, h->side);
          // join even after a failure, so no capture is left forked
          const hipError_t j1 = hipEventRecord(h->ev_join, h->side);
          if (e == hipSuccess) e = launch_rows_subset(false, dst, nx, ny, cy.M, cx, st);
          const hipError_t j2 = hipStreamWaitEvent(st, h->ev_join, 0);
          if (e == hipSuccess) e = j1 != hipSuccess ? j1 : j2;
        }
      } else if (ok() && h->split >= 0) {
        // separators fused with the interior rows (phase 2), then the
        // separator rows (phase 1)
        B();
        e = launch_rows_split_fused(h->split, h->py->dchunk, rho, dst, nx, ny, h->px->dchunk,
                                    diag ? part : nullptr, diag ? colblocks : 0, h->K.dxdy,
                                    diag ? diag_out + 2 * n : nullptr, st);
        E(2);
        if (ok()) {
          B();
          e = launch_rows_sep(dst, nx, ny, h->px->dchunk, st);
          E(1);
        }
      } else {
        if (ok()) {
          B();
          e = launch_reduced_il<2>(cy, rho, nx, dst, nx, cy.M, cy.M - 2, st,
                                   diag ? part : nullptr, diag ? colblocks : 0, h->K.dxdy,
                                   diag ? diag_out + 2 * n : nullptr);
          E(1);
        }
        if (ok()) {
          B();
          e = launch_rows_lds<2>(cx, dst, nx, ny, st);
          E(2);
        }
      }
      src = dst;
      lds = nx;
      recon = true;
    }
    if (tm) tm->on = true;
    if (ok()) {
      // the state written out with the final diagnostics in the same pass
      B();
      e = launch_ch_column_final(src, lds, c, ld, nx, ny, cy, h->K, part,
                                 diag_out ? diag_out + 2 * nsteps : nullptr, st, h->col_order);
      E(3);
    }
    if (ok() && noise) h->noise_step += (unsigned long long)nsteps;
    if (tm && tm->failed) return CHX_EHIP;
    return ok() ? CHX_OK : CHX_EHIP;
  } else {
    double* r = reinterpret_cast<double*>(base + h->off_r);
    for (int n = 0; n < nsteps && ok(); ++n) {
      if (tm) tm->step(n);
      if (diag_out) {
        B();
        e = launch_ch_diag(c, ld, nx, ny, h->K, part, diag_out + 2 * n, st);
        E(3);
      }
      if (ok()) {
        B();
        e = launch_ch_rhs_plain(c, ld, r, nx, nx, ny, h->K, st);
        E(0);
      }
      if (ok()) {
        B();
        e = launch_whole<2>(h->py->dwhole, r, 1, nx, nx, st);
        E(0);
      }
      if (ok()) {
        B();
        e = launch_whole<2>(h->px->dwhole, r, nx, 1, ny, st);
        E(2);
      }
      if (ok()) {
        B();
        e = hipMemcpy2DAsync(c, ld * sizeof(double), r, nx * sizeof(double), nx * sizeof(double),
                             ny, hipMemcpyDeviceToDevice, st);
        E(3);
      }
    }
  }
  if (tm) tm->on = true;
  if (ok() && diag_out) {
    B();
    e = launch_ch_diag(c, ld, nx, ny, h->K, part, diag_out + 2 * nsteps, st);
    E(3);
  }
  if (ok() && noise) h->noise_step += (unsigned long long)nsteps;
  if (tm && tm->failed) return CHX_EHIP;
  return ok() ? CHX_OK : CHX_EHIP;
}

namespace {
// An FP32-refined ensemble: the refined step's phases, one launch per phase
// for all runs (pass k covers the runs with at least k refine passes).
int ens_launch_refined(chx_ens_s* E, int nsteps, double* diag_out, unsigned char* ws,
                       hipStream_t st) {
  const long dstride = 2L * (nsteps + 1);
  const int4* it = E->ditems;
  hipError_t e = hipSuccess;
  for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
    for (int k = 0; k <= E->max_passes && e == hipSuccess; ++k) {
      e = launch_ens_rstep_column(k, k == 0 && diag_out, E->druns, E->hcls, it + E->o_col,
                                  E->rn_col[k], ws, st, k == 0 && n > 0);
      if (e == hipSuccess)
        e = launch_ens_reduced32(E->druns, E->hcls, it + E->o_red, E->rn_red[k], ws, n,
                                 k == 0 ? diag_out : nullptr, dstride, E->red_lds, st,
                                 E->red_shape);
      if (e == hipSuccess)
        e = launch_ens_rows32(E->druns, E->hcls, it + E->o_row, E->rn_row[k], ws, k, st);
    }
    if (e == hipSuccess && n + 1 == nsteps)
      e = launch_ens_rstep_final(E->druns, E->hcls, it + E->o_col, E->rn_col[0], E->dbig,
                                 E->nbig, ws, diag_out, dstride, nsteps, st);
  }
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}
}  // namespace

int ch_adi_step_p2(chx_ch h, double* c, double* cprev, long ld, int nsteps, double* diag_out,
                   void* ws, size_t ws_bytes, chx_stream s) {
  if (!h || !c || !cprev) return CHX_EINVAL;
  if (h->prm.scheme != CHX_SCHEME_P2) return CHX_EINVAL;
  const int nx = h->prm.nx, ny = h->prm.ny;
  if (ld < nx || nsteps < 1) return CHX_EINVAL;
  if (!ws || ws_bytes < h->ws_total) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  {  // the two states must not overlap
    const char* a = reinterpret_cast<const char*>(c);
    const char* b = reinterpret_cast<const char*>(cprev);
    const size_t span = ((size_t)(ny - 1) * ld + nx) * sizeof(double);
    if (a < b + span && b < a + span) return CHX_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(s);
  auto* base = static_cast<unsigned char*>(ws);
  double* rbuf[2] = {reinterpret_cast<double*>(base + h->off_r),
                     reinterpret_cast<double*>(base + h->off_b0)};
  double* w = reinterpret_cast<double*>(base + h->off_b1);
  double* rho = reinterpret_cast<double*>(base + h->off_rho);
  double* part = reinterpret_cast<double*>(base + h->off_part);
  const bool col_chunk = h->py->has_chunk;
  const bool row_lds = h->px->has_chunk && h->px->chunk.S <= 256;
  hipError_t e = hipSuccess;
  // v = L_y^{-1} L_x^{-1} r in place: columns (interleaved), then rows
  // (chunked columns: the chunk correction is left to whoever reads r next)
  const DevChunk* recon = col_chunk ? &h->py->dchunk : nullptr;
  // with chunked columns the right-hand-side kernel has already run the
  // column chunk sweep (y in r, separator parts in rho)
  const DevChunk* sweep = col_chunk ? &h->py->dchunk : nullptr;
  auto solve_in_place = [&](double* r) {
    hipError_t e2 = col_chunk ? launch_reduced_il<2>(h->py->dchunk, rho, nx, r, nx, kChunk,
                                                     kChunk - 2, st)
                              : launch_whole<2>(h->py->dwhole, r, 1, nx, nx, st);
    if (e2 == hipSuccess)
      e2 = row_lds ? launch_rows_lds<2>(h->px->dchunk, r, nx, ny, st)
                   : launch_whole<2>(h->px->dwhole, r, nx, 1, ny, st);
    return e2;
  };
  // The states rotate through c, cprev and w: each later step advances the
  // state inside the right-hand-side kernel (C_new = 2C - Cp + v, written to
  // the buffer holding neither input) and the last update lands in c, cprev.
  struct Buf {
    double* p;
    long ld;
  };
  Buf cur{c, ld}, prev{cprev, ld}, spare{w, nx};
  if (diag_out) e = launch_ch_diag(c, ld, nx, ny, h->K, part, diag_out, st);
  if (e == hipSuccess)
    e = launch_ch2_rhs(c, ld, cprev, ld, nullptr, 0, nullptr, 0, rbuf[0], nx, nx, ny, h->K2,
                       nullptr, sweep, rho, st);
  if (e == hipSuccess) e = solve_in_place(rbuf[0]);
  for (int n = 1; n < nsteps && e == hipSuccess; ++n) {
    double* rv = rbuf[(n - 1) & 1];
    double* rn = rbuf[n & 1];
    e = launch_ch2_rhs(cur.p, cur.ld, prev.p, prev.ld, rv, nx, spare.p, spare.ld, rn, nx, nx, ny,
                       h->K2, recon, sweep, rho, st);
    if (e == hipSuccess && diag_out)
      e = launch_ch_diag(spare.p, spare.ld, nx, ny, h->K, part, diag_out + 2 * n, st);
    const Buf old_prev = prev;
    prev = cur;
    cur = spare;
    spare = old_prev;
    if (e == hipSuccess) e = solve_in_place(rn);
  }
  if (e == hipSuccess)
    e = launch_ch2_update(cur.p, cur.ld, prev.p, prev.ld, rbuf[(nsteps - 1) & 1], nx, c, cprev,
                          ld, nx, ny, recon, st);
  if (e == hipSuccess && diag_out)
    e = launch_ch_diag(c, ld, nx, ny, h->K, part, diag_out + 2 * nsteps, st);
  return e == hipSuccess ? CHX_OK : CHX_EHIP;
}

int ch_adi_step(chx_ch h, double* c, long ld, int nsteps, double* diag_out, void* ws,
                size_t ws_bytes, chx_stream s) {
  hipStream_t st = static_cast<hipStream_t>(s);
  // forced handles draw new noise every call (host-side step counter) and
  // the single-workgroup path is one launch already: both run eagerly
  if (!h || !h->use_graph || h->sigma > 0 || h->small)
    return run_steps(h, c, ld, nsteps, diag_out, ws, ws_bytes, st, nullptr);
  // the argument checks run_steps makes, before anything is captured
  if (!c || h->prm.scheme != CHX_SCHEME_P1 || ld < h->prm.nx || nsteps < 1) return CHX_EINVAL;
  if (!ws || ws_bytes < ws_need(h)) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  if (!h->gexec || h->g_c != c || h->g_ld != ld || h->g_nsteps != nsteps ||
      h->g_diag != diag_out || h->g_ws != ws) {
    h->drop_graph();
    if (!h->cap && hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
      h->cap = nullptr;
      return CHX_EHIP;
    }
    if (!h->g_done && hipEventCreateWithFlags(&h->g_done, hipEventDisableTiming) != hipSuccess) {
      h->g_done = nullptr;
      return CHX_EHIP;
    }
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return CHX_EHIP;
    const int rc = run_steps(h, c, ld, nsteps, diag_out, ws, ws_bytes, h->cap, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(h->cap, &g);
    if (rc != CHX_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != CHX_OK ? rc : CHX_EHIP;
    }
    if (hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      h->gexec = nullptr;
      return CHX_EHIP;
    }
    h->graph = g;
    h->g_c = c;
    h->g_ld = ld;
    h->g_nsteps = nsteps;
    h->g_diag = diag_out;
    h->g_ws = ws;
  }
  if (hipGraphLaunch(h->gexec, st) != hipSuccess) return CHX_EHIP;
  return hipEventRecord(h->g_done, st) == hipSuccess ? CHX_OK : CHX_EHIP;
}

int ch_adi_step_timed(chx_ch h, double* c, long ld, int nsteps, double* diag_out, void* ws,
                      size_t ws_bytes, chx_stream s, int sample_every, double* phase_ms,
                      int* phase_launches) {
  if (!phase_ms || !phase_launches || sample_every < 1) return CHX_EINVAL;
  PhaseTimer tm;
  tm.st = static_cast<hipStream_t>(s);
  tm.every = sample_every;
  // at most 13 timed launches per sampled step (the refined step with 3
  // passes and diagnostics: 4 + 3 per pass), and 4 around the call
  const size_t sampled = (size_t)(nsteps / sample_every) + 1;
  if (!tm.reserve(2 * (16 * sampled + 4))) return CHX_EHIP;
  int rc = run_steps(h, c, ld, nsteps, diag_out, ws, ws_bytes, tm.st, &tm);
  if (rc) return rc;
  if (hipStreamSynchronize(tm.st) != hipSuccess) return CHX_EHIP;
  for (int k = 0; k < 4; ++k) {
    phase_ms[k] = 0.0;
    phase_launches[k] = 0;
  }
  for (size_t k = 0; k < tm.phase.size(); ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, tm.ev[2 * k], tm.ev[2 * k + 1]) != hipSuccess) return CHX_EHIP;
    phase_ms[tm.phase[k]] += ms;
    phase_launches[tm.phase[k]] += 1;
  }
  return CHX_OK;
}

int ch_diagnostics(chx_ch h, const double* c, long ld, double* mass, double* energy,
                   chx_stream s) {
  if (!h || !c || !mass || !energy) return CHX_EINVAL;
  if (ld < h->prm.nx) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* out = h->dscratch + 2 * h->dscratch_parts;
  hipError_t e = launch_ch_diag(c, ld, h->prm.nx, h->prm.ny, h->K, h->dscratch, out, st);
  double host[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, out, sizeof(host), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return CHX_EHIP;
  *mass = host[0];
  *energy = host[1];
  if (!std::isfinite(host[0]) || !std::isfinite(host[1])) return CHX_ENONFINITE;
  return CHX_OK;
}

int ch_energy_decay_rate(const double* diag, int nruns, int nstates, double t0, double dt,
                         double* beta, chx_stream s) {
  if (!diag || !beta || nruns < 1 || nstates < 3 || !(dt > 0) || !std::isfinite(dt) ||
      !std::isfinite(t0))
    return CHX_EINVAL;
  const char* a = reinterpret_cast<const char*>(diag);
  const char* b = reinterpret_cast<const char*>(beta);
  const size_t na = (size_t)nruns * 2 * nstates * sizeof(double);
  const size_t nb = (size_t)nruns * nstates * sizeof(double);
  if (a < b + nb && b < a + na) return CHX_EINVAL;  // overlapping buffers
  return launch_ch_decay_rate(diag, nruns, nstates, t0, dt, beta, static_cast<hipStream_t>(s)) ==
                 hipSuccess
             ? CHX_OK
             : CHX_EHIP;
}

int ch_moments(chx_ch h, const double* c, long ld, double* out, chx_stream s) {
  if (!h || !c || !out) return CHX_EINVAL;
  if (ld < h->prm.nx || (h->prm.nx & 1) || (h->prm.ny & 1)) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  double* dev = h->dscratch + 2 * h->dscratch_parts;
  hipError_t e = launch_ch_simpson(c, ld, h->prm.nx, h->prm.ny, h->dscratch, dev, st);
  double host[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, dev, sizeof(host), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return CHX_EHIP;
  out[0] = host[0];
  out[1] = host[1];
  out[2] = 1.0 / (1.0 - host[1]);
  if (!std::isfinite(host[0]) || !std::isfinite(host[1])) return CHX_ENONFINITE;
  return CHX_OK;
}

int ch_k1(chx_ch h, const double* c, long ld, double* k1, chx_stream s) {
  if (!h || !c || !k1) return CHX_EINVAL;
  const int nx = h->prm.nx, ny = h->prm.ny;
  if (ld < nx) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  const size_t real_b = align256((size_t)nx * ny * sizeof(double));
  const size_t spec_b = align256((size_t)(nx / 2 + 1) * ny * sizeof(double2));
  const long nb = ch_k1_blocks(nx, ny);
  const size_t part_b = align256((size_t)(2 * nb + 2) * sizeof(double));
  if (!h->fft_ready) {
    if (hipMalloc(&h->fft_mem, real_b + spec_b + part_b) != hipSuccess) {
      h->fft_mem = nullptr;
      return CHX_ENOMEM;
    }
    if (hipfftPlan2d(&h->fft, ny, nx, HIPFFT_D2Z) != HIPFFT_SUCCESS) return CHX_EHIP;
    h->fft_ready = true;
  }
  auto* base = static_cast<unsigned char*>(h->fft_mem);
  double* real = reinterpret_cast<double*>(base);
  auto* spec = reinterpret_cast<double2*>(base + real_b);
  double* part = reinterpret_cast<double*>(base + real_b + spec_b);
  double* dout = part + 2 * nb;
  // the transform takes a compact copy (it may also overwrite its input)
  hipError_t e = hipMemcpy2DAsync(real, nx * sizeof(double), c, ld * sizeof(double),
                                  nx * sizeof(double), ny, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return CHX_EHIP;
  if (hipfftSetStream(h->fft, st) != HIPFFT_SUCCESS ||
      hipfftExecD2Z(h->fft, real, reinterpret_cast<hipfftDoubleComplex*>(spec)) != HIPFFT_SUCCESS)
    return CHX_EHIP;
  e = launch_ch_k1(spec, nx, ny, h->prm.lx, h->prm.ly, part, dout, st);
  double host[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, dout, sizeof(host), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return CHX_EHIP;
  *k1 = host[0] / host[1];
  return std::isfinite(*k1) ? CHX_OK : CHX_ENONFINITE;
}

// FP32-refined ensemble: a class is a (grid, parameters, refinement passes)
// combination; each gets one refined single-run handle.
static int ens_create_refined(chx_ens_s* E) {
  E->refined = true;
  const int nruns = E->nruns;
  const std::vector<chx_ch_params>& prm = E->prm;
  std::vector<int> cls_of(nruns, -1);
  std::vector<chx_ch_params> reps;
  for (int r = 0; r < nruns; ++r) {
    const chx_ch_params& q = prm[r];
    if (q.scheme != CHX_SCHEME_P1 || q.nx % 64 != 0 || q.ny % kChunk != 0 ||
        q.nx / kChunk > 256 || q.refine_passes < 1 || q.refine_passes > 3 || !(q.lx > 0) ||
        !(q.ly > 0) || !(q.dt > 0) || !(q.D >= 0) || !(q.gamma >= 0))
      return CHX_EINVAL;
    for (size_t c = 0; c < reps.size(); ++c)
      if (same_grid(reps[c], q)) cls_of[r] = (int)c;
    if (cls_of[r] < 0) {
      if ((int)reps.size() == kEnsMaxClasses) return CHX_EINVAL;
      cls_of[r] = (int)reps.size();
      reps.push_back(q);
    }
    E->max_passes = std::max(E->max_passes, q.refine_passes);
  }
  size_t lds_max = 0;
  for (const auto& q : reps) {  // the plans ch_create makes for such a run
    const double dx = q.lx / q.nx, dy = q.ly / q.ny;
    const double sx = q.D * q.gamma * q.dt / (dx * dx * dx * dx);
    const double sy = q.D * q.gamma * q.dt / (dy * dy * dy * dy);
    const double cxs[5] = {sx, -4 * sx, 1 + 6 * sx, -4 * sx, sx};
    const double cys[5] = {sy, -4 * sy, 1 + 6 * sy, -4 * sy, sy};
    BandPlan *a = nullptr, *b = nullptr;
    int rc = make_plan(2, q.nx, cxs, 1, &a);
    if (rc == CHX_OK) rc = make_plan(2, q.ny, cys, 1, &b);
    if (rc == CHX_OK && (!a->has_chunk || !b->has_chunk)) rc = CHX_EINVAL;
    if (rc == CHX_OK && refinement_fails(a->kappa + b->kappa)) rc = CHX_EREFINE;
    E->px.push_back(a);
    E->py.push_back(b);
    if (rc != CHX_OK) return rc;
    EnsClass ec;
    ec.px = a->dchunk;
    ec.py = b->dchunk;
    ec.K = make_coef(q);
    E->classes.push_back(ec);
    lds_max = std::max(lds_max, ens_reduced_lds_bytes(b->chunk.dcount));
  }
  if (lds_max > 64 * 1024) return CHX_EINVAL;
  E->red_lds = lds_max;
  // more passes first, then larger runs first
  std::vector<int> order(nruns);
  for (int r = 0; r < nruns; ++r) order[r] = r;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (prm[a].refine_passes != prm[b].refine_passes)
      return prm[a].refine_passes > prm[b].refine_passes;
    return (long)prm[a].nx * prm[a].ny > (long)prm[b].nx * prm[b].ny;
  });
  size_t off = 0;
  E->runs.resize(nruns);
  for (int r = 0; r < nruns; ++r) {
    const chx_ch_params& q = prm[r];
    EnsRun& R = E->runs[r];
    std::memset(&R, 0, sizeof(R));
    R.ldc = q.nx;
    R.nx = q.nx;
    R.ny = q.ny;
    R.cls = cls_of[r];
    R.Sc = q.ny / kChunk;
    R.passes = q.refine_passes;
    R.nseg = rstep_segments(q.nx);
    R.ncb = (R.nseg + 3) / 4;
    R.ncolblocks = (long)R.nseg * R.Sc;  // (mass, energy) partials of the column kernels
    const size_t field = align256((size_t)q.nx * q.ny * sizeof(double));
    const size_t field32 = align256((size_t)q.nx * q.ny * sizeof(float));
    R.off_r = off; off += field;
    R.off_y32 = off; off += field32;
    R.off_rho32 = off; off += align256((size_t)R.Sc * 4 * q.nx * sizeof(float));
    for (int k = 0; k <= R.passes; ++k) {
      R.off_v[k] = off;
      off += field32;
    }
    R.off_part = off;
    off += align256((size_t)R.ncolblocks * 2 * sizeof(double));
    E->max_points = std::max(E->max_points, (long)q.nx * q.ny);
  }
  E->ws_total = std::max(off, (size_t)256);
  std::vector<int4> items;
  auto add = [&](int r, int a, int b) { items.push_back(make_int4(r, a, b, 0)); };
  auto prefix = [&](int (&cnt)[4], long o) {
    for (int k = 0; k < 4; ++k) cnt[k] = 0;
    for (size_t t = (size_t)o; t < items.size(); ++t)
      for (int k = 0; k <= prm[items[t].x].refine_passes; ++k) ++cnt[k];
  };
  E->o_col = (long)items.size();
  for (int r : order) {  // blocks of four (segment, chunk) pairs of the run
    const long pairs = (long)E->runs[r].nseg * E->runs[r].Sc;
    for (long b = 0; b < (pairs + 3) / 4; ++b) add(r, (int)b, 0);
  }
  prefix(E->rn_col, E->o_col);
  E->o_row = (long)items.size();
  for (int r : order) {
    const int S = E->runs[r].nx / kChunk, R = 256 / S;
    const int ng = (E->runs[r].ny + R - 1) / R;
    for (int g = 0; g < ng; ++g) add(r, g, 0);
  }
  prefix(E->rn_row, E->o_row);
  // the separator items last: their count depends on the tile shape that
  // creation times (room for the shape with the most blocks)
  E->o_red = (long)items.size();
  size_t max_red = 0;
  for (int sh = 0; sh < kNumEnsRedShapes; ++sh)
    max_red = std::max(max_red, ens_red_items(E, order, sh).size());
  {
    const auto red = ens_red_items(E, order, 0);
    items.insert(items.end(), red.begin(), red.end());
  }
  prefix(E->rn_red, E->o_red);
  E->n_red = (int)(items.size() - E->o_red);
  E->red_order = order;
  E->nbig = nruns;
  for (size_t c = 0; c < E->classes.size(); ++c) E->hcls.c[c] = E->classes[c];
  const size_t b_runs = align256(sizeof(EnsRun) * nruns);
  const size_t b_items =
      align256(sizeof(int4) * std::max<size_t>(E->o_red + max_red, 1));
  const size_t b_lists = align256(sizeof(int) * nruns);
  if (hipMalloc(&E->dmem, b_runs + b_items + b_lists) != hipSuccess) {
    E->dmem = nullptr;
    return CHX_EHIP;
  }
  auto* base = static_cast<unsigned char*>(E->dmem);
  E->druns = reinterpret_cast<EnsRun*>(base);
  E->ditems = reinterpret_cast<int4*>(base + b_runs);
  E->dbig = reinterpret_cast<int*>(base + b_runs + b_items);
  bool ok = hipMemcpy(E->druns, E->runs.data(), sizeof(EnsRun) * nruns, hipMemcpyHostToDevice) ==
                hipSuccess &&
            hipMemcpy(E->ditems, items.data(), sizeof(int4) * items.size(),
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(E->dbig, order.data(), sizeof(int) * nruns, hipMemcpyHostToDevice) ==
                hipSuccess;
  return ok ? ens_tune_red(E, order) : CHX_EHIP;
}

int ch_ensemble_create(int nruns, const chx_ch_params* prm, chx_ens* out) {
  if (!out || !prm || nruns < 1) return CHX_EINVAL;
  *out = nullptr;
  chx_ens_s* E = new (std::nothrow) chx_ens_s();
  if (!E) return CHX_ENOMEM;
  E->nruns = nruns;
  E->prm.assign(prm, prm + nruns);
  int nref = 0;
  for (int r = 0; r < nruns; ++r) nref += prm[r].dtype == CHX_F32_REFINED;
  if (nref > 0) {
    if (nref != nruns) {  // one precision per ensemble
      delete E;
      return CHX_EINVAL;
    }
    const int rc = ens_create_refined(E);
    if (rc != CHX_OK) {
      delete E;
      return rc;
    }
    *out = E;
    return CHX_OK;
  }
  std::vector<int> cls_of(nruns, -1);
  std::vector<chx_ch_params> reps;
  for (int r = 0; r < nruns; ++r) {
    const chx_ch_params& q = prm[r];
    if (q.dtype != CHX_F64 || q.scheme != CHX_SCHEME_P1 || q.nx % 64 != 0 ||
        q.ny % kChunk != 0 || q.nx / kChunk > 256 ||
        !(q.lx > 0) || !(q.ly > 0) || !(q.dt > 0) || !(q.D >= 0) || !(q.gamma >= 0)) {
      delete E;
      return CHX_EINVAL;
    }
    for (size_t c = 0; c < reps.size(); ++c)
      if (same_grid(reps[c], q)) cls_of[r] = (int)c;
    if (cls_of[r] < 0) {
      if ((int)reps.size() == kEnsMaxClasses) {
        delete E;
        return CHX_EINVAL;
      }
      cls_of[r] = (int)reps.size();
      reps.push_back(q);
    }
  }
  size_t lds_max = 0;
  for (const auto& q : reps) {
    const double dx = q.lx / q.nx, dy = q.ly / q.ny;
    const double sx = q.D * q.gamma * q.dt / (dx * dx * dx * dx);
    const double sy = q.D * q.gamma * q.dt / (dy * dy * dy * dy);
    const double cxs[5] = {sx, -4 * sx, 1 + 6 * sx, -4 * sx, sx};
    const double cys[5] = {sy, -4 * sy, 1 + 6 * sy, -4 * sy, sy};
    BandPlan *a = nullptr, *b = nullptr;
    int rc = make_plan(2, q.nx, cxs, 1, &a);
    if (rc == CHX_OK) rc = make_plan(2, q.ny, cys, 1, &b);
    if (rc == CHX_OK && (!a->has_chunk || !b->has_chunk)) rc = CHX_EINVAL;
    E->px.push_back(a);
    E->py.push_back(b);
    if (rc != CHX_OK) {
      delete E;
      return rc;
    }
    EnsClass ec;
    ec.px = a->dchunk;
    ec.py = b->dchunk;
    ec.K = make_coef(q);
    E->classes.push_back(ec);
    lds_max = std::max(lds_max, ens_reduced_lds_bytes(b->chunk.dcount));
  }
  if (lds_max > 64 * 1024) {
    delete E;
    return CHX_EINVAL;
  }
  E->red_lds = lds_max;
  // runs that fit one workgroup's LDS take the single-workgroup path (the
  // rule ch_create applies, so a run advances identically alone or here);
  // the others get work items, larger runs first in every work list
  const size_t max_lds = device_max_lds();
  std::vector<int> small_list, big_list, order;
  for (int r = 0; r < nruns; ++r) {
    if (ch_small_fits(prm[r].nx, prm[r].ny, max_lds)) {
      small_list.push_back(r);
      E->small_threads = std::max(E->small_threads, prm[r].nx * prm[r].ny / kChunk);
      E->small_lds = std::max(E->small_lds, ch_small_lds_bytes(prm[r].nx, prm[r].ny));
    } else {
      big_list.push_back(r);
      order.push_back(r);
    }
  }
  E->nsmall = (int)small_list.size();
  E->nbig = (int)big_list.size();
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long)prm[a].nx * prm[a].ny > (long)prm[b].nx * prm[b].ny;
  });
  size_t off = 0;
  E->runs.resize(nruns);
  std::vector<char> is_small(nruns, 0);
  for (int r : small_list) is_small[r] = 1;
  for (int r = 0; r < nruns; ++r) {
    const chx_ch_params& q = prm[r];
    EnsRun& R = E->runs[r];
    R.c = nullptr;
    R.ldc = q.nx;
    R.nx = q.nx;
    R.ny = q.ny;
    R.cls = cls_of[r];
    R.ncb = ((q.nx >> 6) + 3) / 4;
    R.Sc = q.ny / kChunk;
    R.ncolblocks = (long)R.ncb * R.Sc;
    R.nscale = R.ninv_dx = R.ninv_dy = 0.0;
    R.nseed = 0;
    E->max_points = std::max(E->max_points, (long)q.nx * q.ny);
    if (is_small[r]) {  // no workspace: the field stays in LDS
      R.off_b0 = R.off_b1 = R.off_rho = R.off_part = 0;
      continue;
    }
    const size_t field = align256((size_t)q.nx * q.ny * sizeof(double));
    R.off_b0 = off; off += field;
    R.off_b1 = off; off += field;
    R.off_rho = off; off += align256((size_t)R.Sc * 4 * q.nx * sizeof(double));
    R.off_part = off;
    off += align256((size_t)R.ncolblocks * 2 * sizeof(double));
  }
  E->ws_total = std::max(off, (size_t)256);
  std::vector<int4> items;
  auto add = [&](int r, int a, int b) { items.push_back(make_int4(r, a, b, 0)); };
  E->o_col = (long)items.size();
  for (int r : order)
    for (int kc = 0; kc < E->runs[r].Sc; ++kc)
      for (int cb = 0; cb < E->runs[r].ncb; ++cb) add(r, cb, kc);
  E->n_col = (int)(items.size() - E->o_col);
  E->o_row = (long)items.size();
  E->rows_half = true;
  for (int r : order) {
    const int S = E->runs[r].nx / kChunk, R = 256 / S;
    const int ng = (E->runs[r].ny + R - 1) / R;
    for (int g = 0; g < ng; ++g) add(r, g, 0);
    if (256 % S != 0 || E->runs[r].ny % R != 0) E->rows_half = false;
  }
  E->n_row = (int)(items.size() - E->o_row);
  // the separator items last: their count depends on the tile shape that
  // creation times (room for the shape with the most blocks)
  E->o_red = (long)items.size();
  size_t max_red = 0;
  for (int sh = 0; sh < kNumEnsRedShapes; ++sh)
    max_red = std::max(max_red, ens_red_items(E, order, sh).size());
  {
    const auto red = ens_red_items(E, order, 0);
    items.insert(items.end(), red.begin(), red.end());
    E->n_red = (int)red.size();
  }

  for (size_t c = 0; c < E->classes.size(); ++c) E->hcls.c[c] = E->classes[c];
  const size_t b_runs = align256(sizeof(EnsRun) * nruns);
  const size_t b_items =
      align256(sizeof(int4) * std::max<size_t>(E->o_red + max_red, 1));
  const size_t b_lists = align256(sizeof(int) * nruns);
  if (hipMalloc(&E->dmem, b_runs + b_items + 2 * b_lists) != hipSuccess) {
    E->dmem = nullptr;
    delete E;
    return CHX_EHIP;
  }
  auto* base = static_cast<unsigned char*>(E->dmem);
  E->druns = reinterpret_cast<EnsRun*>(base);
  E->ditems = reinterpret_cast<int4*>(base + b_runs);
  E->dsmall = reinterpret_cast<int*>(base + b_runs + b_items);
  E->dbig = reinterpret_cast<int*>(base + b_runs + b_items + b_lists);
  bool ok = hipMemcpy(E->druns, E->runs.data(), sizeof(EnsRun) * nruns, hipMemcpyHostToDevice) ==
            hipSuccess;
  if (ok && !items.empty())
    ok = hipMemcpy(E->ditems, items.data(), sizeof(int4) * items.size(),
                   hipMemcpyHostToDevice) == hipSuccess;
  if (ok && E->nsmall)
    ok = hipMemcpy(E->dsmall, small_list.data(), sizeof(int) * E->nsmall,
                   hipMemcpyHostToDevice) == hipSuccess;
  if (ok && E->nbig)
    ok = hipMemcpy(E->dbig, big_list.data(), sizeof(int) * E->nbig, hipMemcpyHostToDevice) ==
         hipSuccess;
  if (ok && E->nsmall && E->nbig)
    ok = hipStreamCreateWithFlags(&E->side, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&E->ev_fork, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&E->ev_join, hipEventDisableTiming) == hipSuccess;
  E->red_order = order;
  if (ok && E->nbig > 0) ok = ens_tune_red(E, order) == CHX_OK;
  if (!ok) {
    delete E;
    return CHX_EHIP;
  }
  *out = E;
  return CHX_OK;
}

int ch_ensemble_get_tuning(chx_ens e, int what, int* value) {
  if (!e || !value || what != CHX_TUNE_REDUCED_SHAPE) return CHX_EINVAL;
  *value = e->red_shape;
  return CHX_OK;
}

static void ens_drop_graph(chx_ens E);

int ch_ensemble_set_tuning(chx_ens e, int what, int value) {
  if (!e || what != CHX_TUNE_REDUCED_SHAPE) return CHX_EINVAL;
  if (value < 0 || value >= kNumEnsRedShapes) return CHX_EINVAL;
  if (e->nbig == 0) return value == 0 ? CHX_OK : CHX_EINVAL;
  // queued work may still read the work items
  if (hipDeviceSynchronize() != hipSuccess) return CHX_EHIP;
  ens_drop_graph(e);  // a captured call holds the old items
  return ens_set_red_shape(e, value);
}

int ch_ensemble_destroy(chx_ens e) {
  delete e;
  return CHX_OK;
}

size_t ch_ensemble_ws_bytes(chx_ens e) { return e ? e->ws_total : 0; }

static int ens_step_launch(chx_ens E, int nsteps, double* diag_out, void* ws, unsigned char* w,
                           int use_graph, hipStream_t st);

int ch_ensemble_step(chx_ens E, double* const* c_runs, const long* ld_runs, int nsteps,
                     double* diag_out, void* ws, size_t ws_bytes, int use_graph, chx_stream s) {
  if (!E || !c_runs || nsteps < 1) return CHX_EINVAL;
  if (!ws || ws_bytes < E->ws_total) return CHX_ENOMEM;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return CHX_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(s);
  bool changed = false;
  for (int r = 0; r < E->nruns; ++r) {
    if (!c_runs[r]) return CHX_EINVAL;
    const long ld = ld_runs ? ld_runs[r] : E->runs[r].nx;
    if (ld < E->runs[r].nx) return CHX_EINVAL;
    if (E->runs[r].c != c_runs[r] || E->runs[r].ldc != ld) {
      E->runs[r].c = c_runs[r];
      E->runs[r].ldc = ld;
      changed = true;
    }
  }
  if (changed) {  // work already queued may still read the table
    if (hipStreamSynchronize(st) != hipSuccess) return CHX_EHIP;
    if (hipMemcpy(E->druns, E->runs.data(), sizeof(EnsRun) * E->nruns, hipMemcpyHostToDevice) !=
        hipSuccess)
      return CHX_EHIP;
  }
  auto* w = static_cast<unsigned char*>(ws);
  const int rc_step = ens_step_launch(E, nsteps, diag_out, ws, w, use_graph, st);
  if (rc_step == CHX_OK && E->noise) E->noise_step += (unsigned long long)nsteps;
  return rc_step;
}

// The launches of one ensemble call, eager or from the cached graph.
static int ens_step_launch(chx_ens E, int nsteps, double* diag_out, void* ws, unsigned char* w,
                           int use_graph, hipStream_t st) {
  if (!use_graph) return ens_launch_all(E, nsteps, diag_out, w, st);
  if (!E->gexec || E->g_nsteps != nsteps || E->g_diag != diag_out || E->g_ws != ws) {
    if (E->gexec) (void)hipGraphExecDestroy(E->gexec);
    if (E->graph) (void)hipGraphDestroy(E->graph);
    E->gexec = nullptr;
    E->graph = nullptr;
    if (!E->cap && hipStreamCreateWithFlags(&E->cap, hipStreamNonBlocking) != hipSuccess) {
      E->cap = nullptr;
      return CHX_EHIP;
    }
    if (hipStreamBeginCapture(E->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return CHX_EHIP;
    int rc = ens_launch_all(E, nsteps, diag_out, w, E->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(E->cap, &g);
    if (rc != CHX_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != CHX_OK ? rc : CHX_EHIP;
    }
    if (hipGraphInstantiate(&E->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      E->gexec = nullptr;
      return CHX_EHIP;
    }
    E->graph = g;
    E->g_nsteps = nsteps;
    E->g_diag = diag_out;
    E->g_ws = ws;
  }
  return hipGraphLaunch(E->gexec, st) == hipSuccess ? CHX_OK : CHX_EHIP;
}

static void ens_drop_graph(chx_ens E) {
  if (E->gexec) (void)hipGraphExecDestroy(E->gexec);
  if (E->graph) (void)hipGraphDestroy(E->graph);
  E->gexec = nullptr;
  E->graph = nullptr;
}

int ch_ensemble_set_noise(chx_ens E, double sigma, const unsigned long long* seeds,
                          unsigned long long step0) {
  if (!E || !(sigma >= 0) || !std::isfinite(sigma)) return CHX_EINVAL;
  if (E->refined) return sigma > 0 ? CHX_EINVAL : CHX_OK;  // FP64 ensembles only
  if (sigma > 0 && !seeds) return CHX_EINVAL;
  // queued work may still read the run table or the counter
  if (hipDeviceSynchronize() != hipSuccess) return CHX_EHIP;
  if (sigma > 0) {
    if (!E->dnoise && hipMalloc(&E->dnoise, sizeof(unsigned long long)) != hipSuccess) {
      E->dnoise = nullptr;
      return CHX_ENOMEM;
    }
    for (int r = 0; r < E->nruns; ++r) {
      EnsRun& R = E->runs[r];
      const chx_ch_params& q = E->prm[r];
      const double dx = q.lx / q.nx, dy = q.ly / q.ny;
      R.nscale = q.dt * std::sqrt(sigma / (dx * dy * q.dt));
      R.ninv_dx = 1.0 / dx;
      R.ninv_dy = 1.0 / dy;
      R.nseed = chx_sm_mix(seeds[r]);
    }
    if (hipMemcpy(E->dnoise, &step0, sizeof(step0), hipMemcpyHostToDevice) != hipSuccess)
      return CHX_EHIP;
  }
  if (hipMemcpy(E->druns, E->runs.data(), sizeof(EnsRun) * E->nruns, hipMemcpyHostToDevice) !=
      hipSuccess)
    return CHX_EHIP;
  E->noise = sigma > 0;
  E->noise_step = step0;
  ens_drop_graph(E);  // the launch sequence changes with the forcing
  return CHX_OK;
}

int ch_ensemble_get_noise_step(chx_ens E, unsigned long long* step) {
  if (!E || !step) return CHX_EINVAL;
  *step = E->noise_step;
  return CHX_OK;
}

// Per-run coarsening measures of an ensemble (the s(t) and k1(t) of each
// run, Ch.3 "Numerical Results", for the Ch.7 statistics).
static int ens_fields(chx_ens E, double* const* c_runs, const long* ld_runs,
                      std::vector<const double*>& c, std::vector<long>& ld) {
  c.resize(E->nruns);
  ld.resize(E->nruns);
  for (int r = 0; r < E->nruns; ++r) {
    c[r] = c_runs[r];
    ld[r] = ld_runs ? ld_runs[r] : E->prm[r].nx;
    if (!c[r] || ld[r] < E->prm[r].nx) return CHX_EINVAL;
  }
  return CHX_OK;
}

int ch_ensemble_moments(chx_ens E, double* const* c_runs, const long* ld_runs, double* out,
                        chx_stream s) {
  if (!E || !c_runs || !out) return CHX_EINVAL;
  std::vector<const double*> c;
  std::vector<long> ld;
  int rc = ens_fields(E, c_runs, ld_runs, c, ld);
  if (rc != CHX_OK) return rc;
  for (int r = 0; r < E->nruns; ++r)
    if ((E->prm[r].nx & 1) || (E->prm[r].ny & 1)) return CHX_EINVAL;
  if (!E->mom_mem) {
    long off = 2L * E->nruns;  // the per-run outputs first
    E->mom_off.resize(E->nruns);
    for (int r = 0; r < E->nruns; ++r) {
      E->mom_off[r] = off;
      off += 2L * ((E->prm[r].nx + 63) / 64) * ((E->prm[r].ny + 15) / 16);
    }
    if (hipMalloc(&E->mom_mem, (size_t)off * sizeof(double)) != hipSuccess) {
      E->mom_mem = nullptr;
      return CHX_ENOMEM;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(s);
  double* base = static_cast<double*>(E->mom_mem);
  hipError_t e = hipSuccess;
  for (int r = 0; r < E->nruns && e == hipSuccess; ++r)
    e = launch_ch_simpson(c[r], ld[r], E->prm[r].nx, E->prm[r].ny, base + E->mom_off[r],
                          base + 2 * r, st);
  std::vector<double> host(2 * E->nruns);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), base, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return CHX_EHIP;
  bool finite = true;
  for (int r = 0; r < E->nruns; ++r) {
    out[3 * r] = host[2 * r];
    out[3 * r + 1] = host[2 * r + 1];
    out[3 * r + 2] = 1.0 / (1.0 - host[2 * r + 1]);
    finite = finite && std::isfinite(host[2 * r]) && std::isfinite(host[2 * r + 1]);
  }
  return finite ? CHX_OK : CHX_ENONFINITE;
}

// Undo a partial set-up of the transforms (a later call starts afresh).
static void ens_k1_reset(chx_ens E) {
  for (auto& g : E->k1_groups)
    if (g.plan) (void)hipfftDestroy(g.plan);
  E->k1_groups.clear();
}

int ch_ensemble_k1(chx_ens E, double* const* c_runs, const long* ld_runs, double* k1,
                   chx_stream s) {
  if (!E || !c_runs || !k1) return CHX_EINVAL;
  std::vector<const double*> c;
  std::vector<long> ld;
  int rc = ens_fields(E, c_runs, ld_runs, c, ld);
  if (rc != CHX_OK) return rc;
  if (!E->k1_mem) {
    // runs grouped by grid size; one batched transform per group, the
    // groups taking turns in one real and one spectrum buffer
    for (int r = 0; r < E->nruns; ++r) {
      const int nx = E->prm[r].nx, ny = E->prm[r].ny;
      size_t g = 0;
      while (g < E->k1_groups.size() && !(E->k1_groups[g].nx == nx && E->k1_groups[g].ny == ny))
        ++g;
      if (g == E->k1_groups.size()) E->k1_groups.push_back({nx, ny, {}, 0});
      E->k1_groups[g].runs.push_back(r);
    }
    size_t real_max = 0, spec_max = 0;
    for (auto& g : E->k1_groups) {
      const size_t nb = g.runs.size();
      real_max = std::max(real_max, nb * g.nx * g.ny);
      spec_max = std::max(spec_max, nb * (g.nx / 2 + 1) * g.ny);
      int dims[2] = {g.ny, g.nx};
      if (hipfftPlanMany(&g.plan, 2, dims, nullptr, 1, g.nx * g.ny, nullptr, 1,
                         (g.nx / 2 + 1) * g.ny, HIPFFT_D2Z, (int)nb) != HIPFFT_SUCCESS) {
        g.plan = 0;
        ens_k1_reset(E);
        return CHX_EHIP;
      }
    }
    E->k1_real_off = 0;
    E->k1_spec_off = align256(real_max * sizeof(double));
    E->k1_part_off = E->k1_spec_off + align256(spec_max * sizeof(double2));
    long off = 2L * E->nruns;  // per-run outputs first
    E->k1_poff.resize(E->nruns);
    for (int r = 0; r < E->nruns; ++r) {
      E->k1_poff[r] = off;
      off += 2 * ch_k1_blocks(E->prm[r].nx, E->prm[r].ny);
    }
    if (hipMalloc(&E->k1_mem, E->k1_part_off + (size_t)off * sizeof(double)) != hipSuccess) {
      E->k1_mem = nullptr;
      ens_k1_reset(E);
      return CHX_ENOMEM;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(s);
  auto* base = static_cast<unsigned char*>(E->k1_mem);
  double* real = reinterpret_cast<double*>(base + E->k1_real_off);
  auto* spec = reinterpret_cast<double2*>(base + E->k1_spec_off);
  double* parts = reinterpret_cast<double*>(base + E->k1_part_off);
  hipError_t e = hipSuccess;
  for (auto& g : E->k1_groups) {
    const long pts = (long)g.nx * g.ny, sp = (long)(g.nx / 2 + 1) * g.ny;
    for (size_t j = 0; j < g.runs.size() && e == hipSuccess; ++j) {
      const int r = g.runs[j];
      e = hipMemcpy2DAsync(real + j * pts, g.nx * sizeof(double), c[r], ld[r] * sizeof(double),
                           g.nx * sizeof(double), g.ny, hipMemcpyDeviceToDevice, st);
    }
    if (e != hipSuccess) break;
    if (hipfftSetStream(g.plan, st) != HIPFFT_SUCCESS ||
        hipfftExecD2Z(g.plan, real, reinterpret_cast<hipfftDoubleComplex*>(spec)) !=
            HIPFFT_SUCCESS)
      return CHX_EHIP;
    for (size_t j = 0; j < g.runs.size() && e == hipSuccess; ++j) {
      const int r = g.runs[j];
      e = launch_ch_k1(spec + j * sp, g.nx, g.ny, E->prm[r].lx, E->prm[r].ly,
                       parts + E->k1_poff[r], parts + 2 * r, st);
    }
  }
  std::vector<double> host(2 * E->nruns);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data(), parts, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return CHX_EHIP;
  bool finite = true;
  for (int r = 0; r < E->nruns; ++r) {
    k1[r] = host[2 * r] / host[2 * r + 1];
    finite = finite && std::isfinite(k1[r]);
  }
  return finite ? CHX_OK : CHX_ENONFINITE;
}

// Host-side plan inspection (no device work): the factorisation tables that
// penta_factor / tri_factor upload, for checking the host logic on a CPU.
int chx_host_chunk_tables(int P, const double* coef, int n, int m, double* rec, int rec_cap,
                          double* blocks, int blocks_cap, int* info) {
  if ((P != 1 && P != 2) || !coef || !info) return CHX_EINVAL;
  Band band;
  band.P = P;
  band.periodic = true;
  for (int k = 0; k < 2 * P + 1; ++k) band.coef[k] = coef[k];
  ChunkTables t;
  int rc = build_chunk(band, n, m, &t);
  if (rc) return rc;
  info[0] = t.mi;
  info[1] = t.S;
  info[2] = t.dlo;
  info[3] = t.dcount;
  if (rec && rec_cap >= (int)t.rec.size()) std::memcpy(rec, t.rec.data(), t.rec.size() * 8);
  if (blocks && blocks_cap >= (int)t.blocks.size())
    std::memcpy(blocks, t.blocks.data(), t.blocks.size() * 8);
  return CHX_OK;
}

int chx_host_whole_tables(int P, const double* coef, int n, int periodic, double* rec,
                          int rec_cap, double* minv, int* mi_out) {
  if ((P != 1 && P != 2) || !coef || !mi_out) return CHX_EINVAL;
  Band band;
  band.P = P;
  band.periodic = periodic != 0;
  for (int k = 0; k < 2 * P + 1; ++k) band.coef[k] = coef[k];
  WholeTables t;
  int rc = build_whole(band, n, &t);
  if (rc) return rc;
  *mi_out = t.mi;
  if (rec && rec_cap >= (int)t.rec.size()) std::memcpy(rec, t.rec.data(), t.rec.size() * 8);
  if (minv) std::memcpy(minv, t.minv, sizeof(t.minv));
  return CHX_OK;
}

}  // extern "C"
