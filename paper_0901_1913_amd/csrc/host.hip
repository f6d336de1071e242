// C ABI host layer: argument checks, plan geometry, device tables, workspace
// layout and the launch sequence of the search and its adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fchi2.h"
#include "fchi2_internal.h"
#include "launch.h"
#include "fft_splits.h"

using namespace fchi2;

namespace {

thread_local std::string g_err;

fchi2_status_t fail(fchi2_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

fchi2_status_t hip_fail(hipError_t e, const char* what) {
  return fail(FCHI2_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr)                                      \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return hip_fail(e_, #expr);     \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Tiles of the table the fused first pass reads (2^kFusedTbLog cells, at
// least the kernel width + 3 for every width up to 16).
constexpr int kFusedTbLog = 5;

// Most grid periods a plan's tile tables cover (curves whose harmonic phases
// wrap further are flagged FCHI2_CURVE_WRAP).
constexpr int kMaxLaps = 8;

// Workspace of fchi2_search_noalloc: a file-scope device array of
// FCHI2_NOALLOC_SCRATCH_BYTES that every device running the library holds
// until the process ends.  Host code never uses its name as an address: the
// device address is looked up once per device (hipGetSymbolAddress, with that
// device current) and kept in scratch_ptr.
__device__ __align__(256) unsigned char scratch[FCHI2_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on the current device (looked up on first use).
hipError_t scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
  int r = 0;
  while (((int64_t)1 << r) < v) ++r;
  return r;
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

struct fchi2_plan_s {
  fchi2_plan_desc_t desc;
  std::vector<int64_t> offsets;
  bool fp64 = false;
  size_t elem = 8;        // bytes per complex grid element
  size_t out_elem = 4;    // bytes per Delta chi2 value
  Geom g{};
  FftPlan fp{};
  int log_tile = 10;
  // Spreading fused into the first FFT pass (no spread grid in memory).
  int fused = 0;
  // Persistent batched search: one launch, curves claimed from a device work
  // queue by n_slots workgroups, each with a slot of the workspace (its
  // grids, spectra and tile table) at off_gA + slot * slot_bytes.
  int persist = 0;
  // Curves per launch of the last FFT pass and the solve (0: the whole wave).
  int solve_sub = 0;
  // Overlap of the next wave's spreading with this wave's FFT passes and
  // solve: a second stream (default priority) and the events that order the
  // two; used for waves of at most wave_max / 2 curves, whose two spread
  // grids and tile tables fit in the one-wave buffers.
  hipStream_t side = nullptr;
  hipEvent_t ev_start = nullptr, ev_spread[2] = {nullptr, nullptr},
             ev_first[2] = {nullptr, nullptr};
  int n_slots = 0;
  int n_slots_device = 0;  // workgroups resident on the whole device
  size_t slot_bytes = 0, slot_gB = 0, slot_zc = 0, slot_tb = 0;
  size_t off_queue = 0;
  double eps_piv = 0.0;
  int wave = 1;
  int wave_max = 1;        // the workspace is sized for this many curves
  int64_t max_n = 0;
  int64_t n_total = 0;
  // plan-owned device tables
  int64_t* d_off = nullptr;
  void* d_tw_stage = nullptr;
  void* d_tw_small = nullptr;
  void* d_D = nullptr;
  double* d_gl = nullptr;
  // workspace layout (byte offsets)
  int mom_bpc = 1;
  size_t off_part = 0;
  size_t off_tb = 0;
  size_t off_mom = 0, off_gA = 0, off_gB = 0, off_zc = 0, off_gq = 0, off_gp = 0, off_dw = 0;
  size_t ws_bytes = 0;
  int blocks_per_curve = 0;
  // graph replay
  hipGraphExec_t gexec = nullptr;
  const void* gkey[8] = {nullptr};
  size_t gkey_ws = 0;
  // backward needs a search on this workspace first
  const void* last_ws = nullptr;
  // searches enqueued on the plan so far (the state backward reads is the last one's)
  uint64_t gen = 0;
  // measurement: event pairs around each launch while profiling is on
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_stage;
  double prof_ms[FCHI2_PROF_STAGES] = {0};
  int64_t prof_n[FCHI2_PROF_STAGES] = {0};
};

namespace {

void apply_fft_plan(fchi2_plan_s* pl, const FftPlan& f) {
  pl->fp = f;
  const int64_t S_first = (f.np == 1) ? 1 : (pl->g.L >> f.logn[f.np]);
  const int64_t tile = (int64_t)1 << pl->log_tile;
  pl->g.chunk = (int)(S_first > tile ? S_first : tile);
}

// Record an event on st if profiling (begin of a launch of `stage` when
// stage >= 0, its end when stage < 0).
hipError_t prof_mark(fchi2_plan_s* pl, int stage, hipStream_t st) {
  if (!pl->prof) return hipSuccess;
  if (pl->ev_used == pl->ev_pool.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pl->ev_pool.push_back(e);
  }
  hipEvent_t e = pl->ev_pool[pl->ev_used++];
  if (stage >= 0) pl->ev_stage.push_back(stage);
  return hipEventRecord(e, st);
}

#define PROF_BEGIN(stage)                                              \
  do {                                                                 \
    hipError_t pe_ = prof_mark(pl, (stage), st);                       \
    if (pe_ != hipSuccess) return hip_fail(pe_, "profiling event");    \
  } while (0)
#define PROF_END()                                                     \
  do {                                                                 \
    hipError_t pe_ = prof_mark(pl, -1, st);                            \
    if (pe_ != hipSuccess) return hip_fail(pe_, "profiling event");    \
  } while (0)

// fused_pts: the forward first pass spreads these points (t, x, sigma) in
// its tiles instead of reading gA (null: read the spread grid), finding them
// through the tile table fused_tb (tiles of 2^kFusedTbLog cells).
// after_last (forward, may be null): called with (offset, count) after the
// last pass has written the spectra of curves [curve0 + offset, + count);
// with 0 < sub < nw the last pass runs in sub-waves of sub curves, each
// followed by its call, so the spectra a call reads were just written.
// after_first (may be null): called once the first pass (the last reader of
// gA) is enqueued.
using AfterLast = std::function<fchi2_status_t(int, int)>;
using AfterFirst = std::function<fchi2_status_t()>;
fchi2_status_t enqueue_fft(fchi2_plan_s* pl, int mode, void* gA, void* gB, void* zc,
                           const Moments* mom, int curve0, int nw, hipStream_t st,
                           const Geom* geom = nullptr,
                           const double* const* fused_pts = nullptr,
                           const int32_t* fused_tb = nullptr, int sub = 0,
                           const AfterLast* after_last = nullptr,
                           const AfterFirst* after_first = nullptr) {
  const Geom& g = geom ? *geom : pl->g;
  const FftPlan& fp = pl->fp;
  FftPassArgs a{};
  a.mode = mode;
  a.np = fp.np;
  for (int q = 0; q <= kMaxPasses; ++q) a.logn[q] = fp.logn[q];
  a.logL = fp.logL;
  a.curve0 = curve0;
  a.zc = zc;
  a.grid_out = gA;
  if (fp.np == 1) {
    a.kind = PASS_SINGLE;
    a.q = 1;
    PROF_BEGIN(mode == MODE_FWD ? FCHI2_PROF_FFT_LAST : FCHI2_PROF_BWD_FFT);
    hipError_t e = launch_fft_pass(pl->fp64, a, fp.logL, 0, gA, gA, mom, g, pl->d_tw_stage,
                                   pl->d_tw_small, nw, 1, st);
    if (e != hipSuccess) return hip_fail(e, "fft single pass");
    PROF_END();
    if (after_first) {
      fchi2_status_t r = (*after_first)();
      if (r != FCHI2_OK) return r;
    }
    return after_last ? (*after_last)(0, nw) : FCHI2_OK;
  }
  for (int q = fp.np; q >= 1; --q) {
    a.q = q;
    a.kind = (q == fp.np) ? PASS_FIRST : (q == 1 ? PASS_LAST : PASS_MID);
    const bool fuse = fused_pts && a.kind == PASS_FIRST && mode == MODE_FWD;
    a.fused = fuse ? 1 : 0;
    a.t = fuse ? fused_pts[0] : nullptr;
    a.x = fuse ? fused_pts[1] : nullptr;
    a.sigma = fuse ? fused_pts[2] : nullptr;
    a.tb = fuse ? fused_tb : nullptr;
    a.tb_log = kFusedTbLog;
    a.ntb = (int)((g.L >> kFusedTbLog) * g.laps) + 2;
    const int logn = fp.logn[q];
    const int logt = fp.le[q] - logn;
    const int64_t ncols = g.L >> logn;
    const void* in = (q == fp.np) ? gA : gB;
    void* out = gB;
    const int stage = mode == MODE_BWD ? FCHI2_PROF_BWD_FFT
                      : a.kind == PASS_FIRST ? FCHI2_PROF_FFT_FIRST
                      : a.kind == PASS_MID   ? FCHI2_PROF_FFT_MID
                                             : FCHI2_PROF_FFT_LAST;
    const bool split = q == 1 && mode == MODE_FWD && sub > 0 && sub < nw;
    const int step = split ? sub : nw;
    const size_t grid_curve = (size_t)g.P * (size_t)g.L * pl->elem;
    const size_t zc_curve = (size_t)g.P * 2 * (size_t)g.n_freq * pl->elem;
    for (int off = 0; off < nw; off += step) {
      const int n = (nw - off) < step ? (nw - off) : step;
      FftPassArgs b = a;
      b.curve0 = curve0 + off;
      if (zc) b.zc = (char*)zc + (size_t)off * zc_curve;
      PROF_BEGIN(stage);
      hipError_t e = launch_fft_pass(pl->fp64, b, logn, logt,
                                     (const char*)in + (size_t)off * grid_curve,
                                     (char*)out + (size_t)off * grid_curve, mom, g,
                                     pl->d_tw_stage, pl->d_tw_small, n, ncols, st);
      if (e != hipSuccess) return hip_fail(e, "fft pass");
      PROF_END();
      if (q == 1 && after_last) {
        fchi2_status_t r = (*after_last)(off, n);
        if (r != FCHI2_OK) return r;
      }
    }
    if (q == fp.np && after_first) {
      fchi2_status_t r = (*after_first)();
      if (r != FCHI2_OK) return r;
    }
  }
  return FCHI2_OK;
}

// Whether the forward chain spreads inside the first FFT pass.
bool use_fused(const fchi2_plan_s* pl) { return pl->fused && pl->fp.np >= 2 && !pl->g.band; }

// Whether the persistent kernel can run split f with spreading tiles of
// 2^tile cells: mixed precision, H <= 8, no band, no kept spectra, grids of
// at most 2^20 cells (one workgroup transforms a whole curve), every pass a
// tile of 2^12 elements of 2^5..2^9 rows, spreading tiles of 2^10 or 2^11.
bool persist_ok(const fchi2_plan_s* pl, const FftPlan& f, int tile) {
  if (pl->n_slots < 1 || pl->fp64 || pl->g.band || pl->g.H > kHMax) return false;
  if (pl->g.L > ((int64_t)1 << 20)) return false;
  if (pl->desc.flags & (FCHI2_KEEP_FOR_BACKWARD | FCHI2_WIDE_SOLVE)) return false;
  if (f.np < 2 || (tile != 10 && tile != 11)) return false;
  for (int q = 1; q <= f.np; ++q)
    if (f.le[q] != 12 || f.logn[q] < 5 || f.logn[q] > 9) return false;
  return true;
}
bool use_persist(const fchi2_plan_s* pl) {
  return pl->persist && persist_ok(pl, pl->fp, pl->log_tile);
}
// Whether the autotuner times the persistent schedule: only for batches that
// fill every resident workgroup at the start.  One workgroup runs a whole
// curve, so a few curves would leave most of the device idle;
// FCHI2_PERSISTENT still forces it.
bool persist_worth_timing(const fchi2_plan_s* pl) {
  return pl->n_slots_device > 0 && pl->desc.n_curves >= pl->n_slots_device;
}

// The persistent search of curves [cbeg, cend) (moments already computed).
fchi2_status_t enqueue_persistent(fchi2_plan_s* pl, int cbeg, int cend, const double* t,
                                  const double* x, const double* sigma, char* ws, void* dchi2,
                                  uint8_t* flags, hipStream_t st) {
  PersistArgs a{};
  a.t = t;
  a.x = x;
  a.sigma = sigma;
  a.mom = (const Moments*)(ws + pl->off_mom);
  a.g = pl->g;
  const FftPlan& fp = pl->fp;
  for (int q = 1; q <= fp.np; ++q) {
    FftPassArgs& f = a.fa[q];
    f.kind = (q == fp.np) ? PASS_FIRST : (q == 1 ? PASS_LAST : PASS_MID);
    f.mode = MODE_FWD;
    f.np = fp.np;
    f.q = q;
    for (int d = 0; d <= kMaxPasses; ++d) f.logn[d] = fp.logn[d];
    f.logL = fp.logL;
    f.curve0 = 0;
  }
  a.fa[0] = a.fa[1];
  a.tws = (const cplx<double>*)pl->d_tw_stage;
  a.twsm = (const cplx<double>*)pl->d_tw_small;
  a.D = (const cplx<double>*)pl->d_D;
  a.curve_base = cbeg;
  a.n_curves = cend - cbeg;
  a.log_tile = pl->log_tile;
  a.ntb = (int)((pl->g.L >> pl->log_tile) * pl->g.laps) + 2;
  a.slots = ws + pl->off_gA;
  a.slot_bytes = pl->slot_bytes;
  a.off_gB = pl->slot_gB;
  a.off_zc = pl->slot_zc;
  a.off_tb = pl->slot_tb;
  a.next = (int*)(ws + pl->off_queue);
  a.eps = pl->eps_piv;
  a.out = (float*)dchi2;
  a.flags = flags;
  const int n = cend - cbeg;
  PROF_BEGIN(FCHI2_PROF_PERSISTENT);
  hipError_t e = launch_persistent(a, n < pl->n_slots ? n : pl->n_slots, st);
  if (e != hipSuccess) return hip_fail(e, "persistent search");
  PROF_END();
  return FCHI2_OK;
}

// Whether a search of n curves runs the overlapped wave schedule: staged
// (not fused, not persistent), at least two waves, and waves of at most half
// the buffers' capacity (two spread grids and tables fit).
bool use_overlap(const fchi2_plan_s* pl, int n) {
  return pl->side && !use_fused(pl) && !pl->g.band && n > pl->wave &&
         2 * pl->wave <= pl->wave_max;
}

// The forward chain with the spreading of wave i + 1 on the side stream while
// the main stream runs wave i's FFT passes and what follows them (`tail`,
// made per wave from (c0, nw, spectra): the solve, or the solve with the
// candidate selection).  Wave i spreads into grid A buffer i % 2 (halves of
// the grid A region) with table i % 2 (halves of the table region); the side
// stream waits for the first pass that last read that buffer (wave i - 2),
// the main stream for wave i's spreading.  Every kernel is the one-stream
// search's on the same curves, so the results are identical bit for bit.
// Every piece of side-stream work is waited on by the main stream before the
// call returns to it, so graph capture joins.
using WaveTail = std::function<AfterLast(int, int, void*)>;
fchi2_status_t enqueue_waves_overlap(fchi2_plan_s* pl, int cbeg, int cend, const double* t,
                                     const double* x, const double* sigma, char* ws,
                                     hipStream_t st, int sub, const WaveTail& tail) {
  Moments* mom = (Moments*)(ws + pl->off_mom);
  const bool keep = pl->desc.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)pl->g.P * 2 * pl->g.n_freq * pl->elem;
  const size_t grid_curve = (size_t)pl->g.P * (size_t)pl->g.L * pl->elem;
  const size_t tb_half = align256(tile_bounds_bytes(pl->g, pl->log_tile, pl->wave));
  hipStream_t sd = pl->side;
  hipError_t e = hipEventRecord(pl->ev_start, st);  // moments are done before any spreading
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  if ((e = hipStreamWaitEvent(sd, pl->ev_start, 0)) != hipSuccess)
    return hip_fail(e, "hipStreamWaitEvent");
  int i = 0;
  for (int c0 = cbeg; c0 < cend; c0 += pl->wave, ++i) {
    const int nw = (cend - c0) < pl->wave ? (cend - c0) : pl->wave;
    const int b = i & 1;
    char* gA = ws + pl->off_gA + (size_t)b * grid_curve * pl->wave;
    int32_t* tb = (int32_t*)(ws + pl->off_tb + (size_t)b * tb_half);
    void* gB = ws + pl->off_gB;
    void* zc = ws + pl->off_zc + (keep ? (size_t)c0 * zc_curve : 0);
    if (i >= 2 && (e = hipStreamWaitEvent(sd, pl->ev_first[b], 0)) != hipSuccess)
      return hip_fail(e, "hipStreamWaitEvent");
    if ((e = prof_mark(pl, FCHI2_PROF_SPREAD, sd)) != hipSuccess)
      return hip_fail(e, "profiling event");
    e = launch_spread(pl->fp64, t, x, sigma, mom, pl->g, c0, nw, pl->max_n, tb, gA,
                      pl->log_tile, sd);
    if (e != hipSuccess) return hip_fail(e, "spread");
    if ((e = prof_mark(pl, -1, sd)) != hipSuccess) return hip_fail(e, "profiling event");
    if ((e = hipEventRecord(pl->ev_spread[b], sd)) != hipSuccess)
      return hip_fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(st, pl->ev_spread[b], 0)) != hipSuccess)
      return hip_fail(e, "hipStreamWaitEvent");
    const AfterLast after = tail(c0, nw, zc);
    const AfterFirst first_done = [&]() -> fchi2_status_t {
      hipError_t ef = hipEventRecord(pl->ev_first[b], st);
      return ef == hipSuccess ? FCHI2_OK : hip_fail(ef, "hipEventRecord");
    };
    fchi2_status_t s = enqueue_fft(pl, MODE_FWD, gA, gB, zc, mom, c0, nw, st, nullptr, nullptr,
                                   nullptr, sub, &after, &first_done);
    if (s != FCHI2_OK) return s;
  }
  return FCHI2_OK;
}

// The whole forward chain for curves [cbeg, cend), in waves of pl->wave.
fchi2_status_t enqueue_search(fchi2_plan_s* pl, int cbeg, int cend, const double* t,
                              const double* x, const double* sigma, char* ws, void* dchi2,
                              double* chi2_0, uint8_t* flags, hipStream_t st,
                              void* coef = nullptr) {
  Moments* mom = (Moments*)(ws + pl->off_mom);
  PROF_BEGIN(FCHI2_PROF_MOMENTS);
  hipError_t e = launch_moments(t, x, sigma, pl->d_off + cbeg, cend - cbeg, pl->mom_bpc, pl->g,
                                (MomPart*)(ws + pl->off_part) + (size_t)cbeg * pl->mom_bpc,
                                mom + cbeg, chi2_0 ? chi2_0 + cbeg : nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "moments");
  PROF_END();
  if (use_persist(pl) && !coef)
    return enqueue_persistent(pl, cbeg, cend, t, x, sigma, ws, dchi2, flags, st);
  if (use_overlap(pl, cend - cbeg)) {
    const size_t zc_curve = (size_t)pl->g.P * 2 * pl->g.n_freq * pl->elem;
    const WaveTail tail = [=](int c0, int, void* zc) -> AfterLast {
      return [=](int off, int n) -> fchi2_status_t {
        PROF_BEGIN(FCHI2_PROF_SOLVE);
        hipError_t es = launch_solve(pl->fp64, (char*)zc + (size_t)off * zc_curve, pl->d_D, mom,
                                     pl->g, c0 + off, n, pl->eps_piv, dchi2, flags, st, coef,
                                     (pl->desc.flags & FCHI2_WIDE_SOLVE) != 0);
        if (es != hipSuccess) return hip_fail(es, "solve");
        PROF_END();
        return FCHI2_OK;
      };
    };
    return enqueue_waves_overlap(pl, cbeg, cend, t, x, sigma, ws, st, pl->solve_sub, tail);
  }
  const bool keep = pl->desc.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)pl->g.P * 2 * pl->g.n_freq * pl->elem;
  for (int c0 = cbeg; c0 < cend; c0 += pl->wave) {
    const int nw = (cend - c0) < pl->wave ? (cend - c0) : pl->wave;
    void* gA = ws + pl->off_gA;
    void* gB = ws + pl->off_gB;
    void* zc = ws + pl->off_zc + (keep ? (size_t)c0 * zc_curve : 0);
    const double* pts[3] = {t, x, sigma};
    int32_t* tb = (int32_t*)(ws + pl->off_tb);
    PROF_BEGIN(FCHI2_PROF_SPREAD);
    if (!use_fused(pl))
      e = launch_spread(pl->fp64, t, x, sigma, mom, pl->g, c0, nw, pl->max_n, tb, gA,
                        pl->log_tile, st);
    else
      e = launch_tile_bounds(t, mom, pl->g, c0, nw, pl->max_n, tb, kFusedTbLog, st);
    if (e != hipSuccess) return hip_fail(e, "spread");
    PROF_END();
    const AfterLast solve = [&](int off, int n) -> fchi2_status_t {
      PROF_BEGIN(FCHI2_PROF_SOLVE);
      hipError_t es = launch_solve(pl->fp64, (char*)zc + (size_t)off * zc_curve, pl->d_D, mom,
                                   pl->g, c0 + off, n, pl->eps_piv, dchi2, flags, st, coef,
                                   (pl->desc.flags & FCHI2_WIDE_SOLVE) != 0);
      if (es != hipSuccess) return hip_fail(es, "solve");
      PROF_END();
      return FCHI2_OK;
    };
    fchi2_status_t s = enqueue_fft(pl, MODE_FWD, gA, gB, zc, mom, c0, nw, st, nullptr,
                                   use_fused(pl) ? pts : nullptr, tb, pl->solve_sub, &solve);
    if (s != FCHI2_OK) return s;
  }
  return FCHI2_OK;
}

size_t top_ws_offset(const fchi2_plan_s* pl) { return align256(pl->ws_bytes); }

size_t top_ws_bytes(const fchi2_plan_s* pl, int K) {
  return top_ws_offset(pl) + top_scratch_bytes(pl->g.n_freq, pl->g.H, pl->wave_max, K);
}

// The forward chain with the significance epilogue in place of the rows.
fchi2_status_t enqueue_search_top(fchi2_plan_s* pl, const double* t, const double* x,
                                  const double* sigma, char* ws, int hrow, int64_t k_lo, int K,
                                  double* chi2_0, const TopOut& out, hipStream_t st) {
  const int nc = pl->desc.n_curves;
  Moments* mom = (Moments*)(ws + pl->off_mom);
  PROF_BEGIN(FCHI2_PROF_MOMENTS);
  hipError_t e = launch_moments(t, x, sigma, pl->d_off, nc, pl->mom_bpc, pl->g,
                                (MomPart*)(ws + pl->off_part), mom, chi2_0, st);
  if (e != hipSuccess) return hip_fail(e, "moments");
  PROF_END();
  const bool keep = pl->desc.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)pl->g.P * 2 * pl->g.n_freq * pl->elem;
  const TopScratch sc = top_scratch_carve(ws + top_ws_offset(pl), pl->g.n_freq, pl->g.H,
                                          pl->wave_max, K);
  if (use_overlap(pl, nc)) {
    const WaveTail tail = [=](int c0, int nw, void* zc) -> AfterLast {
      return [=](int, int) -> fchi2_status_t {
        PROF_BEGIN(FCHI2_PROF_SOLVE);
        hipError_t es = launch_solve_top(pl->fp64, zc, pl->d_D, mom, pl->g, c0, nw, pl->eps_piv,
                                         hrow, k_lo, K, sc, st);
        if (es != hipSuccess) return hip_fail(es, "solve with candidate selection");
        PROF_END();
        PROF_BEGIN(FCHI2_PROF_TOP_MERGE);
        es = launch_top_merge(mom, pl->g, c0, nw, hrow, K, sc, out, st);
        if (es != hipSuccess) return hip_fail(es, "candidate merge");
        PROF_END();
        return FCHI2_OK;
      };
    };
    return enqueue_waves_overlap(pl, 0, nc, t, x, sigma, ws, st, 0, tail);
  }
  for (int c0 = 0; c0 < nc; c0 += pl->wave) {
    const int nw = (nc - c0) < pl->wave ? (nc - c0) : pl->wave;
    void* gA = ws + pl->off_gA;
    void* gB = ws + pl->off_gB;
    void* zc = ws + pl->off_zc + (keep ? (size_t)c0 * zc_curve : 0);
    const double* pts[3] = {t, x, sigma};
    int32_t* tb = (int32_t*)(ws + pl->off_tb);
    PROF_BEGIN(FCHI2_PROF_SPREAD);
    if (!use_fused(pl))
      e = launch_spread(pl->fp64, t, x, sigma, mom, pl->g, c0, nw, pl->max_n, tb, gA,
                        pl->log_tile, st);
    else
      e = launch_tile_bounds(t, mom, pl->g, c0, nw, pl->max_n, tb, kFusedTbLog, st);
    if (e != hipSuccess) return hip_fail(e, "spread");
    PROF_END();
    fchi2_status_t s = enqueue_fft(pl, MODE_FWD, gA, gB, zc, mom, c0, nw, st, nullptr,
                                   use_fused(pl) ? pts : nullptr, tb);
    if (s != FCHI2_OK) return s;
    PROF_BEGIN(FCHI2_PROF_SOLVE);
    e = launch_solve_top(pl->fp64, zc, pl->d_D, mom, pl->g, c0, nw, pl->eps_piv, hrow, k_lo, K,
                         sc, st);
    if (e != hipSuccess) return hip_fail(e, "solve with candidate selection");
    PROF_END();
    PROF_BEGIN(FCHI2_PROF_TOP_MERGE);
    e = launch_top_merge(mom, pl->g, c0, nw, hrow, K, sc, out, st);
    if (e != hipSuccess) return hip_fail(e, "candidate merge");
    PROF_END();
  }
  return FCHI2_OK;
}

// Sources sharing one time base (shared-alpha search): geometry of the weight
// grids (the first H pairs of the plan's layout) and of one source's data
// grids (the remaining ceil(H/2) pairs), and the workspace layout.
struct MultiLayout {
  Geom gq, gp;
  int wave = 1;
  size_t off_mt = 0, off_pt = 0, off_ms = 0, off_ps = 0, off_tb = 0, off_gA = 0, off_gB = 0,
         off_zq = 0, off_zp = 0, bytes = 0;
};

MultiLayout multi_layout(const fchi2_plan_s* pl, int S) {
  MultiLayout m;
  m.gq = pl->g;
  m.gq.P = pl->g.H;
  m.gp = pl->g;
  const int pd = (pl->g.H + 1) / 2;
  m.gp.P = pd;
  for (int j = 0; j < pd; ++j)
    for (int c = 0; c < 2; ++c) {
      m.gp.comp_m[j][c] = pl->g.comp_m[pl->g.H + j][c];
      m.gp.comp_kind[j][c] = pl->g.comp_kind[pl->g.H + j][c];
    }
  for (int j = pd; j < kMaxPairs; ++j)
    for (int c = 0; c < 2; ++c) m.gp.comp_m[j][c] = 0;
  const size_t grid_src = (size_t)pd * (size_t)pl->g.L * pl->elem;
  size_t cap = ((size_t)8 << 30) / (2 * grid_src);
  if (cap < 1) cap = 1;
  m.wave = (int)(cap < (size_t)S ? cap : (size_t)S);
  const size_t pairs = std::max<size_t>((size_t)pl->g.H, (size_t)m.wave * pd);
  size_t off = 0;
  m.off_mt = off;
  off = align256(off + sizeof(Moments));
  m.off_pt = off;
  off = align256(off + sizeof(MomPart) * (size_t)pl->mom_bpc);
  m.off_ms = off;
  off = align256(off + sizeof(Moments) * (size_t)S);
  m.off_ps = off;
  off = align256(off + sizeof(MomPart) * (size_t)S * pl->mom_bpc);
  m.off_tb = off;
  off = align256(off + tile_bounds_bytes(pl->g, 10, 1));
  m.off_gA = off;
  off = align256(off + pairs * (size_t)pl->g.L * pl->elem);
  m.off_gB = off;
  off = align256(off + pairs * (size_t)pl->g.L * pl->elem);
  m.off_zq = off;
  off = align256(off + (size_t)pl->g.H * 2 * (size_t)pl->g.n_freq * pl->elem);
  m.off_zp = off;
  off = align256(off + (size_t)m.wave * pd * 2 * (size_t)pl->g.n_freq * pl->elem);
  m.bytes = off;
  return m;
}

fchi2_status_t enqueue_multi(fchi2_plan_s* pl, const MultiLayout& m, const double* t,
                             const double* sigma, const double* x, const double* scale, int S,
                             char* ws, void* dchi2, double* chi2_0, uint8_t* flags,
                             hipStream_t st) {
  Moments* mt = (Moments*)(ws + m.off_mt);
  Moments* ms = (Moments*)(ws + m.off_ms);
  int32_t* tb = (int32_t*)(ws + m.off_tb);
  void* gA = ws + m.off_gA;
  void* gB = ws + m.off_gB;
  void* zq = ws + m.off_zq;
  void* zp = ws + m.off_zp;
  PROF_BEGIN(FCHI2_PROF_MOMENTS);
  // The shared time base: sigma stands in for the data (only the weights,
  // T0, span and the validity of t and sigma are used).
  hipError_t e = launch_moments(t, sigma, sigma, pl->d_off, 1, pl->mom_bpc, pl->g,
                                (MomPart*)(ws + m.off_pt), mt, nullptr, st);
  if (e == hipSuccess)
    e = launch_moments(t, x, sigma, pl->d_off, S, pl->mom_bpc, pl->g, (MomPart*)(ws + m.off_ps),
                       ms, chi2_0, st, true, scale);
  if (e != hipSuccess) return hip_fail(e, "moments");
  PROF_END();
  PROF_BEGIN(FCHI2_PROF_SPREAD);
  e = launch_spread(pl->fp64, t, x, sigma, mt, m.gq, 0, 1, pl->max_n, tb, gA, pl->log_tile, st);
  if (e != hipSuccess) return hip_fail(e, "spread (weights)");
  PROF_END();
  fchi2_status_t s = enqueue_fft(pl, MODE_FWD, gA, gB, zq, mt, 0, 1, st, &m.gq);
  if (s != FCHI2_OK) return s;
  for (int s0 = 0; s0 < S; s0 += m.wave) {
    const int nw = (S - s0) < m.wave ? (S - s0) : m.wave;
    PROF_BEGIN(FCHI2_PROF_SPREAD);
    e = launch_spread(pl->fp64, t, x, sigma, ms, m.gp, s0, nw, pl->max_n, tb, gA, pl->log_tile,
                      st, true);
    if (e != hipSuccess) return hip_fail(e, "spread (sources)");
    PROF_END();
    s = enqueue_fft(pl, MODE_FWD, gA, gB, zp, ms, s0, nw, st, &m.gp);
    if (s != FCHI2_OK) return s;
    PROF_BEGIN(FCHI2_PROF_SOLVE);
    e = launch_solve_multi(pl->fp64, zq, zp, pl->d_D, mt, ms, scale, pl->g, s0, nw, pl->eps_piv,
                           dchi2, flags, st);
    if (e != hipSuccess) return hip_fail(e, "shared-alpha solve");
    PROF_END();
  }
  return FCHI2_OK;
}

fchi2_status_t check_ws(fchi2_plan_s* pl, void* ws, size_t bytes) {
  if (!ws) return fail(FCHI2_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(FCHI2_ERR_ARG, "workspace must be 256-byte aligned");
  if (bytes < pl->ws_bytes)
    return fail(FCHI2_ERR_ARG, "workspace too small: %zu < %zu bytes", bytes, pl->ws_bytes);
  return FCHI2_OK;
}

// Schedule search with `run`.  Stage 1 times every (FFT split, spreading
// tile) on the largest wave (plus the fused first pass and the persistent
// search where allowed); stage 2 times, for the fastest candidate of each of
// the three fastest FFT splits of stage 1 (the best wave size differs between
// splits: their passes share the CUs differently with the overlapped
// spreading), every wave size, each with the last pass and solve run on the
// whole wave or on half-waves (allow_sub).  Each candidate runs 3 times (the first a
// warm-up, the faster of the other two kept); then the three fastest of all
// run again, in turns, five times each, and the one with the lowest time is
// returned: the first rounds rank, the last decides between close candidates
// whose order one noisy measurement could swap.  The plan is left on the
// last candidate tried.
struct TuneCand {
  FftPlan f;
  int tile, wave, fused, persist, sub;
  float ms;
};

template <typename Run>
fchi2_status_t tune_loop(fchi2_plan_s* pl, const std::vector<FftPlan>& splits,
                         const std::vector<int>& waves, bool allow_fused, bool allow_persist,
                         bool allow_sub, Run run, hipStream_t st, float& best_ms,
                         TuneCand& best) {
  hipEvent_t e0, e1;
  hipError_t ce = hipEventCreate(&e0);
  if (ce != hipSuccess) return hip_fail(ce, "hipEventCreate");
  ce = hipEventCreate(&e1);
  if (ce != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(ce, "hipEventCreate");
  }
  fchi2_status_t res = FCHI2_OK;
  // One timed run of candidate c into ms.
  auto time_one = [&](const TuneCand& c, float& ms) {
    pl->log_tile = c.tile;
    pl->wave = c.wave;
    pl->fused = c.fused;
    pl->persist = c.persist;
    pl->solve_sub = c.sub;
    apply_fft_plan(pl, c.f);
    hipError_t e = hipEventRecord(e0, st);
    if (e == hipSuccess) res = run();
    if (e == hipSuccess && res == FCHI2_OK) e = hipEventRecord(e1, st);
    if (e == hipSuccess && res == FCHI2_OK) e = hipEventSynchronize(e1);
    ms = 0.f;
    if (e == hipSuccess && res == FCHI2_OK) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) res = hip_fail(e, "autotune timing");
  };
  auto time_all = [&](std::vector<TuneCand>& cs) {
    for (TuneCand& c : cs) {
      for (int rep = 0; rep < 3 && res == FCHI2_OK; ++rep) {
        float ms = 0.f;
        time_one(c, ms);
        if (rep > 0 && res == FCHI2_OK && ms < c.ms) c.ms = ms;  // first run warms up
      }
      if (res != FCHI2_OK) return;
    }
  };
  auto by_time = [](const TuneCand& a, const TuneCand& b) { return a.ms < b.ms; };
  std::vector<TuneCand> cands;
  const int w0 = waves[0];
  for (const FftPlan& f : splits) {
    for (int tile : {10, 11, 12, 13}) cands.push_back(TuneCand{f, tile, w0, 0, 0, 0, 1e30f});
    // The fused schedule has no spreading tile.
    if (allow_fused && f.np >= 2) cands.push_back(TuneCand{f, 10, w0, 1, 0, 0, 1e30f});
    // The persistent search has no waves.
    for (int tile : {10, 11})
      if (allow_persist && persist_ok(pl, f, tile) && persist_worth_timing(pl))
        cands.push_back(TuneCand{f, tile, w0, 0, 1, 0, 1e30f});
  }
  time_all(cands);
  if (res == FCHI2_OK && !cands.empty()) {
    std::stable_sort(cands.begin(), cands.end(), by_time);
    std::vector<TuneCand> more;
    std::vector<FftPlan> taken;
    auto same_split = [](const FftPlan& a, const FftPlan& b) {
      if (a.np != b.np) return false;
      for (int q = 1; q <= a.np; ++q)
        if (a.logn[q] != b.logn[q] || a.le[q] != b.le[q]) return false;
      return true;
    };
    for (size_t i = 0; i < cands.size() && taken.size() < 3; ++i) {
      if (cands[i].persist) continue;
      bool seen = false;
      for (const FftPlan& f : taken) seen = seen || same_split(f, cands[i].f);
      if (seen) continue;
      taken.push_back(cands[i].f);
      for (int wave : waves)
        for (int half = 0; half <= (allow_sub ? 1 : 0); ++half) {
          TuneCand c = cands[i];
          c.wave = wave;
          c.sub = half ? wave / 2 : 0;
          c.ms = 1e30f;
          if (half && c.sub < 1) continue;
          if (wave == w0 && !half) continue;  // timed in stage 1
          more.push_back(c);
        }
    }
    time_all(more);
    cands.insert(cands.end(), more.begin(), more.end());
  }
  if (res == FCHI2_OK && !cands.empty()) {
    std::stable_sort(cands.begin(), cands.end(), by_time);
    const size_t top = cands.size() < 3 ? cands.size() : 3;
    std::vector<float> again(top, 1e30f);
    for (int rep = 0; rep < 5 && res == FCHI2_OK; ++rep)
      for (size_t i = 0; i < top && res == FCHI2_OK; ++i) {
        float ms = 0.f;
        time_one(cands[i], ms);
        if (res == FCHI2_OK && ms < again[i]) again[i] = ms;
      }
    if (res == FCHI2_OK) {
      size_t bi = 0;
      for (size_t i = 1; i < top; ++i)
        if (again[i] < again[bi]) bi = i;
      if (again[bi] < best_ms) {
        best_ms = again[bi];
        best = cands[bi];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

void apply_tuned(fchi2_plan_s* pl, const TuneCand& c) {
  pl->log_tile = c.tile;
  pl->wave = c.wave;
  pl->fused = c.fused;
  pl->persist = c.persist;
  pl->solve_sub = c.sub;
  apply_fft_plan(pl, c.f);
}

}  // namespace

extern "C" {

const char* fchi2_status_string(fchi2_status_t s) {
  switch (s) {
    case FCHI2_OK: return "ok";
    case FCHI2_ERR_ARG: return "invalid argument";
    case FCHI2_ERR_NOMEM: return "out of device memory";
    case FCHI2_ERR_HIP: return "HIP runtime error";
    case FCHI2_ERR_STATE: return "invalid state";
    case FCHI2_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* fchi2_last_error(void) { return g_err.c_str(); }

fchi2_status_t fchi2_plan(const fchi2_plan_desc_t* desc, void* stream, fchi2_plan_t* out) {
  g_err.clear();
  if (!desc || !out) return fail(FCHI2_ERR_ARG, "desc and out must not be NULL");
  *out = nullptr;
  const fchi2_plan_desc_t& d = *desc;
  if (d.n_curves < 1) return fail(FCHI2_ERR_ARG, "n_curves must be >= 1 (got %d)", d.n_curves);
  if (!d.offsets) return fail(FCHI2_ERR_ARG, "offsets must not be NULL");
  if (d.offsets[0] != 0) return fail(FCHI2_ERR_ARG, "offsets[0] must be 0");
  for (int c = 0; c < d.n_curves; ++c)
    if (d.offsets[c + 1] < d.offsets[c])
      return fail(FCHI2_ERR_ARG, "offsets must be nondecreasing (curve %d)", c);
  if (!(d.f_max > 0.0) || !std::isfinite(d.f_max))
    return fail(FCHI2_ERR_ARG, "f_max must be finite and > 0");
  if (d.H < 1 || d.H > FCHI2_H_MAX)
    return fail(FCHI2_ERR_ARG, "H must be in 1..%d (got %d)", FCHI2_H_MAX, d.H);
  int64_t n_freq = d.n_freq;
  double span = 0.0;  // longest span, if the caller gave them
  if (d.t_span) {
    for (int c = 0; c < d.n_curves; ++c) {
      if (!(d.t_span[c] >= 0.0) || !std::isfinite(d.t_span[c]))
        return fail(FCHI2_ERR_ARG, "t_span[%d] must be finite and >= 0", c);
      span = d.t_span[c] > span ? d.t_span[c] : span;
    }
  }
  if (n_freq == 0) {
    const double os = d.oversampling == 0.0 ? 5.0 : d.oversampling;
    if (!(os > 0.0) || !std::isfinite(os))
      return fail(FCHI2_ERR_ARG, "oversampling must be finite and > 0");
    if (!d.t_span) return fail(FCHI2_ERR_ARG, "n_freq = 0 needs t_span (host per-curve spans)");
    if (!(span > 0.0)) return fail(FCHI2_ERR_ARG, "n_freq = 0 needs a curve with span > 0");
    n_freq = fchi2_auto_n_freq(d.H, d.f_max, os, span);
    if (n_freq == 0)
      return fail(FCHI2_ERR_UNSUPPORTED,
                  "n_freq from os * H * span * f_max = %.4g exceeds 2^24",
                  os * (double)d.H * span * d.f_max);
  }
  if (!is_pow2(n_freq)) return fail(FCHI2_ERR_ARG, "n_freq must be a power of two");
  if (n_freq < (1 << 10) || n_freq > (1 << 24))
    return fail(FCHI2_ERR_UNSUPPORTED, "n_freq must be in 2^10..2^24");
  if (d.precision != FCHI2_FP64 && d.precision != FCHI2_MIXED)
    return fail(FCHI2_ERR_ARG, "precision must be FCHI2_FP64 or FCHI2_MIXED");
  if (d.flags & ~(uint32_t)(FCHI2_KEEP_FOR_BACKWARD | FCHI2_GRAPH | FCHI2_FUSED_SPREAD |
                            FCHI2_WIDE_SOLVE | FCHI2_PERSISTENT | FCHI2_TWO_STREAMS))
    return fail(FCHI2_ERR_ARG, "unknown flag bits 0x%x", d.flags);
  if ((d.H > kHMax || (d.flags & FCHI2_WIDE_SOLVE)) && (d.flags & FCHI2_KEEP_FOR_BACKWARD))
    return fail(FCHI2_ERR_UNSUPPORTED, "backward needs H <= %d (the register solver)", kHMax);
  if ((d.H > kHMax || (d.flags & FCHI2_WIDE_SOLVE)) && d.first_bin > 0)
    return fail(FCHI2_ERR_UNSUPPORTED, "band plans need H <= %d (the register solver)", kHMax);
  if ((d.flags & FCHI2_FUSED_SPREAD) && d.first_bin > 0)
    return fail(FCHI2_ERR_UNSUPPORTED, "band plans (first_bin > 0) spread in a kernel of their own");
  if (d.kernel_width != 0 && d.kernel_width != 1 && (d.kernel_width < 4 || d.kernel_width > 16))
    return fail(FCHI2_ERR_ARG, "kernel_width must be 0, 1 (floor gridding) or 4..16");
  if (d.kernel_width == 1 && (d.flags & FCHI2_KEEP_FOR_BACKWARD))
    return fail(FCHI2_ERR_UNSUPPORTED, "floor gridding has no backward");
  if (d.curves_per_wave < 0) return fail(FCHI2_ERR_ARG, "curves_per_wave must be >= 0");
  if (d.first_bin < 0) return fail(FCHI2_ERR_ARG, "first_bin must be >= 0");
  if (d.first_bin > ((int64_t)1 << 40))
    return fail(FCHI2_ERR_UNSUPPORTED, "first_bin must be <= 2^40");
  if (d.first_bin > 0 && (d.flags & FCHI2_KEEP_FOR_BACKWARD))
    return fail(FCHI2_ERR_UNSUPPORTED, "band plans (first_bin > 0) have no backward");
  if (d.first_bin > 0 && d.kernel_width == 1)
    return fail(FCHI2_ERR_UNSUPPORTED, "band plans (first_bin > 0) have no floor gridding");

  fchi2_plan_s* pl = new fchi2_plan_s();
  pl->desc = d;
  pl->desc.n_freq = n_freq;
  pl->desc.t_span = nullptr;  // caller memory, not kept
  pl->offsets.assign(d.offsets, d.offsets + d.n_curves + 1);
  pl->desc.offsets = pl->offsets.data();
  pl->n_total = pl->offsets.back();
  pl->fp64 = (d.precision == FCHI2_FP64);
  pl->elem = pl->fp64 ? 16 : 8;
  pl->out_elem = pl->fp64 ? 8 : 4;
  pl->eps_piv = pl->fp64 ? 1e-13 : 1e-6;

  Geom& g = pl->g;
  g.n_freq = n_freq;
  // Real grids of 4 n_freq cells keep bins k < n_freq (upsampling 2 over
  // [-n_freq, n_freq)); a band plan's complex grids are centred on the band,
  // whose offsets [-n_freq/2, n_freq/2) need 2 n_freq cells for the same
  // upsampling.
  g.L = (d.first_bin > 0 ? 2 : 4) * n_freq;
  g.df = d.f_max / (double)n_freq;
  g.w = d.kernel_width ? d.kernel_width : (pl->fp64 ? 14 : 10);
  g.half_w = 0.5 * g.w;
  g.beta = 2.30 * g.w;
  g.c_off = g.w == 1 ? 0 : g.w / 2 + 2;
  // Grid periods the tile tables cover.  The phase m u of harmonic m runs
  // over m df span cycles: beyond one cycle it wraps around the periodic grid
  // (Section 3b sizes its arrays to cover 2H times the span, which holds only
  // for a fine enough grid).  With the spans known, exactly what the longest
  // curve needs (at most kMaxLaps); otherwise two periods.
  g.laps = 2;
  if (span > 0.0) {
    const double reach = (2.0 * d.H) * span * (d.f_max / (double)n_freq) * (double)g.L +
                         (double)g.c_off + (double)(g.w / 2) + 3.0;
    const double lp = std::floor(reach / (double)g.L) + 1.0;
    g.laps = (int)std::min<double>(std::max<double>(lp, 1.0), (double)kMaxLaps);
  }
  g.H = d.H;
  g.band = d.first_bin > 0 ? 1 : 0;
  g.k0 = d.first_bin;
  g.P = g.band ? 3 * d.H : d.H + (d.H + 1) / 2;
  std::memset(g.comp_m, 0, sizeof g.comp_m);
  std::memset(g.comp_kind, 0, sizeof g.comp_kind);
  // Band plans: the modulated strengths are complex, so grid p holds one
  // harmonic, q_{p+1} for p < 2H and p_{p-2H+1} after.
  // Otherwise like is packed with like, so each FFT's rounding noise scales
  // with the norm of grids of the same kind: pairs p < H hold the weight grids
  // (q_{2p+1}, q_{2p+2}); pairs p >= H hold the weighted-data grids
  // (p_{2j+1}, p_{2j+2}), j = p - H, the second part empty past H.
  for (int p = 0; p < g.P && g.band; ++p) {
    g.comp_m[p][0] = (int8_t)(p < 2 * d.H ? p + 1 : p - 2 * d.H + 1);
    g.comp_kind[p][0] = (int8_t)(p < 2 * d.H ? 0 : 1);
  }
  for (int p = 0; p < g.P && !g.band; ++p) {
    if (p < d.H) {
      g.comp_m[p][0] = (int8_t)(2 * p + 1);
      g.comp_m[p][1] = (int8_t)(2 * p + 2);
      g.comp_kind[p][0] = 0;
      g.comp_kind[p][1] = 0;
    } else {
      const int j = p - d.H;
      g.comp_m[p][0] = (int8_t)(2 * j + 1);
      g.comp_m[p][1] = (int8_t)(2 * j + 2 <= d.H ? 2 * j + 2 : 0);
      g.comp_kind[p][0] = 1;
      g.comp_kind[p][1] = 1;
    }
  }
  const int logL = ilog2(g.L);
  if (!plan_fft(logL, 12, pl->fp)) {
    delete pl;
    return fail(FCHI2_ERR_UNSUPPORTED, "no FFT pass split for L = 2^%d", logL);
  }
  pl->log_tile = 10;
  pl->fused = (d.flags & FCHI2_FUSED_SPREAD) ? 1 : 0;
  pl->persist = (d.flags & FCHI2_PERSISTENT) ? 1 : 0;
  apply_fft_plan(pl, pl->fp);

  // Waves: bound the two grid buffers to ~8 GiB unless the caller chose.
  const size_t grid_curve = (size_t)g.P * (size_t)g.L * pl->elem;
  if (d.curves_per_wave > 0) {
    pl->wave = d.curves_per_wave < d.n_curves ? d.curves_per_wave : d.n_curves;
  } else {
    size_t cap = ((size_t)8 << 30) / (2 * grid_curve);
    if (cap < 1) cap = 1;
    pl->wave = (int)(cap < (size_t)d.n_curves ? cap : (size_t)d.n_curves);
  }
  pl->wave_max = pl->wave;
  const bool keep = d.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)g.P * 2 * (size_t)g.n_freq * pl->elem;
  pl->blocks_per_curve = (int)((g.n_freq + 255) / 256);
  int64_t max_n = 0;
  for (int c = 0; c < d.n_curves; ++c) {
    const int64_t n = pl->offsets[c + 1] - pl->offsets[c];
    max_n = n > max_n ? n : max_n;
  }
  pl->max_n = max_n;
  pl->mom_bpc = (int)std::min<int64_t>(256, std::max<int64_t>(1, (max_n + 1023) / 1024));
  size_t off = 0;
  pl->off_mom = off;
  off = align256(off + sizeof(Moments) * (size_t)d.n_curves);
  pl->off_part = off;
  off = align256(off + sizeof(MomPart) * (size_t)d.n_curves * pl->mom_bpc);
  pl->off_tb = off;
  // Sized for the finest table: the fused first pass's tiles of 2^kFusedTbLog
  // cells (the spreading kernel's tiles are 2^10 cells or more).
  off = align256(off + tile_bounds_bytes(g, kFusedTbLog, pl->wave));
  pl->off_gA = off;
  off = align256(off + grid_curve * pl->wave);
  pl->off_gB = off;
  off = align256(off + grid_curve * pl->wave);
  pl->off_zc = off;
  off = align256(off + zc_curve * (keep ? (size_t)d.n_curves : (size_t)pl->wave));
  if (keep) {
    pl->off_gq = off;
    off = align256(off + sizeof(double) * (size_t)pl->n_total);
    pl->off_gp = off;
    off = align256(off + sizeof(double) * (size_t)pl->n_total);
    pl->off_dw = off;
    off = align256(off + sizeof(double) * (size_t)d.n_curves * pl->blocks_per_curve);
  }
  // The persistent search's work-queue counter.
  pl->off_queue = off;
  off = align256(off + sizeof(int));
  pl->ws_bytes = off;

  // Persistent search slots: as many workgroups as fit on the device at once
  // (no more than there are curves), each with one pair's grids, all pairs'
  // spectra and the tile table (tiles of 2^10 cells), laid out over the wave
  // buffers (gA, gB, zc), which the persistent search does not otherwise use;
  // never more slots than fit there.
  if (!pl->fp64 && !g.band && d.H <= kHMax && !keep) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        persist_occupancy(d.H, &per_cu) == hipSuccess && cus > 0 && per_cu > 0) {
      const size_t grid1 = (size_t)g.L * pl->elem;
      pl->slot_gB = align256(grid1);
      pl->slot_zc = pl->slot_gB + align256(grid1);
      pl->slot_tb = pl->slot_zc + align256(zc_curve);
      pl->slot_bytes = align256(pl->slot_tb + tile_bounds_bytes(g, 10, 1));
      const size_t room = pl->off_queue - pl->off_gA;
      int64_t n = (int64_t)cus * per_cu;
      pl->n_slots_device = (int)n;
      n = std::min<int64_t>(n, d.n_curves);
      n = std::min<int64_t>(n, (int64_t)(room / pl->slot_bytes));
      pl->n_slots = (int)n;
    }
    (void)hipGetLastError();
  }

  // Device tables.
  hipStream_t st = (hipStream_t)stream;
  auto cleanup_fail = [&](fchi2_status_t s) {
    fchi2_destroy(pl);
    return s;
  };
  hipError_t alloc_err = hipSuccess;
  auto dev_alloc = [&](void** p, size_t bytes) -> bool {
    alloc_err = hipMalloc(p, bytes);
    return alloc_err == hipSuccess;
  };
  const int LT = 1 << kStageLog;
  const int64_t NSM = (int64_t)1 << fft_tile_log(pl->fp64);
  const int n_gl = 128;
  if (!dev_alloc((void**)&pl->d_off, sizeof(int64_t) * (d.n_curves + 1)) ||
      !dev_alloc(&pl->d_tw_stage, 16 * (size_t)LT) ||
      !dev_alloc(&pl->d_tw_small, 16 * (size_t)NSM) ||
      !dev_alloc(&pl->d_D, 16 * (size_t)g.n_freq) ||
      !dev_alloc((void**)&pl->d_gl, sizeof(double) * n_gl)) {
    (void)hipGetLastError();
    // Out of device memory is NOMEM; anything else (no device, a broken
    // runtime) is a HIP error carrying the runtime's message.
    if (alloc_err == hipErrorOutOfMemory)
      return cleanup_fail(fail(FCHI2_ERR_NOMEM, "plan table allocation failed"));
    return cleanup_fail(hip_fail(alloc_err, "plan table allocation"));
  }
  // FP64 twiddle tables: omega_{2^13}^e and omega_L^e for e < 2^tile.
  std::vector<double> hs(2 * (size_t)LT), hsm(2 * (size_t)NSM);
  auto root = [](int64_t e, int64_t n, double* out2) {
    const long double ang = 2.0L * (long double)M_PI * (long double)(e % n) / (long double)n;
    out2[0] = (double)std::cos(ang);
    out2[1] = (double)std::sin(ang);
  };
  for (int64_t e = 0; e < LT; ++e) root(e, LT, &hs[2 * e]);
  for (int64_t e = 0; e < NSM; ++e) root(e, g.L, &hsm[2 * e]);
  std::vector<double> gx, gw, gl(n_gl);
  gauss_legendre(n_gl, gx, gw);
  // Positive nodes; weights fold in the kernel value and the factor w.
  for (int q = 0; q < n_gl / 2; ++q) {
    const double z = gx[n_gl / 2 + q];
    const double phi = std::exp(g.beta * (std::sqrt(1.0 - z * z) - 1.0));
    gl[q] = z;
    gl[n_gl / 2 + q] = (double)g.w * gw[n_gl / 2 + q] * phi;
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(pl->d_off, pl->offsets.data(), sizeof(int64_t) * (d.n_curves + 1),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_tw_stage, hs.data(), sizeof(double) * hs.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_tw_small, hsm.data(), sizeof(double) * hsm.size(),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(pl->d_gl, gl.data(), sizeof(double) * n_gl, hipMemcpyHostToDevice,
                          st)) != hipSuccess ||
      (e = launch_deconv_init(pl->d_D, g, pl->d_gl, pl->d_gl + n_gl / 2, n_gl / 2,
                              st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    return cleanup_fail(hip_fail(e, "plan table setup"));
  }
  // The no-allocation search's device scratch: look up its address on this
  // device now (set-up), so that later calls only read the cached pointer.
  void* sp = nullptr;
  if ((e = scratch_address(&sp)) != hipSuccess)
    return cleanup_fail(hip_fail(e, "hipGetSymbolAddress(scratch)"));
  // The spreading stream of the overlapped wave schedule (default priority).
  if (d.n_curves > 1 && !g.band && (d.flags & FCHI2_TWO_STREAMS)) {
    if ((e = hipStreamCreateWithFlags(&pl->side, hipStreamNonBlocking)) != hipSuccess)
      return cleanup_fail(hip_fail(e, "hipStreamCreateWithFlags"));
    for (hipEvent_t* ev : {&pl->ev_start, &pl->ev_spread[0], &pl->ev_spread[1], &pl->ev_first[0],
                           &pl->ev_first[1]})
      if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess)
        return cleanup_fail(hip_fail(e, "hipEventCreateWithFlags"));
  }
  *out = pl;
  return FCHI2_OK;
}

int64_t fchi2_auto_n_freq(int32_t H, double f_max, double oversampling, double span) {
  if (H < 1 || H > FCHI2_H_MAX) return 0;
  if (!(f_max > 0.0) || !(oversampling > 0.0) || !(span > 0.0)) return 0;
  if (!std::isfinite(f_max) || !std::isfinite(oversampling) || !std::isfinite(span)) return 0;
  const double want = std::ceil(oversampling * (double)H * span * f_max);
  if (!(want <= (double)(1 << 24))) return 0;
  int64_t n = (int64_t)1 << 10;
  while ((double)n < want) n <<= 1;
  return n;
}

int64_t fchi2_plan_n_freq(fchi2_plan_t plan) { return plan ? plan->g.n_freq : 0; }

size_t fchi2_workspace_bytes(fchi2_plan_t plan) { return plan ? plan->ws_bytes : 0; }

int64_t fchi2_total_points(fchi2_plan_t plan) { return plan ? plan->n_total : 0; }

fchi2_status_t fchi2_search(fchi2_plan_t plan, const double* t, const double* x,
                            const double* sigma, void* workspace, size_t workspace_bytes,
                            void* dchi2, double* chi2_0, uint8_t* flags, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !dchi2) return fail(FCHI2_ERR_ARG, "t, x, sigma and dchi2 must not be NULL");
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  plan->last_ws = workspace;
  ++plan->gen;

  if ((plan->desc.flags & FCHI2_GRAPH) && st != nullptr && !plan->prof) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK(hipStreamIsCapturing(st, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      const void* key[8] = {t, x, sigma, workspace, dchi2, chi2_0, flags, nullptr};
      bool same = plan->gexec != nullptr && plan->gkey_ws == workspace_bytes;
      for (int i = 0; i < 8 && same; ++i) same = (plan->gkey[i] == key[i]);
      if (!same) {
        if (plan->gexec) {
          (void)hipGraphExecDestroy(plan->gexec);
          plan->gexec = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        fchi2_status_t es =
            enqueue_search(plan, 0, plan->desc.n_curves, t, x, sigma, ws, dchi2, chi2_0, flags, st);
        hipGraph_t graph = nullptr;
        hipError_t ee = hipStreamEndCapture(st, &graph);
        if (es != FCHI2_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return es;
        }
        if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
        hipError_t ie = hipGraphInstantiate(&plan->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
          plan->gexec = nullptr;
          return hip_fail(ie, "hipGraphInstantiate");
        }
        for (int i = 0; i < 8; ++i) plan->gkey[i] = key[i];
        plan->gkey_ws = workspace_bytes;
      }
      HIPCHK(hipGraphLaunch(plan->gexec, st));
      return FCHI2_OK;
    }
  }
  return enqueue_search(plan, 0, plan->desc.n_curves, t, x, sigma, ws, dchi2, chi2_0, flags, st);
}

fchi2_status_t fchi2_search_noalloc(fchi2_plan_t plan, const double* t, const double* x,
                                    const double* sigma, void* dchi2, double* chi2_0,
                                    uint8_t* flags, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !dchi2) return fail(FCHI2_ERR_ARG, "t, x, sigma and dchi2 must not be NULL");
  if (plan->ws_bytes > (size_t)FCHI2_NOALLOC_SCRATCH_BYTES)
    return fail(FCHI2_ERR_ARG,
                "plan workspace of %zu bytes exceeds the no-allocation scratch of %zu bytes "
                "(fewer curves per wave or bins would fit)",
                plan->ws_bytes, (size_t)FCHI2_NOALLOC_SCRATCH_BYTES);
  if (plan->prof)
    return fail(FCHI2_ERR_STATE, "profiling creates events; disable it for this call");
  void* ws = nullptr;
  HIPCHK(scratch_address(&ws));
  // Nothing in the scratch needs to start at zero: every stage writes what the
  // next one reads (the same contract as a fresh caller workspace).
  plan->last_ws = nullptr;  // the scratch is not a workspace backward can be given
  ++plan->gen;
  return enqueue_search(plan, 0, plan->desc.n_curves, t, x, sigma, (char*)ws, dchi2, chi2_0,
                        flags, (hipStream_t)stream);
}

fchi2_status_t fchi2_search_coeffs(fchi2_plan_t plan, const double* t, const double* x,
                                   const double* sigma, void* workspace, size_t workspace_bytes,
                                   void* dchi2, double* chi2_0, uint8_t* flags, void* coeffs,
                                   void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !dchi2 || !coeffs)
    return fail(FCHI2_ERR_ARG, "t, x, sigma, dchi2 and coeffs must not be NULL");
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  plan->last_ws = workspace;
  ++plan->gen;
  return enqueue_search(plan, 0, plan->desc.n_curves, t, x, sigma, (char*)workspace, dchi2,
                        chi2_0, flags, (hipStream_t)stream, coeffs);
}

fchi2_status_t fchi2_search_curves(fchi2_plan_t plan, int32_t first, int32_t count,
                                   const double* t, const double* x, const double* sigma,
                                   void* workspace, size_t workspace_bytes, void* dchi2,
                                   double* chi2_0, uint8_t* flags, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !dchi2) return fail(FCHI2_ERR_ARG, "t, x, sigma and dchi2 must not be NULL");
  if (first < 0 || count < 1 || (int64_t)first + count > plan->desc.n_curves)
    return fail(FCHI2_ERR_ARG, "curve range [%d, %d) outside 0..%d", first, first + count,
                plan->desc.n_curves);
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  // Only a search over every curve leaves a state fchi2_backward can use.
  plan->last_ws = (first == 0 && count == plan->desc.n_curves) ? workspace : nullptr;
  ++plan->gen;
  return enqueue_search(plan, first, first + count, t, x, sigma, (char*)workspace, dchi2, chi2_0,
                        flags, (hipStream_t)stream);
}

uint64_t fchi2_search_generation(fchi2_plan_t plan) { return plan ? plan->gen : 0; }

fchi2_status_t fchi2_backward(fchi2_plan_t plan, const double* t, const double* x,
                              const double* sigma, const void* grad_dchi2, void* workspace,
                              size_t workspace_bytes, double* grad_x, double* grad_sigma,
                              void* stream) {
  return fchi2_backward_at(plan, plan ? plan->gen : 0, t, x, sigma, grad_dchi2, workspace,
                           workspace_bytes, grad_x, grad_sigma, stream);
}

fchi2_status_t fchi2_backward_at(fchi2_plan_t plan, uint64_t generation, const double* t,
                                 const double* x, const double* sigma, const void* grad_dchi2,
                                 void* workspace, size_t workspace_bytes, double* grad_x,
                                 double* grad_sigma, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!(plan->desc.flags & FCHI2_KEEP_FOR_BACKWARD))
    return fail(FCHI2_ERR_STATE, "plan was created without FCHI2_KEEP_FOR_BACKWARD");
  if (!t || !x || !sigma || !grad_dchi2 || !grad_x || !grad_sigma)
    return fail(FCHI2_ERR_ARG, "t, x, sigma, grad_dchi2, grad_x and grad_sigma must not be NULL");
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  if (plan->last_ws != workspace)
    return fail(FCHI2_ERR_STATE, "fchi2_search has not run on this workspace");
  if (generation != plan->gen)
    return fail(FCHI2_ERR_STATE,
                "the workspace holds the state of search %llu, not of search %llu (another "
                "search ran on the plan since)",
                (unsigned long long)plan->gen, (unsigned long long)generation);
  hipStream_t st = (hipStream_t)stream;
  fchi2_plan_s* pl = plan;
  char* ws = (char*)workspace;
  Moments* mom = (Moments*)(ws + plan->off_mom);
  const size_t zc_curve = (size_t)plan->g.P * 2 * plan->g.n_freq * plan->elem;
  double* gq = (double*)(ws + plan->off_gq);
  double* gp = (double*)(ws + plan->off_gp);
  double* dw = (double*)(ws + plan->off_dw);
  for (int c0 = 0; c0 < plan->desc.n_curves; c0 += plan->wave) {
    const int nw = (plan->desc.n_curves - c0) < plan->wave ? (plan->desc.n_curves - c0) : plan->wave;
    void* gA = ws + plan->off_gA;
    void* gB = ws + plan->off_gB;
    const void* zc = ws + plan->off_zc + (size_t)c0 * zc_curve;
    PROF_BEGIN(FCHI2_PROF_BWD_SOLVE);
    hipError_t e = launch_adjoint_solve(plan->fp64, zc, plan->d_D, mom, plan->g, c0, nw,
                                        plan->eps_piv, grad_dchi2, gA, dw,
                                        plan->blocks_per_curve, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint solve");
    PROF_END();
    s = enqueue_fft(plan, MODE_BWD, gA, gB, nullptr, mom, c0, nw, st);
    if (s != FCHI2_OK) return s;
    int64_t max_n = 0;
    for (int c = c0; c < c0 + nw; ++c) {
      const int64_t n = plan->offsets[c + 1] - plan->offsets[c];
      max_n = n > max_n ? n : max_n;
    }
    PROF_BEGIN(FCHI2_PROF_BWD_GATHER);
    e = launch_gather(plan->fp64, t, mom, plan->g, c0, nw, gA, gq, gp, max_n, st);
    if (e != hipSuccess) return hip_fail(e, "gather");
    PROF_END();
    PROF_BEGIN(FCHI2_PROF_BWD_FINAL);
    // The forward's moment partials (MomPart, 4 doubles each, mom_bpc per
    // curve) are free during the backward: they hold the chunk sums here.
    e = launch_finalize(x, sigma, mom, plan->g, c0, nw, dw, plan->blocks_per_curve, gq, gp,
                        grad_x, grad_sigma, (double*)(ws + plan->off_part), plan->mom_bpc, st);
    if (e != hipSuccess) return hip_fail(e, "finalize");
    PROF_END();
  }
  return FCHI2_OK;
}

size_t fchi2_top_peaks_scratch_bytes(fchi2_plan_t plan, int32_t K) {
  if (!plan || K < 1 || K > 64) return 0;
  return peaks_scratch_bytes(plan->g.n_freq, plan->desc.n_curves, K);
}

fchi2_status_t fchi2_top_peaks(fchi2_plan_t plan, const void* dchi2, int32_t hrow, int64_t k_lo,
                               int32_t K, void* scratch, size_t scratch_bytes, int64_t* out_idx,
                               void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!dchi2 || !scratch || !out_idx) return fail(FCHI2_ERR_ARG, "NULL pointer argument");
  if (K < 1 || K > 64) return fail(FCHI2_ERR_ARG, "K must be in 1..64");
  if (hrow < 0 || hrow >= plan->g.H) return fail(FCHI2_ERR_ARG, "hrow must be in 0..H-1");
  if (k_lo < 1 || k_lo > plan->g.n_freq - 2)
    return fail(FCHI2_ERR_ARG, "k_lo must be in 1..n_freq-2");
  if (((uintptr_t)scratch & 255) != 0) return fail(FCHI2_ERR_ARG, "scratch must be 256-byte aligned");
  if (scratch_bytes < fchi2_top_peaks_scratch_bytes(plan, K))
    return fail(FCHI2_ERR_ARG, "scratch too small");
  hipError_t e = launch_peaks(plan->fp64, dchi2, plan->g.n_freq, plan->g.H, hrow,
                              plan->desc.n_curves, k_lo, K, scratch, out_idx,
                              (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "top peaks");
  return FCHI2_OK;
}

size_t fchi2_search_top_workspace_bytes(fchi2_plan_t plan, int32_t K) {
  if (!plan || K < 1 || K > 64) return 0;
  return top_ws_bytes(plan, K);
}

fchi2_status_t fchi2_search_top(fchi2_plan_t plan, const double* t, const double* x,
                                const double* sigma, void* workspace, size_t workspace_bytes,
                                int32_t hrow, int64_t k_lo, int32_t K, double* chi2_0,
                                const fchi2_top_out_t* out, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !out || !out->idx || !out->log_p)
    return fail(FCHI2_ERR_ARG, "t, x, sigma, out, out->idx and out->log_p must not be NULL");
  if (K < 1 || K > 64) return fail(FCHI2_ERR_ARG, "K must be in 1..64");
  if (hrow < 0 || hrow >= plan->g.H) return fail(FCHI2_ERR_ARG, "hrow must be in 0..H-1");
  if (k_lo < 0) return fail(FCHI2_ERR_ARG, "k_lo must be >= 0");
  if (plan->g.H > kHMax)
    return fail(FCHI2_ERR_UNSUPPORTED, "the significance epilogue needs H <= %d", kHMax);
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  if (workspace_bytes < top_ws_bytes(plan, K))
    return fail(FCHI2_ERR_ARG, "workspace too small for K = %d: %zu < %zu bytes", K,
                workspace_bytes, top_ws_bytes(plan, K));
  plan->last_ws = workspace;
  ++plan->gen;
  TopOut o{out->idx, out->log_p, out->dchi2, out->dchi2_adj, out->flags, out->chi2_best,
           out->curve_flags};
  return enqueue_search_top(plan, t, x, sigma, (char*)workspace, hrow, k_lo, K, chi2_0, o,
                            (hipStream_t)stream);
}

size_t fchi2_fine_scratch_bytes(fchi2_plan_t plan, int32_t K, int32_t R) {
  if (!plan || K < 1 || K > 256 || R < 1 || R > 4096) return 0;
  const int nc = plan->desc.n_curves;
  return align256(sizeof(Moments) * (size_t)nc) +
         align256(sizeof(MomPart) * (size_t)nc * plan->mom_bpc) +
         align256(fine_part_bytes(plan->g.H, nc, plan->max_n, K, R));
}

fchi2_status_t fchi2_fine_search(fchi2_plan_t plan, const double* t, const double* x,
                                 const double* sigma, const double* f_center, int32_t K,
                                 int32_t R, double half_width, int32_t hrow, void* scratch,
                                 size_t scratch_bytes, const fchi2_fine_out_t* out,
                                 void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !f_center || !out || !out->f_best || !out->dchi2_best)
    return fail(FCHI2_ERR_ARG,
                "t, x, sigma, f_center, out, out->f_best and out->dchi2_best must not be NULL");
  if (K < 1 || K > 256) return fail(FCHI2_ERR_ARG, "K must be in 1..256");
  if (R < 1 || R > 4096) return fail(FCHI2_ERR_ARG, "R must be in 1..4096");
  if (plan->g.H > kHMax)
    return fail(FCHI2_ERR_UNSUPPORTED, "the fine search needs H <= %d", kHMax);
  if (!(half_width >= 0.0) || !std::isfinite(half_width))
    return fail(FCHI2_ERR_ARG, "half_width must be finite and >= 0");
  if (hrow < 0 || hrow >= plan->g.H) return fail(FCHI2_ERR_ARG, "hrow must be in 0..H-1");
  if (!scratch) return fail(FCHI2_ERR_ARG, "scratch is NULL");
  if (((uintptr_t)scratch & 255) != 0) return fail(FCHI2_ERR_ARG, "scratch must be 256-byte aligned");
  const size_t need = fchi2_fine_scratch_bytes(plan, K, R);
  if (scratch_bytes < need)
    return fail(FCHI2_ERR_ARG, "scratch too small: %zu < %zu bytes", scratch_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  fchi2_plan_s* pl = plan;
  const int nc = plan->desc.n_curves;
  char* sc = (char*)scratch;
  Moments* mom = (Moments*)sc;
  MomPart* part = (MomPart*)(sc + align256(sizeof(Moments) * (size_t)nc));
  double* sums = (double*)(sc + align256(sizeof(Moments) * (size_t)nc) +
                           align256(sizeof(MomPart) * (size_t)nc * plan->mom_bpc));
  PROF_BEGIN(FCHI2_PROF_MOMENTS);
  hipError_t e = launch_moments(t, x, sigma, plan->d_off, nc, plan->mom_bpc, plan->g, part, mom,
                                nullptr, st);
  if (e != hipSuccess) return hip_fail(e, "moments");
  PROF_END();
  FineOut o{out->rows, out->f_best, out->dchi2_best, out->coef, out->flags};
  PROF_BEGIN(FCHI2_PROF_FINE);
  e = launch_fine(t, x, sigma, mom, plan->g.H, nc, plan->max_n, f_center, K, R, half_width, sums,
                  hrow, o, st);
  if (e != hipSuccess) return hip_fail(e, "fine search");
  PROF_END();
  return FCHI2_OK;
}

size_t fchi2_search_multi_workspace_bytes(fchi2_plan_t plan, int32_t n_sources) {
  if (!plan || n_sources < 1 || plan->desc.n_curves != 1 || plan->g.H > 5 || plan->g.band)
    return 0;
  return multi_layout(plan, n_sources).bytes;
}

fchi2_status_t fchi2_search_multi(fchi2_plan_t plan, const double* t, const double* sigma,
                                  const double* x, const double* scale, int32_t n_sources,
                                  void* workspace, size_t workspace_bytes, void* dchi2,
                                  double* chi2_0, uint8_t* flags, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !sigma || !x || !scale || !dchi2)
    return fail(FCHI2_ERR_ARG, "t, sigma, x, scale and dchi2 must not be NULL");
  if (plan->desc.n_curves != 1)
    return fail(FCHI2_ERR_ARG, "the shared time base needs a plan of one curve");
  if (plan->g.H > 5) return fail(FCHI2_ERR_UNSUPPORTED, "shared-alpha search supports H <= 5");
  if (plan->g.band) return fail(FCHI2_ERR_UNSUPPORTED, "band plans have no shared-alpha search");
  if (n_sources < 1) return fail(FCHI2_ERR_ARG, "n_sources must be >= 1");
  if (!workspace) return fail(FCHI2_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0)
    return fail(FCHI2_ERR_ARG, "workspace must be 256-byte aligned");
  const MultiLayout m = multi_layout(plan, n_sources);
  if (workspace_bytes < m.bytes)
    return fail(FCHI2_ERR_ARG, "workspace too small: %zu < %zu bytes", workspace_bytes, m.bytes);
  plan->last_ws = nullptr;  // no backward for this form
  ++plan->gen;
  return enqueue_multi(plan, m, t, sigma, x, scale, n_sources, (char*)workspace, dchi2, chi2_0,
                       flags, (hipStream_t)stream);
}

fchi2_status_t fchi2_autotune_multi(fchi2_plan_t plan, const double* t, const double* sigma,
                                    const double* x, const double* scale, int32_t n_sources,
                                    void* workspace, size_t workspace_bytes, void* dchi2,
                                    void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !sigma || !x || !scale || !dchi2)
    return fail(FCHI2_ERR_ARG, "t, sigma, x, scale and dchi2 must not be NULL");
  if (plan->desc.n_curves != 1)
    return fail(FCHI2_ERR_ARG, "the shared time base needs a plan of one curve");
  if (plan->g.H > 5) return fail(FCHI2_ERR_UNSUPPORTED, "shared-alpha search supports H <= 5");
  if (plan->g.band) return fail(FCHI2_ERR_UNSUPPORTED, "band plans have no shared-alpha search");
  if (n_sources < 1) return fail(FCHI2_ERR_ARG, "n_sources must be >= 1");
  if (!workspace || ((uintptr_t)workspace & 255) != 0)
    return fail(FCHI2_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < multi_layout(plan, n_sources).bytes)
    return fail(FCHI2_ERR_ARG, "workspace too small");
  fchi2_plan_s* pl = plan;
  hipStream_t st = (hipStream_t)stream;
  if (pl->gexec) {
    (void)hipGraphExecDestroy(pl->gexec);
    pl->gexec = nullptr;
  }
  const std::vector<FftPlan> splits = fft_splits(pl->fp.logL, pl->fp64);
  const std::vector<int> waves = {pl->wave};
  const bool prof = pl->prof;
  pl->prof = false;
  float best_ms = 1e30f;
  TuneCand best{pl->fp, pl->log_tile, pl->wave, pl->fused, pl->persist, pl->solve_sub, 0.f};
  fchi2_status_t res = tune_loop(
      pl, splits, waves, false, false, false,
      [&]() {
        return enqueue_multi(pl, multi_layout(pl, n_sources), t, sigma, x, scale, n_sources,
                             (char*)workspace, dchi2, nullptr, nullptr, st);
      },
      st, best_ms, best);
  pl->prof = prof;
  apply_tuned(pl, best);
  pl->last_ws = nullptr;
  ++pl->gen;
  return res;
}

fchi2_status_t fchi2_detrend(fchi2_plan_t plan, const double* t, const double* x,
                             const double* sigma, int32_t degree, double* x_out, double* coef,
                             void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !x_out)
    return fail(FCHI2_ERR_ARG, "t, x, sigma and x_out must not be NULL");
  if (degree < 0 || degree > 3) return fail(FCHI2_ERR_ARG, "degree must be in 0..3");
  hipError_t e = launch_detrend(t, x, sigma, plan->d_off, plan->desc.n_curves, degree,
                                plan->max_n, x_out, coef, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "detrend");
  return FCHI2_OK;
}

fchi2_status_t fchi2_profile(fchi2_plan_t plan, int32_t enable) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  plan->prof = enable != 0;
  plan->ev_used = 0;
  plan->ev_stage.clear();
  for (int i = 0; i < FCHI2_PROF_STAGES; ++i) {
    plan->prof_ms[i] = 0.0;
    plan->prof_n[i] = 0;
  }
  return FCHI2_OK;
}

fchi2_status_t fchi2_profile_read(fchi2_plan_t plan, double* total_ms, int64_t* launches) {
  g_err.clear();
  if (!plan || !total_ms || !launches) return fail(FCHI2_ERR_ARG, "NULL argument");
  for (size_t i = 0; i < plan->ev_stage.size(); ++i) {
    hipEvent_t a = plan->ev_pool[2 * i], b = plan->ev_pool[2 * i + 1];
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    plan->prof_ms[plan->ev_stage[i]] += ms;
    plan->prof_n[plan->ev_stage[i]] += 1;
  }
  plan->ev_used = 0;
  plan->ev_stage.clear();
  for (int i = 0; i < FCHI2_PROF_STAGES; ++i) {
    total_ms[i] = plan->prof_ms[i];
    launches[i] = plan->prof_n[i];
  }
  return FCHI2_OK;
}

fchi2_status_t fchi2_autotune(fchi2_plan_t plan, const double* t, const double* x,
                              const double* sigma, void* workspace, size_t workspace_bytes,
                              void* dchi2, const char* cache_path, void* stream) {
  g_err.clear();
  if (!plan) return fail(FCHI2_ERR_ARG, "plan is NULL");
  if (!t || !x || !sigma || !dchi2) return fail(FCHI2_ERR_ARG, "NULL pointer argument");
  fchi2_status_t s = check_ws(plan, workspace, workspace_bytes);
  if (s != FCHI2_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  fchi2_plan_s* pl = plan;
  int lg_nc = 0, lg_n = 0;
  while ((1 << lg_nc) < pl->desc.n_curves) ++lg_nc;
  while (((int64_t)1 << lg_n) < pl->max_n) ++lg_n;
  char key[160];
  snprintf(key, sizeof key, "gfx950 H=%d nf=%lld prec=%d w=%d curves=2^%d maxn=2^%d wavemax=%d",
           pl->g.H, (long long)pl->g.n_freq, pl->fp64 ? 0 : 1, pl->g.w, lg_nc, lg_n,
           pl->wave_max);
  const std::vector<FftPlan> splits = fft_splits(pl->fp.logL, pl->fp64);
  auto apply = [&](const int* ln, const int* le, int np, int tile, int wave) -> bool {
    for (const FftPlan& f : splits) {
      if (f.np != np) continue;
      bool same = true;
      for (int q = 1; q <= np; ++q) same = same && f.logn[q] == ln[q] && f.le[q] == le[q];
      if (!same) continue;
      pl->log_tile = tile;
      pl->wave = wave;
      apply_fft_plan(pl, f);
      return true;
    }
    return false;
  };
  if (pl->gexec) {
    (void)hipGraphExecDestroy(pl->gexec);
    pl->gexec = nullptr;
  }
  // Cached choice?
  if (cache_path) {
    if (FILE* fh = fopen(cache_path, "r")) {
      char line[512];
      bool found = false;
      while (!found && fgets(line, sizeof line, fh)) {
        const char* tag = strstr(line, " | ");
        if (!tag || strncmp(line, key, strlen(key)) != 0 || line + strlen(key) != tag) continue;
        int np = 0, ln[kMaxPasses + 1] = {0}, le[kMaxPasses + 1] = {0}, tile = 0, wave = 0;
        // Lines without the fused / persist / sub fields name the staged
        // schedule on whole waves.
        int fz = 0, ps = 0, sb = 0;
        if (sscanf(tag,
                   " | np=%d fft=%d,%d,%d,%d le=%d,%d,%d,%d tile=%d wave=%d fused=%d persist=%d "
                   "sub=%d",
                   &np, &ln[1], &ln[2], &ln[3], &ln[4], &le[1], &le[2], &le[3], &le[4], &tile,
                   &wave, &fz, &ps, &sb) >= 11 &&
            tile >= 10 && tile <= 13 && wave >= 1 && wave <= pl->wave_max &&
            (fz == 0 || (fz == 1 && !pl->g.band)) && (ps == 0 || ps == 1) && sb >= 0 &&
            sb <= wave) {
          found = apply(ln, le, np, tile, wave);
          if (found && ps == 1 && !persist_ok(pl, pl->fp, tile)) found = false;
          if (found) {
            pl->fused = fz;
            pl->persist = ps;
            pl->solve_sub = sb;
          }
        }
      }
      fclose(fh);
      if (found) return FCHI2_OK;
    }
  }
  // Time every candidate on the caller's data.
  // Waves of wave_max, /2, /4, /6, /8, /10, /12 curves: smaller waves keep a
  // wave's spectra (and part of its grids) in the 256 MB Infinity Cache
  // between the pass that writes them and the kernel that reads them, and
  // (at most half the buffers) overlap the next wave's spreading with the
  // current wave's passes.
  std::vector<int> waves = {pl->wave_max};
  if (pl->desc.n_curves > 1)
    for (int div : {2, 4, 6, 8, 10, 12}) {
      const int w = pl->wave_max / div;
      if (w >= 1 && w != waves.back()) waves.push_back(w);
    }
  const bool prof = pl->prof;
  pl->prof = false;
  float best_ms = 1e30f;
  TuneCand best{pl->fp, pl->log_tile, pl->wave, pl->fused, pl->persist, pl->solve_sub, 0.f};
  const bool allow_fused = !pl->g.band;
  fchi2_status_t res = tune_loop(
      pl, splits, waves, allow_fused, true, pl->desc.n_curves > 1,
      [&]() {
        return enqueue_search(pl, 0, pl->desc.n_curves, t, x, sigma, (char*)workspace, dchi2,
                              nullptr, nullptr, st);
      },
      st, best_ms, best);
  pl->prof = prof;
  apply_tuned(pl, best);
  const FftPlan& best_f = best.f;
  pl->last_ws = nullptr;
  ++pl->gen;
  if (res != FCHI2_OK) return res;
  if (cache_path) {
    if (FILE* fh = fopen(cache_path, "a")) {
      fprintf(fh,
              "%s | np=%d fft=%d,%d,%d,%d le=%d,%d,%d,%d tile=%d wave=%d fused=%d persist=%d "
              "sub=%d ms=%.4f\n",
              key, best_f.np, best_f.logn[1], best_f.logn[2], best_f.logn[3], best_f.logn[4],
              best_f.le[1], best_f.le[2], best_f.le[3], best_f.le[4], best.tile, best.wave,
              best.fused, best.persist, best.sub, best_ms);
      fclose(fh);
    }
  }
  return FCHI2_OK;
}

fchi2_status_t fchi2_plan_info(fchi2_plan_t plan, int32_t* info, int32_t n) {
  g_err.clear();
  if (!plan || !info || n < 8) return fail(FCHI2_ERR_ARG, "plan/info NULL or n < 8");
  info[0] = plan->fp.np;
  for (int q = 1; q <= kMaxPasses; ++q) info[q] = plan->fp.logn[q];
  info[5] = plan->log_tile;
  info[6] = plan->wave;
  info[7] = plan->g.w;
  for (int q = 1; q <= kMaxPasses && 7 + q < n; ++q) info[7 + q] = q <= plan->fp.np ? plan->fp.le[q] : 0;
  if (n > 12) info[12] = use_fused(plan) ? 1 : 0;
  if (n > 13) info[13] = use_persist(plan) ? 1 : 0;
  if (n > 14) info[14] = plan->solve_sub;
  return FCHI2_OK;
}

fchi2_status_t fchi2_plan_set_schedule(fchi2_plan_t plan, const int32_t* info, int32_t n) {
  g_err.clear();
  if (!plan || !info || n < 14) return fail(FCHI2_ERR_ARG, "plan/info NULL or n < 14");
  fchi2_plan_s* pl = plan;
  const int np = info[0];
  const int tile = info[5], wave = info[6], fz = info[12], ps = info[13];
  if (tile < 10 || tile > 13) return fail(FCHI2_ERR_ARG, "spreading tile must be 2^10..2^13");
  if (wave < 1 || wave > pl->wave_max)
    return fail(FCHI2_ERR_ARG, "curves per wave must be in 1..%d", pl->wave_max);
  if ((fz != 0 && fz != 1) || (ps != 0 && ps != 1))
    return fail(FCHI2_ERR_ARG, "fused and persistent entries must be 0 or 1");
  if (fz == 1 && pl->g.band) return fail(FCHI2_ERR_UNSUPPORTED, "band plans are not fused");
  const FftPlan* found = nullptr;
  const std::vector<FftPlan> splits = fft_splits(pl->fp.logL, pl->fp64);
  for (const FftPlan& f : splits) {
    bool same = f.np == np;
    for (int q = 1; q <= np && same; ++q)
      same = f.logn[q] == info[q] && f.le[q] == info[7 + q];
    if (same) found = &f;
  }
  if (!found) return fail(FCHI2_ERR_UNSUPPORTED, "not one of the plan's FFT schedules");
  if (ps == 1 && !persist_ok(pl, *found, tile))
    return fail(FCHI2_ERR_UNSUPPORTED, "the persistent search does not take this schedule");
  if (pl->gexec) {
    (void)hipGraphExecDestroy(pl->gexec);
    pl->gexec = nullptr;
  }
  const int sb = n > 14 ? info[14] : 0;
  if (sb < 0 || sb > wave) return fail(FCHI2_ERR_ARG, "solve sub-wave must be in 0..wave");
  pl->log_tile = tile;
  pl->wave = wave;
  pl->fused = fz;
  pl->persist = ps;
  pl->solve_sub = sb;
  apply_fft_plan(pl, *found);
  pl->last_ws = nullptr;
  ++pl->gen;
  return FCHI2_OK;
}

void fchi2_destroy(fchi2_plan_t plan) {
  if (!plan) return;
  for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
  if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
  if (plan->d_off) (void)hipFree(plan->d_off);
  if (plan->d_tw_stage) (void)hipFree(plan->d_tw_stage);
  if (plan->d_tw_small) (void)hipFree(plan->d_tw_small);
  if (plan->d_D) (void)hipFree(plan->d_D);
  if (plan->d_gl) (void)hipFree(plan->d_gl);
  for (hipEvent_t e : {plan->ev_start, plan->ev_spread[0], plan->ev_spread[1], plan->ev_first[0],
                       plan->ev_first[1]})
    if (e) (void)hipEventDestroy(e);
  if (plan->side) (void)hipStreamDestroy(plan->side);
  delete plan;
}

}  // extern "C"
