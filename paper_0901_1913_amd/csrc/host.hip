// C ABI host layer: argument checks, plan geometry, device tables, workspace
// layout and the launch sequence of the search and its adjoint.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fchi2.h"
#include "fchi2_internal.h"
#include "launch.h"

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

// Choose the FFT digit split of L = 2^logL into np passes of radix <= 2^10.
// Constraints: each pass tile holds 2^LE elements as N_q rows x T columns and
// the T columns of one tile must share their other digits.
bool plan_fft(int logL, int LE, FftPlan& fp) {
  if (logL <= LE) {
    if (logL < 12) return false;
    fp.np = 1;
    fp.logn[1] = logL;
    fp.logL = logL;
    return true;
  }
  for (int np = 2; np <= kMaxPasses; ++np) {
    int best_min = -1;
    int best[kMaxPasses + 1] = {0};
    int ln[kMaxPasses + 1];
    // Enumerate compositions of logL into np parts in [4, 10].
    const int lo = 4, hi = 10;
    int total = 1;
    for (int q = 0; q < np; ++q) total *= (hi - lo + 1);
    for (int code = 0; code < total; ++code) {
      int c = code, sum = 0, mn = 99;
      for (int q = 1; q <= np; ++q) {
        ln[q] = lo + c % (hi - lo + 1);
        c /= (hi - lo + 1);
        sum += ln[q];
        mn = ln[q] < mn ? ln[q] : mn;
      }
      if (sum != logL) continue;
      bool ok = true;
      // PASS_FIRST (digit np): T = 2^(LE - ln[np]) columns within digit 1.
      if (LE - ln[np] > ln[1]) ok = false;
      // PASS_MID (digit q): T <= Tail_q = prod_{d > q} N_d.
      for (int q = 2; q < np && ok; ++q) {
        int tail = 0;
        for (int d = q + 1; d <= np; ++d) tail += ln[d];
        if (LE - ln[q] > tail) ok = false;
      }
      // PASS_LAST: T <= L / N_1.
      if (LE - ln[1] > logL - ln[1]) ok = false;
      for (int q = 1; q <= np; ++q)
        if (LE - ln[q] < 0) ok = false;
      if (!ok) continue;
      if (mn > best_min) {
        best_min = mn;
        for (int q = 1; q <= np; ++q) best[q] = ln[q];
      }
    }
    if (best_min >= 0) {
      fp.np = np;
      for (int q = 1; q <= np; ++q) fp.logn[q] = best[q];
      fp.logL = logL;
      return true;
    }
  }
  return false;
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
  int tw_s = 0;
  int log_tile = 10;
  double eps_piv = 0.0;
  int wave = 1;
  int64_t n_total = 0;
  // plan-owned device tables
  int64_t* d_off = nullptr;
  void* d_tw_stage = nullptr;
  void* d_tw_lo = nullptr;
  void* d_tw_hi = nullptr;
  void* d_D = nullptr;
  double* d_gl = nullptr;
  // workspace layout (byte offsets)
  size_t off_mom = 0, off_gA = 0, off_gB = 0, off_zc = 0, off_gq = 0, off_gp = 0, off_dw = 0;
  size_t ws_bytes = 0;
  int blocks_per_curve = 0;
  // graph replay
  hipGraphExec_t gexec = nullptr;
  const void* gkey[8] = {nullptr};
  size_t gkey_ws = 0;
  // backward needs a search on this workspace first
  const void* last_ws = nullptr;
};

namespace {

fchi2_status_t enqueue_fft(fchi2_plan_s* pl, int mode, void* gA, void* gB, void* zc,
                           const Moments* mom, int curve0, int nw, hipStream_t st) {
  const FftPlan& fp = pl->fp;
  const int LE = fft_tile_log(pl->fp64);
  FftPassArgs a{};
  a.mode = mode;
  a.np = fp.np;
  for (int q = 0; q <= kMaxPasses; ++q) a.logn[q] = fp.logn[q];
  a.logL = fp.logL;
  a.tw_s = pl->tw_s;
  a.curve0 = curve0;
  a.zc = zc;
  a.grid_out = gA;
  if (fp.np == 1) {
    a.kind = PASS_SINGLE;
    a.q = 1;
    hipError_t e = launch_fft_pass(pl->fp64, a, fp.logL, 0, gA, gA, mom, pl->g, pl->d_tw_stage,
                                   pl->d_tw_lo, pl->d_tw_hi, nw, 1, st);
    if (e != hipSuccess) return hip_fail(e, "fft single pass");
    return FCHI2_OK;
  }
  for (int q = fp.np; q >= 1; --q) {
    a.q = q;
    a.kind = (q == fp.np) ? PASS_FIRST : (q == 1 ? PASS_LAST : PASS_MID);
    const int logn = fp.logn[q];
    const int logt = LE - logn;
    const int64_t ncols = pl->g.L >> logn;
    const void* in = (q == fp.np) ? gA : gB;
    void* out = gB;
    hipError_t e = launch_fft_pass(pl->fp64, a, logn, logt, in, out, mom, pl->g, pl->d_tw_stage,
                                   pl->d_tw_lo, pl->d_tw_hi, nw, ncols, st);
    if (e != hipSuccess) return hip_fail(e, "fft pass");
  }
  return FCHI2_OK;
}

fchi2_status_t enqueue_search(fchi2_plan_s* pl, const double* t, const double* x,
                              const double* sigma, char* ws, void* dchi2, double* chi2_0,
                              uint8_t* flags, hipStream_t st) {
  Moments* mom = (Moments*)(ws + pl->off_mom);
  hipError_t e = launch_moments(t, x, sigma, pl->d_off, pl->desc.n_curves, pl->g, mom, chi2_0, st);
  if (e != hipSuccess) return hip_fail(e, "moments");
  const bool keep = pl->desc.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)pl->g.P * 2 * pl->g.n_freq * pl->elem;
  for (int c0 = 0; c0 < pl->desc.n_curves; c0 += pl->wave) {
    const int nw = (pl->desc.n_curves - c0) < pl->wave ? (pl->desc.n_curves - c0) : pl->wave;
    void* gA = ws + pl->off_gA;
    void* gB = ws + pl->off_gB;
    void* zc = ws + pl->off_zc + (keep ? (size_t)c0 * zc_curve : 0);
    e = launch_spread(pl->fp64, t, x, sigma, mom, pl->g, c0, nw, gA, pl->log_tile, st);
    if (e != hipSuccess) return hip_fail(e, "spread");
    fchi2_status_t s = enqueue_fft(pl, MODE_FWD, gA, gB, zc, mom, c0, nw, st);
    if (s != FCHI2_OK) return s;
    e = launch_solve(pl->fp64, zc, pl->d_D, mom, pl->g, c0, nw, pl->eps_piv, dchi2, flags, st);
    if (e != hipSuccess) return hip_fail(e, "solve");
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
  if (!is_pow2(d.n_freq)) return fail(FCHI2_ERR_ARG, "n_freq must be a power of two");
  if (d.n_freq < (1 << 10) || d.n_freq > (1 << 24))
    return fail(FCHI2_ERR_UNSUPPORTED, "n_freq must be in 2^10..2^24");
  if (d.precision != FCHI2_FP64 && d.precision != FCHI2_MIXED)
    return fail(FCHI2_ERR_ARG, "precision must be FCHI2_FP64 or FCHI2_MIXED");
  if (d.flags & ~(uint32_t)(FCHI2_KEEP_FOR_BACKWARD | FCHI2_GRAPH))
    return fail(FCHI2_ERR_ARG, "unknown flag bits 0x%x", d.flags);
  if (d.kernel_width != 0 && (d.kernel_width < 4 || d.kernel_width > 16))
    return fail(FCHI2_ERR_ARG, "kernel_width must be 0 or 4..16");
  if (d.curves_per_wave < 0) return fail(FCHI2_ERR_ARG, "curves_per_wave must be >= 0");

  fchi2_plan_s* pl = new fchi2_plan_s();
  pl->desc = d;
  pl->offsets.assign(d.offsets, d.offsets + d.n_curves + 1);
  pl->desc.offsets = pl->offsets.data();
  pl->n_total = pl->offsets.back();
  pl->fp64 = (d.precision == FCHI2_FP64);
  pl->elem = pl->fp64 ? 16 : 8;
  pl->out_elem = pl->fp64 ? 8 : 4;
  pl->eps_piv = pl->fp64 ? 1e-13 : 1e-6;

  Geom& g = pl->g;
  g.n_freq = d.n_freq;
  g.L = 4 * d.n_freq;
  g.df = d.f_max / (double)d.n_freq;
  g.w = d.kernel_width ? d.kernel_width : (pl->fp64 ? 14 : 8);
  g.half_w = 0.5 * g.w;
  g.beta = 2.30 * g.w;
  g.c_off = g.w / 2 + 2;
  g.H = d.H;
  g.P = d.H + (d.H + 1) / 2;
  std::memset(g.comp_m, 0, sizeof g.comp_m);
  std::memset(g.comp_kind, 0, sizeof g.comp_kind);
  // Like is packed with like, so each FFT's rounding noise scales with the
  // norm of grids of the same kind: pairs p < H hold the weight grids
  // (q_{2p+1}, q_{2p+2}); pairs p >= H hold the weighted-data grids
  // (p_{2j+1}, p_{2j+2}), j = p - H, the second part empty past H.
  for (int p = 0; p < g.P; ++p) {
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
  if (!plan_fft(logL, fft_tile_log(pl->fp64), pl->fp)) {
    delete pl;
    return fail(FCHI2_ERR_UNSUPPORTED, "no FFT pass split for L = 2^%d", logL);
  }
  pl->tw_s = (logL + 1) / 2;
  pl->log_tile = 10;
  const int64_t S_first = (pl->fp.np == 1) ? 1 : (g.L >> pl->fp.logn[pl->fp.np]);
  const int64_t tile = (int64_t)1 << pl->log_tile;
  g.chunk = (int)(S_first > tile ? S_first : tile);

  // Waves: bound the two grid buffers to ~8 GiB unless the caller chose.
  const size_t grid_curve = (size_t)g.P * (size_t)g.L * pl->elem;
  if (d.curves_per_wave > 0) {
    pl->wave = d.curves_per_wave < d.n_curves ? d.curves_per_wave : d.n_curves;
  } else {
    size_t cap = ((size_t)8 << 30) / (2 * grid_curve);
    if (cap < 1) cap = 1;
    pl->wave = (int)(cap < (size_t)d.n_curves ? cap : (size_t)d.n_curves);
  }
  const bool keep = d.flags & FCHI2_KEEP_FOR_BACKWARD;
  const size_t zc_curve = (size_t)g.P * 2 * (size_t)g.n_freq * pl->elem;
  pl->blocks_per_curve = (int)((g.n_freq + 255) / 256);
  size_t off = 0;
  pl->off_mom = off;
  off = align256(off + sizeof(Moments) * (size_t)d.n_curves);
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
  pl->ws_bytes = off;

  // Device tables.
  hipStream_t st = (hipStream_t)stream;
  auto cleanup_fail = [&](fchi2_status_t s) {
    fchi2_destroy(pl);
    return s;
  };
  auto dev_alloc = [&](void** p, size_t bytes) -> bool {
    return hipMalloc(p, bytes) == hipSuccess;
  };
  const int LT = 1 << kStageLog;
  const int64_t nlo = (int64_t)1 << pl->tw_s, nhi = g.L >> pl->tw_s;
  const int n_gl = 128;
  if (!dev_alloc((void**)&pl->d_off, sizeof(int64_t) * (d.n_curves + 1)) ||
      !dev_alloc(&pl->d_tw_stage, pl->elem * LT) || !dev_alloc(&pl->d_tw_lo, pl->elem * nlo) ||
      !dev_alloc(&pl->d_tw_hi, pl->elem * nhi) || !dev_alloc(&pl->d_D, pl->elem * g.n_freq) ||
      !dev_alloc((void**)&pl->d_gl, sizeof(double) * n_gl)) {
    (void)hipGetLastError();
    return cleanup_fail(fail(FCHI2_ERR_NOMEM, "plan table allocation failed"));
  }
  std::vector<char> hs(pl->elem * LT), hl(pl->elem * nlo), hh(pl->elem * nhi);
  auto put = [&](std::vector<char>& v, int64_t i, double re, double im) {
    if (pl->fp64) {
      double* p = (double*)v.data();
      p[2 * i] = re;
      p[2 * i + 1] = im;
    } else {
      float* p = (float*)v.data();
      p[2 * i] = (float)re;
      p[2 * i + 1] = (float)im;
    }
  };
  auto root = [](int64_t e, int64_t n, double& re, double& im) {
    // exp(+2 pi i e / n) with the angle reduced to the first octant.
    const long double ang = 2.0L * (long double)M_PI * (long double)(e % n) / (long double)n;
    re = (double)std::cos(ang);
    im = (double)std::sin(ang);
  };
  double re, im;
  for (int64_t e = 0; e < LT; ++e) {
    root(e, LT, re, im);
    put(hs, e, re, im);
  }
  for (int64_t e = 0; e < nlo; ++e) {
    root(e, g.L, re, im);
    put(hl, e, re, im);
  }
  for (int64_t e = 0; e < nhi; ++e) {
    root(e << pl->tw_s, g.L, re, im);
    put(hh, e, re, im);
  }
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
      (e = hipMemcpyAsync(pl->d_tw_stage, hs.data(), hs.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->d_tw_lo, hl.data(), hl.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->d_tw_hi, hh.data(), hh.size(), hipMemcpyHostToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(pl->d_gl, gl.data(), sizeof(double) * n_gl, hipMemcpyHostToDevice,
                          st)) != hipSuccess ||
      (e = launch_deconv_init(pl->fp64, pl->d_D, g, pl->d_gl, pl->d_gl + n_gl / 2, n_gl / 2,
                              st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess) {
    return cleanup_fail(hip_fail(e, "plan table setup"));
  }
  *out = pl;
  return FCHI2_OK;
}

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

  if ((plan->desc.flags & FCHI2_GRAPH) && st != nullptr) {
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
        fchi2_status_t es = enqueue_search(plan, t, x, sigma, ws, dchi2, chi2_0, flags, st);
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
  return enqueue_search(plan, t, x, sigma, ws, dchi2, chi2_0, flags, st);
}

fchi2_status_t fchi2_backward(fchi2_plan_t plan, const double* t, const double* x,
                              const double* sigma, const void* grad_dchi2, void* workspace,
                              size_t workspace_bytes, double* grad_x, double* grad_sigma,
                              void* stream) {
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
  hipStream_t st = (hipStream_t)stream;
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
    hipError_t e = launch_adjoint_solve(plan->fp64, zc, plan->d_D, mom, plan->g, c0, nw,
                                        plan->eps_piv, grad_dchi2, gA, dw,
                                        plan->blocks_per_curve, st);
    if (e != hipSuccess) return hip_fail(e, "adjoint solve");
    s = enqueue_fft(plan, MODE_BWD, gA, gB, nullptr, mom, c0, nw, st);
    if (s != FCHI2_OK) return s;
    int64_t max_n = 0;
    for (int c = c0; c < c0 + nw; ++c) {
      const int64_t n = plan->offsets[c + 1] - plan->offsets[c];
      max_n = n > max_n ? n : max_n;
    }
    e = launch_gather(plan->fp64, t, mom, plan->g, c0, nw, gA, gq, gp, max_n, st);
    if (e != hipSuccess) return hip_fail(e, "gather");
    e = launch_finalize(x, sigma, mom, plan->g, c0, nw, dw, plan->blocks_per_curve, gq, gp,
                        grad_x, grad_sigma, st);
    if (e != hipSuccess) return hip_fail(e, "finalize");
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

void fchi2_destroy(fchi2_plan_t plan) {
  if (!plan) return;
  if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
  if (plan->d_off) (void)hipFree(plan->d_off);
  if (plan->d_tw_stage) (void)hipFree(plan->d_tw_stage);
  if (plan->d_tw_lo) (void)hipFree(plan->d_tw_lo);
  if (plan->d_tw_hi) (void)hipFree(plan->d_tw_hi);
  if (plan->d_D) hipFree(plan->d_D);
  if (plan->d_gl) (void)hipFree(plan->d_gl);
  delete plan;
}

}  // extern "C"
