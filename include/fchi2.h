/*
 * fchi2.h - C ABI of the MI355X (gfx950) F-chi2 period-search library.
 *
 * The library computes, for irregularly sampled data (t_i, x_i, sigma_i), the
 * chi2 reduction obtained by fitting a Fourier series truncated at H'
 * harmonics (Palmer, Fast chi2 period search, eq. eqtrunc and eq. eqchigen),
 * minimised over its 2H'+1 linear coefficients at every trial frequency of a
 * dense grid, for every H' = 1..H at once (Section 1: evaluations for several
 * H share their stages):
 *
 *   Delta chi2(f_k, H') = chi2_0 - min_A sum_i w_i (x_i - Phi_H'(A, f_k, t_i))^2
 *                       = beta^T alpha^-1 beta                      (eq. eqchix)
 *
 * with w_i = sigma_i^-2, chi2_0 = sum_i w_i (x_i - xbar)^2, xbar the weighted
 * mean (Section 3b and 3d), f_k = k * f_max / n_freq for k = 0..n_freq-1.
 * alpha and beta are built from the transforms P(f), Q(f) of the weighted data
 * and the weights (eq. eqPQ) by product-to-sum identities (Section 2), the
 * transforms are computed with FFTs (Section 3b), and the normal equations are
 * solved per frequency (Section 3c, 3d).
 *
 * Conventions for every entry point:
 *  - Pointers named "device" point to GPU memory on the current HIP device;
 *    "host" pointers to host memory.  The caller owns every buffer; the
 *    library never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it; no call synchronises the stream, except
 *    fchi2_plan, which initialises plan tables and returns after they are
 *    ready.
 *  - fchi2_search(_curves), fchi2_backward, fchi2_top_peaks,
 *    fchi2_search_top, fchi2_fine_search, fchi2_search_multi and
 *    fchi2_detrend allocate no memory and make no blocking call, so they may
 *    be captured in a HIP graph (fchi2_autotune and fchi2_autotune_multi
 *    synchronise).
 *  - Errors are reported by the return code only (no exceptions, no abort);
 *    fchi2_last_error() gives a message for the calling thread.  Argument
 *    errors are detected on the host before any device work is enqueued.
 *  - Per-curve data errors (non-finite values, sigma <= 0, unsorted t, an
 *    empty curve, or a span too long for the frequency grid) do not fail the
 *    call: that curve's outputs become NaN and its flag bytes carry the
 *    FCHI2_CURVE_* bits; other curves are unaffected.
 *  - A plan must not be used by two threads at once.
 */
#ifndef FCHI2_H_
#define FCHI2_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fchi2_plan_s* fchi2_plan_t;

typedef enum {
  FCHI2_OK = 0,
  FCHI2_ERR_ARG = 1,          /* invalid argument (message says which)       */
  FCHI2_ERR_NOMEM = 2,        /* plan tables: out of device memory           */
  FCHI2_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed  */
  FCHI2_ERR_STATE = 4,        /* call not valid for this plan's flags/state  */
  FCHI2_ERR_UNSUPPORTED = 5   /* size or parameter outside what is built     */
} fchi2_status_t;

typedef enum {
  FCHI2_FP64 = 0,   /* FP64 spreading, FFT, assembly and solve                */
  FCHI2_MIXED = 1   /* FP64 arithmetic (the spreading kernel's exponential to
                       FP32 accuracy); grids, spectra and the Delta chi2
                       output stored in FP32 (FP32 HBM traffic)              */
} fchi2_precision_t;

/* Plan flags. */
#define FCHI2_KEEP_FOR_BACKWARD 1u /* keep all spectra in the workspace      */
#define FCHI2_GRAPH 2u             /* replay searches through a HIP graph    */
#define FCHI2_WIDE_SOLVE 8u        /* solve every bin with the wave-per-bin
                                      solver (automatic for H > 8); same
                                      results as the register solver; no
                                      backward or band plans                 */
#define FCHI2_FUSED_SPREAD 4u      /* spread inside the first FFT pass's
                                      tiles (no spread grid in memory); the
                                      results are the same bit for bit; the
                                      autotuner may change it; not for band
                                      plans                                  */
#define FCHI2_TWO_STREAMS 32u      /* allow the overlapped wave schedule:
                                      the plan creates a second stream
                                      (default priority) on which the next
                                      wave's spreading runs beside the
                                      current wave's passes, joined back
                                      into the caller's stream by events
                                      (stream order and graph capture are
                                      kept; the same results bit for bit).
                                      Without it all work is on the
                                      caller's stream                     */
#define FCHI2_PERSISTENT 16u       /* search all curves in one persistent
                                      launch: workgroups claim curves from a
                                      device work queue and run each curve's
                                      whole chain in a workspace slot; the
                                      results are the same bit for bit; used
                                      where the schedule allows it (MIXED,
                                      H <= 8, no band, no backward, L =
                                      4 n_freq <= 2^20, FFT passes of
                                      2^12-element tiles with 2^5..2^9 rows,
                                      spreading tiles of 2^10 or 2^11 cells),
                                      else ignored; the autotuner may change
                                      it, and times it itself only for
                                      batches with at least as many curves
                                      as workgroups resident on the device  */

/* Largest H supported by the search (fchi2_search, _curves, _coeffs,
 * _noalloc, fchi2_autotune, fchi2_top_peaks).  Up to 8 the per-bin solve
 * keeps the whole Cholesky factor in one thread's registers; from 9 to 16 a
 * wave solves each bin with the matrix rows spread over its lanes.  Backward,
 * the significance epilogue, the fine search and band plans need H <= 8
 * (FCHI2_ERR_UNSUPPORTED otherwise); the shared-alpha search H <= 5. */
#define FCHI2_H_MAX 16

/* Per-bin flag bits (flags output of fchi2_search). */
#define FCHI2_BIN_PIVOT 1u   /* a pivot of the normal matrix was dropped      */
#define FCHI2_BIN_LOW_F 2u   /* f_k < 1 / span (variability, not periodicity) */
#define FCHI2_BIN_DC 4u      /* k = 0; Delta chi2 is defined as 0             */
/* Per-curve bits (set in every flag byte of a rejected curve). */
#define FCHI2_CURVE_NONFINITE 8u   /* non-finite t/x/sigma or sigma <= 0     */
#define FCHI2_CURVE_UNSORTED 16u   /* t not ascending within the curve       */
#define FCHI2_CURVE_WRAP 32u       /* harmonic phase wraps more periods than
                                      the plan covers (see fchi2_plan)      */
#define FCHI2_CURVE_FEW 64u        /* fewer than 2H+1 points (not fatal)     */
#define FCHI2_CURVE_EMPTY 128u     /* no points                               */

typedef struct {
  int32_t n_curves;          /* >= 1                                          */
  const int64_t* offsets;    /* host, n_curves+1 CSR offsets into t/x/sigma,
                                offsets[0] = 0, nondecreasing; copied by
                                fchi2_plan                                     */
  double f_max;              /* > 0: bins f_k = k f_max / n_freq, k < n_freq  */
  int32_t H;                 /* 1 .. FCHI2_H_MAX                              */
  int64_t n_freq;            /* power of two, 2^10 .. 2^24; or 0: chosen by
                                fchi2_auto_n_freq(H, f_max, oversampling,
                                max t_span) (see below)                       */
  int32_t precision;         /* fchi2_precision_t                             */
  uint32_t flags;            /* FCHI2_KEEP_FOR_BACKWARD | FCHI2_GRAPH |
                                FCHI2_FUSED_SPREAD | FCHI2_WIDE_SOLVE |
                                FCHI2_PERSISTENT | FCHI2_TWO_STREAMS          */
  int32_t kernel_width;      /* spreading kernel taps, 0 = default
                                (14 for FP64, 10 for MIXED); 4..16; or 1 =
                                floor gridding as printed in Section 3b (each
                                time replaced by the start of its cell of
                                width 1/(4 n_freq df), no kernel, no
                                deconvolution; reproduces the paper's
                                sensitivity loss; no backward)                */
  int32_t curves_per_wave;   /* curves transformed together; 0 = automatic   */
  int64_t first_bin;         /* k0 >= 0: the plan searches the band of bins
                                f = (k0 + k) f_max / n_freq, k < n_freq (one
                                share of a search split by frequency band
                                over several devices).  0 = the ordinary
                                search from f = 0.  k0 > 0 multiplies every
                                point's strengths by exp(+2 pi i kc m u) (kc =
                                k0 + n_freq/2 the band's middle bin, u =
                                df (t - T0), FP64 phase) and gives each
                                harmonic its own complex grid of 2 n_freq
                                cells centred on the band (as many grid
                                elements as the packed real grids of the
                                ordinary search; n_freq >= 2^11); such plans
                                support fchi2_search, fchi2_search_curves,
                                fchi2_autotune and fchi2_search_top (ln p
                                with the bin index k0 + k of the search; idx,
                                chi2_best and dchi2_adj per band; the bin
                                beyond each end of the band is solved too, so
                                the band's first and last bins are ranked), not
                                backward, shared alpha or floor gridding      */
  double oversampling;       /* os for n_freq = 0 (0 = default 5); > 0       */
  const double* t_span;      /* host [n_curves]: each curve's time span
                                (last minus first time), or NULL; required
                                when n_freq = 0.  Also sizes the tables for
                                phases that wrap around the grid (below)      */
} fchi2_plan_desc_t;

/*
 * Trial-grid size rule used when fchi2_plan_desc_t.n_freq is 0 (Section 3a:
 * the bin spacing must be finer than 1/(H * span) to resolve the H-th
 * harmonic's phase over the span, and f_max is the highest frequency of
 * interest; Section 3b sizes the arrays from the span):
 *     n_freq = next power of two >= ceil(os * H * span * f_max),
 * at least 2^10.  os = 5 reproduces the grids of the plain (span 100, H 3,
 * f_max 10: 2^14) and long-curve (span 3000, H 5, f_max 50: 2^22)
 * workloads; os >= 2 keeps 2H * span * f_max / n_freq <= 1 (no wrap of
 * the harmonic phase within one grid period).  Pure host function.
 * Returns 0 for non-finite or non-positive arguments, H outside
 * 1..FCHI2_H_MAX, or a result above 2^24.
 */
int64_t fchi2_auto_n_freq(int32_t H, double f_max, double oversampling, double span);

/*
 * Create a plan.  Validates `desc`, derives the grid geometry (grid length
 * L = 4 n_freq cells per harmonic grid, 2 n_freq in a band plan; Section 3b's
 * zero-padded arrays), the FFT pass split and the spreading kernel, and
 * builds its device tables (twiddles, deconvolution) on `stream`, waiting for
 * them.  Allocates device memory for those tables (owned by the plan); a
 * plan of several curves with FCHI2_TWO_STREAMS (not a band plan) also
 * creates a second stream of default priority and a few events (owned by the
 * plan) for the overlapped wave schedule of fchi2_search.  On success *out receives the plan.
 * The grids are periodic: when 2H * span * f_max / n_freq exceeds 1 the
 * harmonic phases wrap around them, which is handled (the transforms at
 * integer bins are unchanged by whole periods); the tile tables cover enough
 * periods for the longest span in t_span (up to 8), or 2 periods when t_span
 * is NULL; a curve needing more is flagged FCHI2_CURVE_WRAP.
 * Errors: FCHI2_ERR_ARG (bad desc or NULL out), FCHI2_ERR_UNSUPPORTED,
 * FCHI2_ERR_NOMEM, FCHI2_ERR_HIP.
 */
fchi2_status_t fchi2_plan(const fchi2_plan_desc_t* desc, void* stream, fchi2_plan_t* out);

/* Bins per curve of the plan (the derived value when desc.n_freq was 0; 0 for NULL). */
int64_t fchi2_plan_n_freq(fchi2_plan_t plan);

/* Bytes of device workspace fchi2_search / fchi2_backward need (0 for NULL). */
size_t fchi2_workspace_bytes(fchi2_plan_t plan);

/* Total number of points (offsets[n_curves]) of the plan. */
int64_t fchi2_total_points(fchi2_plan_t plan);

/*
 * Delta chi2 for all curves, bins and H' = 1..H (Sections 3b-3d).
 *  t, x, sigma  device FP64 [n_total] in the plan's CSR layout; t ascending
 *               within each curve (unsorted curves are flagged)
 *  workspace    device, >= fchi2_workspace_bytes(plan) bytes, 256-byte
 *               aligned; its contents are overwritten (and, with
 *               FCHI2_KEEP_FOR_BACKWARD, read by fchi2_backward)
 *  dchi2        device [n_curves][H][n_freq], row h holds H' = h + 1;
 *               double for FCHI2_FP64, float for FCHI2_MIXED
 *  chi2_0       device FP64 [n_curves] or NULL
 *  flags        device uint8 [n_curves][n_freq] (FCHI2_BIN_* / FCHI2_CURVE_*)
 *               or NULL
 * All work is enqueued on `stream`, except with FCHI2_TWO_STREAMS and waves
 * of at most half the buffers' capacity (a tuned or set schedule): then the
 * spreading of the next wave runs on the plan's second stream while `stream`
 * runs the current wave's FFT passes and solve; the two are ordered by
 * events and all of it is joined back into `stream` (stream order and graph
 * capture behave as for one stream).  The results are the same bit for bit.
 * Errors: FCHI2_ERR_ARG (NULL plan/pointer, misaligned or small workspace),
 * FCHI2_ERR_HIP.
 */
fchi2_status_t fchi2_search(fchi2_plan_t plan, const double* t, const double* x,
                            const double* sigma, void* workspace, size_t workspace_bytes,
                            void* dchi2, double* chi2_0, uint8_t* flags, void* stream);

/*
 * fchi2_search without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The workspace is a device array of
 * FCHI2_NOALLOC_SCRATCH_BYTES inside the library (each device the library
 * runs on holds one until the process ends); this call allocates nothing,
 * makes no blocking call and never replays a graph itself (it may be
 * captured).  Outputs and their layout are those of fchi2_search, bit for
 * bit.  Every call on one device shares that device's array: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  Leaves no state for fchi2_backward.
 * Errors: FCHI2_ERR_ARG (NULL, or fchi2_workspace_bytes(plan) above
 * FCHI2_NOALLOC_SCRATCH_BYTES: plan fewer curves per wave or fewer bins),
 * FCHI2_ERR_STATE (profiling on), FCHI2_ERR_HIP.
 */
#define FCHI2_NOALLOC_SCRATCH_BYTES (64u << 20) /* 64 MiB per device */
fchi2_status_t fchi2_search_noalloc(fchi2_plan_t plan, const double* t, const double* x,
                                    const double* sigma, void* dchi2, double* chi2_0,
                                    uint8_t* flags, void* stream);

/*
 * fchi2_search that also returns, at every bin, the coefficients of the
 * H-harmonic fit (eq. eqcoeffs: A = alpha^-1 beta; Section 3d notes they are
 * an intermediate result of the solve), with the weighted mean added back to
 * A_0 (Section 3b's centring), so that the model is
 *   x(t) = A_0 + sum_h A_{2h-1} sin(2 pi h f (t - T0)) + A_{2h} cos(2 pi h f (t - T0)),
 * T0 the curve's first time and f = f_k (sign of Section 2's transforms).
 *  coeffs  device [n_curves][2H+1][n_freq], float (MIXED) | double (FP64)
 * A dropped pivot leaves its coefficient at 0; bin 0 gives A_0 = xbar and
 * zeros; a rejected curve gives NaN.  Other arguments as fchi2_search (never
 * replayed through a graph); leaves the state fchi2_backward reads.
 * Errors: as fchi2_search.
 */
fchi2_status_t fchi2_search_coeffs(fchi2_plan_t plan, const double* t, const double* x,
                                   const double* sigma, void* workspace, size_t workspace_bytes,
                                   void* dchi2, double* chi2_0, uint8_t* flags, void* coeffs,
                                   void* stream);

/*
 * fchi2_search restricted to curves [first, first + count) of the plan: the
 * same kernels over fewer curves (count = 1 is the plain single-curve form).
 * Arguments and layouts are those of fchi2_search (full-size arrays; only the
 * rows of the selected curves are written).  Never replayed through a graph.
 * A search over a strict subset leaves no state for fchi2_backward.
 * Errors: as fchi2_search, and FCHI2_ERR_ARG for a range outside the plan.
 */
fchi2_status_t fchi2_search_curves(fchi2_plan_t plan, int32_t first, int32_t count,
                                   const double* t, const double* x, const double* sigma,
                                   void* workspace, size_t workspace_bytes, void* dchi2,
                                   double* chi2_0, uint8_t* flags, void* stream);

/*
 * Gradient of a scalar loss through Delta chi2 (adjoint of the whole chain:
 * solve, assembly, deconvolution, FFT and spreading, then the weighted mean;
 * derived from eq. eqchigen and eq. eqchix).
 *  grad_dchi2   device, same layout and type as dchi2 of fchi2_search:
 *               dLoss/dDelta chi2(k, H')
 *  grad_x       device FP64 [n_total]: dLoss/dx_i (overwritten)
 *  grad_sigma   device FP64 [n_total]: dLoss/dsigma_i (overwritten)
 * The plan must have FCHI2_KEEP_FOR_BACKWARD and fchi2_search must have run
 * on the same inputs and workspace (else FCHI2_ERR_STATE).  Rejected curves
 * get NaN gradients.
 */
fchi2_status_t fchi2_backward(fchi2_plan_t plan, const double* t, const double* x,
                              const double* sigma, const void* grad_dchi2, void* workspace,
                              size_t workspace_bytes, double* grad_x, double* grad_sigma,
                              void* stream);

/*
 * Number of searches enqueued on the plan so far (fchi2_search,
 * fchi2_search_curves, fchi2_search_top, fchi2_search_multi and the
 * autotuners each count one).  The workspace state fchi2_backward reads
 * belongs to the most recent one; a caller that runs several searches on one
 * plan records this value right after the forward it will differentiate.
 * Returns 0 for NULL.
 */
uint64_t fchi2_search_generation(fchi2_plan_t plan);

/*
 * fchi2_backward for the search whose generation (fchi2_search_generation
 * right after it) is `generation`: returns FCHI2_ERR_STATE, with no device
 * work, if any other search has run on the plan since, so a gradient is never
 * taken from another forward's spectra.  Arguments otherwise as
 * fchi2_backward (which is this call with the current generation).
 */
fchi2_status_t fchi2_backward_at(fchi2_plan_t plan, uint64_t generation, const double* t,
                                 const double* x, const double* sigma, const void* grad_dchi2,
                                 void* workspace, size_t workspace_bytes, double* grad_x,
                                 double* grad_sigma, void* stream);

/*
 * Indices of the K largest strict local maxima of row `hrow` (H' = hrow + 1)
 * of each curve's Delta chi2 (the best frequencies, Section 3e): bins k in
 * [k_lo, n_freq - 2] with D[k] > D[k-1] and D[k] >= D[k+1], ordered by value,
 * ties to the lower k; missing entries are -1.
 *  dchi2     device, as written by fchi2_search
 *  scratch   device, >= fchi2_top_peaks_scratch_bytes(plan, K) bytes
 *  out_idx   device int64 [n_curves][K]
 * Errors: FCHI2_ERR_ARG (K outside 1..64, bad hrow or k_lo, NULL), FCHI2_ERR_HIP.
 */
size_t fchi2_top_peaks_scratch_bytes(fchi2_plan_t plan, int32_t K);
fchi2_status_t fchi2_top_peaks(fchi2_plan_t plan, const void* dchi2, int32_t hrow, int64_t k_lo,
                               int32_t K, void* scratch, size_t scratch_bytes, int64_t* out_idx,
                               void* stream);

/*
 * Significance epilogue (Section 3e), fused with the per-bin solve: runs the
 * whole search but, instead of writing the Delta chi2 rows, keeps per curve
 * the K candidate bins with the smallest
 *     ln p(f_k) = ln k + ln Q(Delta chi2(k, H') | 2H'),   H' = hrow + 1,
 * Q being the upper tail of the chi2 distribution with 2H' degrees of freedom
 * (the number of trials so far is taken proportional to f, hence to k).
 * Candidates are the strict local maxima D[k] > D[k-1], D[k] >= D[k+1] of row
 * hrow over the eligible bins: k >= max(k_lo, 1), f_k >= 1/span (no
 * FCHI2_BIN_LOW_F flag) and k <= n_freq - 2; ties in ln p go to the lower k.
 * Band plans (first_bin > 0) also solve the bin before their first and the
 * bin after their last, so there every bin k >= k_lo is eligible, the first
 * and last compared with those outside neighbours.  The Delta chi2 values are exactly those fchi2_search writes (same rounding),
 * so both select the same bins.  Also returns the adjusted reduction
 *     Delta chi2_adj = Delta chi2 * N_dof / chi2_best,
 * with chi2_best = chi2_0 - (largest Delta chi2 of row hrow over the eligible
 * bins, k up to n_freq - 1) and N_dof = n - 2H' - 1 (NaN when N_dof <= 0).
 *  out->idx        device int64 [n_curves][K]: bins, best first; -1 past the
 *                  last candidate (required)
 *  out->log_p      device FP64 [n_curves][K]: ln p; NaN past the last (required)
 *  out->dchi2      device FP64 [n_curves][K][H]: Delta chi2 for H' = 1..H at
 *                  the bin (may be NULL)
 *  out->dchi2_adj  device FP64 [n_curves][K] (may be NULL)
 *  out->flags      device u8 [n_curves][K]: FCHI2_BIN_* flags of the bin
 *                  (may be NULL)
 *  out->chi2_best  device FP64 [n_curves]; NaN if no bin is eligible (may be NULL)
 *  out->curve_flags device u8 [n_curves]: the FCHI2_CURVE_* bits of each
 *                  curve; a curve with a fatal bit has no candidates (may be NULL)
 *  chi2_0          device FP64 [n_curves] or NULL, as for fchi2_search
 *  workspace       >= fchi2_search_top_workspace_bytes(plan, K) bytes, 256-byte
 *                  aligned (the plan's workspace plus the per-wave candidate lists)
 * K is in 1..64.  Runs eagerly (no graph replay); with
 * FCHI2_KEEP_FOR_BACKWARD it leaves the state fchi2_backward needs.
 * Errors: FCHI2_ERR_ARG (NULL, K, hrow, k_lo < 0, workspace), FCHI2_ERR_HIP.
 */
typedef struct {
  int64_t* idx;
  double* log_p;
  double* dchi2;
  double* dchi2_adj;
  uint8_t* flags;
  double* chi2_best;
  uint8_t* curve_flags;
} fchi2_top_out_t;
size_t fchi2_search_top_workspace_bytes(fchi2_plan_t plan, int32_t K);
fchi2_status_t fchi2_search_top(fchi2_plan_t plan, const double* t, const double* x,
                                const double* sigma, void* workspace, size_t workspace_bytes,
                                int32_t hrow, int64_t k_lo, int32_t K, double* chi2_0,
                                const fchi2_top_out_t* out, void* stream);

/*
 * Fine search on the ungridded data (Section 3e): around K centre frequencies
 * per curve, Delta chi2 is computed directly from the points (FP64 sums of
 * w e^{+i 2 pi m f tau}, m = 1..2H, and w y e^{+i 2 pi m f tau}, m = 1..H,
 * tau = t - T0 with T0 the curve's first time) at the R trial frequencies
 *     f_r = f_center + half_width * (2 r / (R - 1) - 1),  r = 0..R-1
 * (f_center alone when R = 1), then solved as in fchi2_search (FP64, pivot
 * threshold 1e-13), whatever the plan's precision.  The best trial of row
 * hrow (largest Delta chi2, ties to the lower r) is returned with its
 * coefficients A = alpha^-1 beta of the H-harmonic model (eq. eqcoeffs; basis
 * 1, sin(2 pi h f tau), cos(2 pi h f tau), h = 1..H; xbar added back to A_0;
 * a dropped pivot leaves its coefficient at 0).  A centre that is NaN or
 * <= 0, a trial frequency <= 0 and a curve with a fatal data flag give NaN
 * outputs.  The grid of the plan is not used: only its curves, H and offsets.
 *  f_center       device FP64 [n_curves][K] (e.g. k * f_max / n_freq of the
 *                 candidates of fchi2_search_top, NaN for a missing one)
 *  out->rows      device FP64 [n_curves][K][R][H]: Delta chi2 at every trial
 *                 (may be NULL)
 *  out->f_best    device FP64 [n_curves][K] (required)
 *  out->dchi2_best device FP64 [n_curves][K][H] (required)
 *  out->coef      device FP64 [n_curves][K][2H+1] (may be NULL)
 *  out->flags     device u8 [n_curves][K]: FCHI2_BIN_PIVOT / FCHI2_BIN_LOW_F of
 *                 the best trial, or the curve's FCHI2_CURVE_* bits (may be NULL)
 *  scratch        device, >= fchi2_fine_scratch_bytes(plan, K, R) bytes,
 *                 256-byte aligned
 * K is in 1..256, R in 1..4096.  Sums over a curve's points are taken in a
 * fixed order (deterministic).
 * Errors: FCHI2_ERR_ARG (NULL, K, R, half_width, hrow, scratch), FCHI2_ERR_HIP.
 */
typedef struct {
  double* rows;
  double* f_best;
  double* dchi2_best;
  double* coef;
  uint8_t* flags;
} fchi2_fine_out_t;
size_t fchi2_fine_scratch_bytes(fchi2_plan_t plan, int32_t K, int32_t R);
fchi2_status_t fchi2_fine_search(fchi2_plan_t plan, const double* t, const double* x,
                                 const double* sigma, const double* f_center, int32_t K,
                                 int32_t R, double half_width, int32_t hrow, void* scratch,
                                 size_t scratch_bytes, const fchi2_fine_out_t* out,
                                 void* stream);

/*
 * Shared-alpha search for many sources observed at the same times with
 * errors proportional to one sigma (Section 5: the inverse normal matrix of a
 * frequency is the same for all of them).  Source s has data x[s][i] and
 * errors scale[s] * sigma[i]; its Delta chi2 equals fchi2_search on
 * (t, x[s], scale[s] * sigma).  Here the weight grids, their FFT and the
 * Cholesky factor of alpha are computed once per frequency and only beta is
 * formed per source; Delta chi2 of source s is the base-weight value divided
 * by scale[s]^2.
 *  plan      a plan of ONE curve (offsets {0, n}: the shared time base), H <= 5
 *  t, sigma  device FP64 [n], t ascending
 *  x         device FP64 [n_sources][n]
 *  scale     device FP64 [n_sources], > 0 (a source with a bad scale or data
 *            gets NaN rows and chi2_0)
 *  dchi2     device [n_sources][H][n_freq], float (MIXED) or double (FP64)
 *  chi2_0    device FP64 [n_sources] or NULL
 *  flags     device u8 [n_freq] or NULL: bin flags, shared by all sources (or
 *            the FCHI2_CURVE_* bits of the time base if it is rejected)
 *  workspace >= fchi2_search_multi_workspace_bytes(plan, n_sources) bytes,
 *            256-byte aligned (sources are processed in waves bounding the
 *            grid memory to ~8 GiB)
 * No backward.  The workspace query returns 0 for an unsupported plan.
 * Errors: FCHI2_ERR_ARG, FCHI2_ERR_UNSUPPORTED (H > 5), FCHI2_ERR_HIP.
 */
size_t fchi2_search_multi_workspace_bytes(fchi2_plan_t plan, int32_t n_sources);
/* The autotuner of fchi2_autotune for this form: times the FFT splits and
 * spreading tiles on fchi2_search_multi with the caller's data (dchi2 is
 * scratch) and keeps the fastest in the plan.  Synchronises `stream`. */
fchi2_status_t fchi2_autotune_multi(fchi2_plan_t plan, const double* t, const double* sigma,
                                    const double* x, const double* scale, int32_t n_sources,
                                    void* workspace, size_t workspace_bytes, void* dchi2,
                                    void* stream);
fchi2_status_t fchi2_search_multi(fchi2_plan_t plan, const double* t, const double* sigma,
                                  const double* x, const double* scale, int32_t n_sources,
                                  void* workspace, size_t workspace_bytes, void* dchi2,
                                  double* chi2_0, uint8_t* flags, void* stream);

/*
 * Polynomial detrending (the option of the paper's reference implementation
 * described in Section 4: remove a slow polynomial variation, up to t^3,
 * before searching for periodic variation on top of it).  For every curve of
 * the plan, subtracts the weighted least-squares polynomial of the given
 * degree in t (minimising sum (x - p(t))^2 / sigma^2) and writes the
 * residuals; search them with any other entry point.  The fit is taken in
 * Legendre polynomials of u = 2 (t - T0) / span - 1 (T0 and span from the
 * first and last time of the curve), Cholesky in FP64; a pivot below 1e-12
 * of its diagonal is dropped (fewer than degree + 1 distinct times).
 *  degree  0..3 (0: subtract the weighted mean)
 *  x_out   device FP64 [n_total]; may be x itself (in place)
 *  coef    device FP64 [n_curves][degree + 1] Legendre coefficients, or NULL
 * Non-finite inputs propagate NaN to the curve's residuals.
 * Errors: FCHI2_ERR_ARG (NULL, degree), FCHI2_ERR_HIP.
 */
fchi2_status_t fchi2_detrend(fchi2_plan_t plan, const double* t, const double* x,
                             const double* sigma, int32_t degree, double* x_out, double* coef,
                             void* stream);

/*
 * Measurement support.  fchi2_profile(plan, 1) makes every later
 * fchi2_search / fchi2_backward on the plan record a HIP event pair around
 * each kernel launch, on the stream of that call (graph replay is bypassed
 * while profiling).  fchi2_profile_read waits for the recorded events and
 * fills total_ms[s] (milliseconds summed over launches) and launches[s] for
 * each stage s = FCHI2_PROF_*, accumulated since fchi2_profile was last
 * called.  fchi2_profile(plan, 0) stops recording and clears the totals.
 *  total_ms, launches  host arrays of FCHI2_PROF_STAGES entries
 * Errors: FCHI2_ERR_ARG (NULL), FCHI2_ERR_HIP.
 */
#define FCHI2_PROF_MOMENTS 0
#define FCHI2_PROF_SPREAD 1
#define FCHI2_PROF_FFT_FIRST 2
#define FCHI2_PROF_FFT_MID 3
#define FCHI2_PROF_FFT_LAST 4
#define FCHI2_PROF_SOLVE 5
#define FCHI2_PROF_BWD_SOLVE 6
#define FCHI2_PROF_BWD_FFT 7
#define FCHI2_PROF_BWD_GATHER 8
#define FCHI2_PROF_BWD_FINAL 9
#define FCHI2_PROF_TOP_MERGE 10
#define FCHI2_PROF_FINE 11
#define FCHI2_PROF_PERSISTENT 12
#define FCHI2_PROF_STAGES 13
fchi2_status_t fchi2_profile(fchi2_plan_t plan, int32_t enable);
fchi2_status_t fchi2_profile_read(fchi2_plan_t plan, double* total_ms, int64_t* launches);

/*
 * Autotuner.  Times every candidate schedule of the plan on the caller's data
 * (the FFT digit splits with the fewest passes and, for grids of at most
 * 2^20 cells, the most balanced splits with one pass more, for FP32 grids each on FFT tiles of 4096 or 8192
 * elements per pass, spreading tiles of 1024 to 8192 cells or, outside band
 * plans, the spreading fused into the first FFT pass, waves of wave_max,
 * wave_max/2, /4, /6, /8, /10, /12 curves with the last FFT pass and the
 * solve on whole or half waves, and for batches that fill the device the
 * persistent search; splits and tiles are ranked on the largest wave, wave
 * sizes for the best candidate of each of the three fastest splits) with HIP
 * events on `stream` (two timed runs each after a warm-up, then the three
 * fastest five more times each, in turns), keeps the fastest in the plan,
 * and appends it to the
 * text file `cache_path` (may be NULL) keyed by the shape bucket (H, n_freq,
 * precision, kernel width, log2 curves, log2 largest curve, wave_max).  If
 * the file already holds the key, the cached schedule is applied without
 * timing.  The outputs of later searches may differ from the untuned plan's
 * only by rounding.  Synchronises `stream`; not for graph capture.
 *  t, x, sigma, workspace, dchi2  as for fchi2_search (dchi2 is scratch here)
 * Errors: FCHI2_ERR_ARG, FCHI2_ERR_HIP.
 */
fchi2_status_t fchi2_autotune(fchi2_plan_t plan, const double* t, const double* x,
                              const double* sigma, void* workspace, size_t workspace_bytes,
                              void* dchi2, const char* cache_path, void* stream);

/*
 * Current schedule of a plan: info[0] = FFT passes, info[1..4] = log2 radix of
 * digits 1..4 (0 if unused), info[5] = log2 spreading tile, info[6] = curves
 * per wave, info[7] = kernel width, and with n >= 12 info[8..11] = log2 FFT
 * tile elements of passes 1..4 (0 if unused), with n >= 13 info[12] = 1 if
 * the spreading runs inside the first FFT pass, with n >= 14 info[13] = 1 if
 * searches run as one persistent launch, with n >= 15 info[14] = curves per
 * launch of the last FFT pass and the solve (0: the whole wave).  n must be
 * >= 8.
 */
fchi2_status_t fchi2_plan_info(fchi2_plan_t plan, int32_t* info, int32_t n);

/*
 * Apply a schedule in the layout fchi2_plan_info reports (n >= 14: FFT
 * passes, log2 radices, log2 spreading tile, curves per wave, -, log2 FFT
 * tiles, fused, persistent, and with n >= 15 the last pass's sub-wave, else
 * 0; info[7] is ignored) without timing anything, e.g.
 * one an earlier fchi2_autotune chose, to reproduce a run.  The split must be
 * one of the autotuner's candidates for the plan.  Like fchi2_autotune it
 * ends the state a backward call would read.
 * Errors: FCHI2_ERR_ARG (NULL, n, tile, wave, flags), FCHI2_ERR_UNSUPPORTED
 * (a split the plan does not build, fused band plan, persistent schedule the
 * persistent search does not take).
 */
fchi2_status_t fchi2_plan_set_schedule(fchi2_plan_t plan, const int32_t* info, int32_t n);

/* Free the plan and its device tables (no-op for NULL). */
void fchi2_destroy(fchi2_plan_t plan);

/* Static description of a status code. */
const char* fchi2_status_string(fchi2_status_t status);

/* Message of the last error on the calling thread ("" if none). */
const char* fchi2_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FCHI2_H_ */
