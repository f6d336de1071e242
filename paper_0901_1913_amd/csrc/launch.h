// Host-side launchers of the F-chi2 kernels (internal).
#pragma once

#include "fchi2_internal.h"

namespace fchi2 {

struct FftPassArgs {
  int kind;                    // PassKind
  int mode;                    // PassMode
  int np;                      // number of passes
  int q;                       // digit handled by this pass (1 = least significant)
  int logn[kMaxPasses + 1];    // log2 N_d per digit d = 1..np
  int logL;
  int curve0;                  // first curve of the wave
  void* zc;                    // forward: pruned spectra [wave][P][2][n_freq]
  void* grid_out;              // adjoint: natural-order grid output
  int fused;                   // forward first pass: spread the points in the tile
  const double* t;             // fused: the curves' points (CSR, as for the search)
  const double* x;
  const double* sigma;
  const int32_t* tb;           // fused: tile table of tiles of 2^tb_log cells
  int tb_log;                  //   (2^tb_log >= w + 3), ntb entries per harmonic
  int ntb;
};

// Moments, validity flags and chi2_0 of every curve: bpc workgroups per
// curve reduce chunks into part[n_curves][bpc], then one pass combines them.
// shared_t: every curve c uses the points [offsets[0], offsets[1]) of t and
// sigma with data x[c * n + i]; scale (nullable): per-curve error scale, the
// reported chi2_0 is divided by its square.
hipError_t launch_moments(const double* t, const double* x, const double* sigma,
                          const int64_t* offsets, int n_curves, int bpc, const Geom& g,
                          MomPart* part, Moments* mom, double* chi2_0, hipStream_t st,
                          bool shared_t = false, const double* scale = nullptr);

// Spread w and w*(x - xbar) of each curve of the wave onto its P packed grids.
// tb: tile -> point-range table, tile_bounds_bytes(g, log_tile, n_curves).
hipError_t launch_spread(bool fp64, const double* t, const double* x, const double* sigma,
                         const Moments* mom, const Geom& g, int curve0, int n_curves,
                         int64_t max_n, int32_t* tb, void* grid, int log_tile, hipStream_t st,
                         bool share_tb = false);
size_t tile_bounds_bytes(const Geom& g, int log_tile, int n_curves);
// The tile table alone (tiles of 2^log_tile cells): the fused first FFT pass
// reads it to find each row segment's points.
hipError_t launch_tile_bounds(const double* t, const Moments* mom, const Geom& g, int curve0,
                              int n_curves, int64_t max_n, int32_t* tb, int log_tile,
                              hipStream_t st);

// log2 of the elements of the largest FFT tile (rows x columns held in LDS).
int fft_tile_log(bool fp64);
// tws: omega_{2^13}^e (FP64), twsm: omega_L^e for e < 2^fft_tile_log(fp64) (FP64).
hipError_t launch_fft_pass(bool fp64, const FftPassArgs& a, int logn, int logt, const void* in,
                           void* out, const Moments* mom, const Geom& g, const void* tws,
                           const void* twsm, int n_curves, int64_t ncols, hipStream_t st);

// Persistent batched search (MIXED plans, H <= 8, FFT splits of 4096-element
// tiles with 2^5..2^9 rows per pass, spreading tiles of 2^10 or 2^11 cells):
// one launch of n_slots workgroups takes curves [curve_base, curve_base +
// n_curves) from the queue counter *next and runs each one's whole chain in
// its own slot of slot_bytes (gA at 0, gB at off_gB, spectra at off_zc, tile
// table at off_tb).  The moments must be computed first.
struct PersistArgs {
  const double* t;
  const double* x;
  const double* sigma;
  const Moments* mom;
  Geom g;
  // fa[q]: the arguments of forward pass q = 1..np (kind, split, logL), with
  // curve0 = 0: the pass reads its curve's moments at mom[c].  Prebuilt per
  // pass so that the kernel indexes the split from its argument block.
  FftPassArgs fa[kMaxPasses + 1];
  const cplx<double>* tws;
  const cplx<double>* twsm;
  const cplx<double>* D;
  int curve_base;
  int n_curves;
  int log_tile;
  int ntb;
  char* slots;
  size_t slot_bytes, off_gB, off_zc, off_tb;
  int* next;
  double eps;
  float* out;
  uint8_t* flags;
};
size_t persist_smem_bytes();
hipError_t persist_occupancy(int H, int* blocks_per_cu);
hipError_t launch_persistent(const PersistArgs& a, int n_slots, hipStream_t st);

// Deconvolution / origin-shift factors D[k] = exp(-2 pi i k c_off / L) / phi_hat(k).
// FP64 complex [n_freq].
hipError_t launch_deconv_init(void* D, const Geom& g, const double* gl_x, const double* gl_w,
                              int n_gl, hipStream_t st);

// Normal-matrix assembly, Cholesky and prefix Delta chi2 per bin; coef
// (nullable): the H model's coefficients [curve][2H+1][n_freq], output type.
// H <= 8 uses the register solver (one bin per thread) unless `wide`; H > 8
// always the wave-per-bin solver (H <= 16, not for band plans).
hipError_t launch_solve(bool fp64, const void* zc, const void* D, const Moments* mom,
                        const Geom& g, int curve0, int n_curves, double eps_piv, void* dchi2,
                        uint8_t* flags, hipStream_t st, void* coef = nullptr,
                        bool wide = false);

// Shared-alpha solve for sources at the same times (H <= 5): alpha from the
// weight spectra zq (slot 0, H pairs), beta per source from zp (ceil(H/2)
// pairs per wave slot); rows of source s scaled by 1/scale[s]^2.
hipError_t launch_solve_multi(bool fp64, const void* zq, const void* zp, const void* D,
                              const Moments* mom_t, const Moments* mom_s, const double* scale,
                              const Geom& g, int src0, int n_src, double eps_piv, void* dchi2,
                              uint8_t* flags, hipStream_t st);

// Adjoint of the solve: per-bin gradients into the packed adjoint spectra.
hipError_t launch_adjoint_solve(bool fp64, const void* zc, const void* D, const Moments* mom,
                                const Geom& g, int curve0, int n_curves, double eps_piv,
                                const void* grad_dchi2, void* spec, double* dW_part,
                                int blocks_per_curve, hipStream_t st);

// Interpolate the adjoint grids at the points (transpose of the spreading).
hipError_t launch_gather(bool fp64, const double* t, const Moments* mom, const Geom& g,
                         int curve0, int n_curves, const void* grid, double* gq, double* gp,
                         int64_t max_n, hipStream_t st);

// Reduce the per-curve terms and write d/dx, d/dsigma; scratch holds
// 2 * nch doubles per curve of the wave's curves (indexed by absolute curve).
hipError_t launch_finalize(const double* x, const double* sigma, const Moments* mom,
                           const Geom& g, int curve0, int n_curves, const double* dW_part,
                           int blocks_per_curve, const double* gq, const double* gp,
                           double* grad_x, double* grad_sigma, double* scratch, int nch,
                           hipStream_t st);

// Top-K strict local maxima of one Delta chi2 row per curve.
hipError_t launch_peaks(bool fp64, const void* dchi2, int64_t n_freq, int H, int hrow,
                        int n_curves, int64_t k_lo, int K, void* scratch, int64_t* out_idx,
                        hipStream_t st);
size_t peaks_scratch_bytes(int64_t n_freq, int n_curves, int K);

// Per-block candidate lists of the significance epilogue (one wave of curves).
struct TopScratch {
  double* score;   // [curve][block][K] ln p, ascending per block (+inf: empty)
  int64_t* k;      // [curve][block][K] bin (-1: empty)
  uint8_t* flag;   // [curve][block][K] bin flags
  double* d;       // [curve][block][K][H] Delta chi2 rows at the bin
  double* bmax;    // [curve][block] largest eligible Delta chi2 of the ranked row
  // merged lists of groups of up to 256 blocks
  double* g_score;  // [curve][group][K]
  int64_t* g_k;     // [curve][group][K]
  int64_t* g_q;     // [curve][group][K] index of the record in the arrays above
  double* g_max;    // [curve][group]
};
// Per-curve results (absolute curve index); any pointer but idx and log_p may be null.
struct TopOut {
  int64_t* idx;
  double* log_p;
  double* dchi2;      // [curve][K][H]
  double* dchi2_adj;  // [curve][K]
  uint8_t* flags;     // [curve][K]
  double* chi2_best;  // [curve]
  uint8_t* curve_flags;  // [curve]
};
int top_blocks(int64_t n_freq);
size_t top_scratch_bytes(int64_t n_freq, int H, int n_curves, int K);
TopScratch top_scratch_carve(void* base, int64_t n_freq, int H, int n_curves, int K);
// Fused per-bin solve and per-block candidate selection.
hipError_t launch_solve_top(bool fp64, const void* zc, const void* D, const Moments* mom,
                            const Geom& g, int curve0, int n_curves, double eps_piv, int hrow,
                            int64_t k_lo, int K, const TopScratch& sc, hipStream_t st);
// Per-curve merge of the block lists, significance and adjusted reduction.
hipError_t launch_top_merge(const Moments* mom, const Geom& g, int curve0, int n_curves,
                            int hrow, int K, const TopScratch& sc, const TopOut& out,
                            hipStream_t st);

// Subtract each curve's weighted least-squares polynomial of the given degree
// (0..3) in t; coef (nullable) receives its Legendre coefficients in u.
hipError_t launch_detrend(const double* t, const double* x, const double* sigma,
                          const int64_t* offsets, int n_curves, int degree, int64_t max_n,
                          double* x_out, double* coef, hipStream_t st);

// Fine search on the ungridded points around given centre frequencies.
struct FineOut {
  double* rows;        // [curve][K][R][H] or null
  double* f_best;      // [curve][K]
  double* dchi2_best;  // [curve][K][H]
  double* coef;        // [curve][K][2H+1] or null
  uint8_t* flags;      // [curve][K] or null
};
int fine_chunks(int64_t max_n);
size_t fine_part_bytes(int H, int n_curves, int64_t max_n, int K, int R);
hipError_t launch_fine(const double* t, const double* x, const double* sigma, const Moments* mom,
                       int H, int n_curves, int64_t max_n, const double* fc, int K, int R,
                       double hw, double* part, int hrow, const FineOut& out, hipStream_t st);

}  // namespace fchi2
