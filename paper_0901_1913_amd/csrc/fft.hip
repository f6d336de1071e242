// Batched complex FFTs of the packed harmonic grids (sign +i, unnormalised):
//   X[k] = sum_j x[j] exp(+2 pi i j k / L),  L = 2^logL.
// The sign follows the transforms P(f), Q(f) of eq. eqPQ (Section 2), which
// use exp(+i 2 pi f t).
//
// Scheme: L = N_1 * N_2 * ... * N_np, input digit j_1 least significant.
// Recursively (decimation in time),
//   X[k' + (L/N_1) k_1] = sum_{j_1} w_{N_1}^{j_1 k_1} w_L^{j_1 k'} Y_{j_1}[k'],
//   Y_{j_1} = FFT_{L/N_1}(x[j_1 + N_1 * .]).
// Passes run from the most significant digit (PASS_FIRST) down to j_1
// (PASS_LAST).  Grids are stored in HBM as S (float or double); every tile is
// held in LDS and transformed in FP64, and the twiddles between passes are
// formed per workgroup in FP64 from exactly reduced exponents, so HBM storage
// is the only place a mixed-precision plan rounds to FP32.  Every pass is a batch of N_q-point FFTs done in LDS on a tile
// of N_q rows x T consecutive columns, so global reads and writes are runs of
// T (or N_q) consecutive elements.  PASS_FIRST reads the natural-order grid
// written by the spreading kernel and writes a digit-reversed prefix layout;
// middle passes work in place; PASS_LAST writes natural order, pruned to the
// bins the next stage needs.  Zero rows (grid beyond its nonzero extent, or
// the unused middle of the adjoint spectrum) are never read.
//
// Fused first pass (FUSED): instead of reading the spread grid, the tile's
// cells {g0 + cc + (L/N) r} are computed in place from the curve's points, so
// the spreading's grid never goes through memory.  Each thread owns whole row
// segments of the tile and sums the kernel taps of the points near them, in
// point order, with the same kernel argument (cell - position, exact) as the
// standalone spreading: the cell values, and so every later result, are the
// same bit for bit.
#include "fchi2_internal.h"
#include "launch.h"
#include "fft_tile.h"

namespace fchi2 {

namespace {

template <typename S, int LOGN, int LOGT>
hipError_t launch_one(const FftPassArgs& a, const void* in, void* out, const Moments* mom,
                      const Geom& g, const void* tws, const void* twsm, int n_curves,
                      int64_t ncols, hipStream_t st) {
  dim3 grid((unsigned)(ncols >> LOGT), (unsigned)g.P, (unsigned)n_curves);
  dim3 blk(((1 << LOGN) << LOGT) / kEPT);
  if (a.fused) {
    if (a.kind != PASS_FIRST || a.mode != MODE_FWD || g.band || !a.t || !a.x || !a.sigma ||
        !a.tb || (1 << a.tb_log) < g.w + 3)
      return hipErrorInvalidValue;
    if constexpr (LOGT >= 1)
      hipLaunchKernelGGL((k_fft_pass<S, LOGN, LOGT, true>), grid, blk, 0, st, a,
                         (const cplx<S>*)in, (cplx<S>*)out, mom, g, (const C*)tws,
                         (const C*)twsm);
    else
      return hipErrorInvalidValue;
  } else {
    hipLaunchKernelGGL((k_fft_pass<S, LOGN, LOGT, false>), grid, blk, 0, st, a,
                       (const cplx<S>*)in, (cplx<S>*)out, mom, g, (const C*)tws, (const C*)twsm);
  }
  return hipGetLastError();
}

template <typename S>
hipError_t dispatch(const FftPassArgs& a, int logn, int logt, const void* in, void* out,
                    const Moments* mom, const Geom& g, const void* tws, const void* twsm,
                    int n_curves, int64_t ncols, hipStream_t st) {
  if (logt == 0) {
    if (logn == 12) return launch_one<S, 12, 0>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
    if constexpr (tile_log_max<S>() == 13)
      if (logn == 13) return launch_one<S, 13, 0>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
    return hipErrorInvalidValue;
  }
  if (logn + logt == 12) {
    switch (logn) {
      case 4: return launch_one<S, 4, 8>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      case 5: return launch_one<S, 5, 7>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      case 6: return launch_one<S, 6, 6>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      case 7: return launch_one<S, 7, 5>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      case 8: return launch_one<S, 8, 4>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      case 9: return launch_one<S, 9, 3>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
      default: return hipErrorInvalidValue;
    }
  }
  if constexpr (tile_log_max<S>() == 13) {
    if (logn + logt == 13) {
      switch (logn) {
        case 4: return launch_one<S, 4, 9>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        case 5: return launch_one<S, 5, 8>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        case 6: return launch_one<S, 6, 7>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        case 7: return launch_one<S, 7, 6>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        case 8: return launch_one<S, 8, 5>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        case 9: return launch_one<S, 9, 4>(a, in, out, mom, g, tws, twsm, n_curves, ncols, st);
        default: return hipErrorInvalidValue;
      }
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

int fft_tile_log(bool fp64) { return fp64 ? tile_log_max<double>() : tile_log_max<float>(); }

hipError_t launch_fft_pass(bool fp64, const FftPassArgs& a, int logn, int logt, const void* in,
                           void* out, const Moments* mom, const Geom& g, const void* tws,
                           const void* twsm, int n_curves, int64_t ncols, hipStream_t st) {
  if (fp64) return dispatch<double>(a, logn, logt, in, out, mom, g, tws, twsm, n_curves, ncols, st);
  return dispatch<float>(a, logn, logt, in, out, mom, g, tws, twsm, n_curves, ncols, st);
}

}  // namespace fchi2
