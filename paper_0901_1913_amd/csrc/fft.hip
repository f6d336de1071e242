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
// (PASS_LAST).  Every pass is a batch of N_q-point FFTs done in LDS on a tile
// of N_q rows x T consecutive columns, so global reads and writes are runs of
// T (or N_q) consecutive elements.  PASS_FIRST reads the natural-order grid
// written by the spreading kernel and writes a digit-reversed prefix layout;
// middle passes work in place; PASS_LAST writes natural order, pruned to the
// bins the next stage needs.  Zero rows (grid beyond its nonzero extent, or
// the unused middle of the adjoint spectrum) are never read.
#include "fchi2_internal.h"
#include "launch.h"

namespace fchi2 {

namespace {

constexpr double kC16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
    0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978,
    0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674};
constexpr double kS16[16] = {
    0.0, 0.38268343236508978, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508978,
    0.0, -0.38268343236508978, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508978};

// v * exp(+2 pi i E / N) for compile-time E, N <= 16.
template <typename R, int N, int E>
__device__ __forceinline__ cplx<R> mul_root(cplx<R> v) {
  constexpr int e = E % N;
  if constexpr (e == 0) {
    return v;
  } else if constexpr (4 * e == N) {
    return cmk<R>(-v.y, v.x);
  } else if constexpr (2 * e == N) {
    return cmk<R>(-v.x, -v.y);
  } else if constexpr (4 * e == 3 * N) {
    return cmk<R>(v.y, -v.x);
  } else {
    constexpr int k = e * (16 / N);
    const R c = (R)kC16[k];
    const R s = (R)kS16[k];
    return cmk<R>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

template <int N, int I>
constexpr int bitrev() {
  int r = 0, x = I;
  for (int b = 1; b < N; b <<= 1) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

template <typename R, int N, int I>
__device__ __forceinline__ void bitrev_perm(cplx<R>* v) {
  if constexpr (I < N) {
    constexpr int J = bitrev<N, I>();
    if constexpr (I < J) {
      cplx<R> t = v[I];
      v[I] = v[J];
      v[J] = t;
    }
    bitrev_perm<R, N, I + 1>(v);
  }
}

template <typename R, int N, int S, int K, int J>
__device__ __forceinline__ void bfly_j(cplx<R>* v) {
  if constexpr (J < S) {
    constexpr int e = J * (N / (2 * S));
    cplx<R> t = mul_root<R, N, e>(v[K + J + S]);
    cplx<R> u = v[K + J];
    v[K + J] = cadd(u, t);
    v[K + J + S] = csub(u, t);
    bfly_j<R, N, S, K, J + 1>(v);
  }
}
template <typename R, int N, int S, int K>
__device__ __forceinline__ void bfly_k(cplx<R>* v) {
  if constexpr (K < N) {
    bfly_j<R, N, S, K, 0>(v);
    bfly_k<R, N, S, K + 2 * S>(v);
  }
}
template <typename R, int N, int S>
__device__ __forceinline__ void dit_stages(cplx<R>* v) {
  if constexpr (S < N) {
    bfly_k<R, N, S, 0>(v);
    dit_stages<R, N, 2 * S>(v);
  }
}

// In-register N-point DFT (N <= 16), natural order in and out, sign +i.
template <typename R, int N>
__device__ __forceinline__ void dft_reg(cplx<R>* v) {
  bitrev_perm<R, N, 0>(v);
  dit_stages<R, N, 1>(v);
}

constexpr int kNT = 256;  // threads per FFT workgroup

template <typename R>
struct TileElems;
template <>
struct TileElems<float> {
  static constexpr int log = 13;  // 8192 complex floats per tile (64 KiB)
};
template <>
struct TileElems<double> {
  static constexpr int log = 12;  // 4096 complex doubles per tile (64 KiB)
};

// One Stockham radix-RAD stage over the tile [N rows][T columns] in LDS.
template <typename R, int LOGN, int LOGT, int LOGNS>
__device__ __forceinline__ void lds_stage(cplx<R>* sm, const cplx<R>* __restrict__ tw,
                                          int tid) {
  constexpr int N = 1 << LOGN;
  constexpr int T = 1 << LOGT;
  constexpr int NS = 1 << LOGNS;
  constexpr int LOGRAD = (LOGN - LOGNS) >= 4 ? 4 : (LOGN - LOGNS);
  constexpr int RAD = 1 << LOGRAD;
  constexpr int PT = (T == 1) ? 1 : T + 1;
  constexpr int NBF = (N / RAD) * T;
  constexpr int PER = NBF / kNT;
  static_assert(PER >= 1 && PER * kNT == NBF, "tile too small for the workgroup");
  constexpr int TWS = kStageLog - LOGNS - LOGRAD;
  static_assert(TWS >= 0, "stage twiddle table too small");

  cplx<R> v[PER][RAD];
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int bi = tid + it * kNT;
    const int c = bi & (T - 1);
    const int b = bi >> LOGT;
#pragma unroll
    for (int i = 0; i < RAD; ++i) v[it][i] = sm[(b + i * (N / RAD)) * PT + c];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < PER; ++it) {
    const int bi = tid + it * kNT;
    const int c = bi & (T - 1);
    const int b = bi >> LOGT;
    const int j = b & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int i = 1; i < RAD; ++i) v[it][i] = cmul(v[it][i], tw[(j * i) << TWS]);
    }
    dft_reg<R, RAD>(v[it]);
    const int row0 = ((b >> LOGNS) << (LOGNS + LOGRAD)) + j;
#pragma unroll
    for (int i = 0; i < RAD; ++i) sm[(row0 + i * NS) * PT + c] = v[it][i];
  }
  __syncthreads();
}

template <typename R, int LOGN, int LOGT, int LOGNS>
__device__ __forceinline__ void lds_fft(cplx<R>* sm, const cplx<R>* __restrict__ tw, int tid) {
  if constexpr (LOGNS < LOGN) {
    lds_stage<R, LOGN, LOGT, LOGNS>(sm, tw, tid);
    constexpr int step = (LOGN - LOGNS) >= 4 ? 4 : (LOGN - LOGNS);
    lds_fft<R, LOGN, LOGT, LOGNS + step>(sm, tw, tid);
  }
}

// omega_L^e from the two-level table: lo[e & (2^s - 1)] * hi[e >> s].
template <typename R>
__device__ __forceinline__ cplx<R> tw_L(const cplx<R>* __restrict__ lo,
                                        const cplx<R>* __restrict__ hi, int64_t e, int s) {
  const int64_t m = ((int64_t)1 << s) - 1;
  return cmul(lo[e & m], hi[e >> s]);
}

template <typename R, int LOGN, int LOGT>
__global__ __launch_bounds__(kNT) void k_fft_pass(FftPassArgs a, const cplx<R>* in,
                                                 cplx<R>* out,
                                                 const Moments* __restrict__ mom, Geom g,
                                                 const cplx<R>* __restrict__ tw_stage,
                                                 const cplx<R>* __restrict__ tw_lo,
                                                 const cplx<R>* __restrict__ tw_hi) {
  constexpr int N = 1 << LOGN;
  constexpr int T = 1 << LOGT;
  constexpr int PT = (T == 1) ? 1 : T + 1;
  constexpr int ELEMS = N * T;
  __shared__ cplx<R> sm[N * PT];

  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int cw = blockIdx.z;
  const Moments mo = mom[a.curve0 + cw];
  if (mo.flags & kCurveFatal) return;

  const int64_t L = g.L;
  const int logL = a.logL;
  const int64_t grid_off = ((int64_t)cw * g.P + p) * L;
  const cplx<R>* src = in + grid_off;
  const int64_t g0 = (int64_t)blockIdx.x * T;  // first column of this tile
  const cplx<R> zero = cmk<R>((R)0, (R)0);

  // Sum of log2 N over digits below q.
  int low_bits = 0;
  for (int d = 1; d < a.q; ++d) low_bits += a.logn[d];

  if (a.kind == PASS_FIRST || a.kind == PASS_SINGLE) {
    // Column c = g0 + cc, row r at c + S * r, S = L / N.
    const int64_t S = L >> LOGN;
    int64_t r_skip_lo, r_skip_hi;  // rows in [r_skip_lo, r_skip_hi) are zero
    if (a.mode == MODE_FWD) {
      const int64_t E = pair_extent(mo, g, p);
      r_skip_lo = (E + S - 1) / S;
      r_skip_hi = N;
    } else {
      r_skip_lo = g.n_freq / S;
      r_skip_hi = (L - g.n_freq) / S;
    }
#pragma unroll 4
    for (int it = 0; it < ELEMS / kNT; ++it) {
      const int e = tid + it * kNT;
      const int cc = e & (T - 1);
      const int r = e >> LOGT;
      cplx<R> v = zero;
      if (r < r_skip_lo || r >= r_skip_hi) v = src[g0 + cc + S * r];
      sm[r * PT + cc] = v;
    }
  } else if (a.kind == PASS_MID) {
    const int64_t Tail = L >> (low_bits + LOGN);
    const int64_t pre = g0 / Tail;
    const int64_t K0 = g0 - pre * Tail;
    const cplx<R>* base = src + pre * ((int64_t)N * Tail) + K0;
#pragma unroll 4
    for (int it = 0; it < ELEMS / kNT; ++it) {
      const int e = tid + it * kNT;
      const int cc = e & (T - 1);
      const int r = e >> LOGT;
      sm[r * PT + cc] = base[r * Tail + cc];
    }
  } else {  // PASS_LAST
    const int64_t Tail = L >> LOGN;
    const cplx<R>* base = src + g0;
#pragma unroll 4
    for (int it = 0; it < ELEMS / kNT; ++it) {
      const int e = tid + it * kNT;
      const int cc = e & (T - 1);
      const int r = e >> LOGT;
      sm[r * PT + cc] = base[r * Tail + cc];
    }
  }
  __syncthreads();

  lds_fft<R, LOGN, LOGT, 0>(sm, tw_stage, tid);

  cplx<R>* dst = out + grid_off;
  if (a.kind == PASS_FIRST) {
    // Output row for column c is rev(c) * N + k (digit-reversed prefix).
    const int np = a.np;
    // Twiddle digit j_{np-1} = c >> (bits of digits 1..np-2); modulus N_{np-1} * N.
    int bits_below = 0;
    for (int d = 1; d < np - 1; ++d) bits_below += a.logn[d];
    const int logM = a.logn[np - 1] + LOGN;
    const int64_t Mmask = ((int64_t)1 << logM) - 1;
    const int sh = logL - logM;
#pragma unroll 4
    for (int it = 0; it < ELEMS / kNT; ++it) {
      const int e = tid + it * kNT;
      const int k = e & (N - 1);
      const int cc = e >> LOGN;
      const int64_t c = g0 + cc;
      // Mixed-radix reversal: rev = ((j_1 N_2 + j_2) N_3 + j_3) ... + j_{np-1}.
      int64_t rev = 0, rest = c;
      for (int d = 1; d < np; ++d) {
        const int64_t dig = rest & (((int64_t)1 << a.logn[d]) - 1);
        rest >>= a.logn[d];
        rev = (rev << a.logn[d]) | dig;
      }
      cplx<R> v = sm[k * PT + cc];
      const int64_t jd = c >> bits_below;
      const int64_t ex = ((jd * (int64_t)k) & Mmask) << sh;
      v = cmul(v, tw_L(tw_lo, tw_hi, ex, a.tw_s));
      dst[rev * N + k] = v;
    }
  } else if (a.kind == PASS_MID) {
    const int64_t Tail = L >> (low_bits + LOGN);
    const int64_t pre = g0 / Tail;
    const int64_t K0 = g0 - pre * Tail;
    const int64_t jd = pre & (((int64_t)1 << a.logn[a.q - 1]) - 1);
    int logTail = logL - low_bits - LOGN;
    const int logM = a.logn[a.q - 1] + LOGN + logTail;
    const int64_t Mmask = ((int64_t)1 << logM) - 1;
    const int sh = logL - logM;
    cplx<R>* base = dst + pre * ((int64_t)N * Tail) + K0;
#pragma unroll 4
    for (int it = 0; it < ELEMS / kNT; ++it) {
      const int e = tid + it * kNT;
      const int cc = e & (T - 1);
      const int k = e >> LOGT;
      const int64_t Kp = K0 + cc + Tail * k;
      const int64_t ex = ((jd * Kp) & Mmask) << sh;
      base[k * Tail + cc] = cmul(sm[k * PT + cc], tw_L(tw_lo, tw_hi, ex, a.tw_s));
    }
  } else {
    // PASS_LAST / PASS_SINGLE: X index = K + Tail * k, natural order.
    const int64_t Tail = L >> LOGN;
    const int64_t nf = g.n_freq;
    if (a.mode == MODE_FWD) {
      cplx<R>* z0 = (cplx<R>*)a.zc + ((int64_t)cw * g.P + p) * 2 * nf;
      cplx<R>* z1 = z0 + nf;
#pragma unroll 4
      for (int it = 0; it < ELEMS / kNT; ++it) {
        const int e = tid + it * kNT;
        const int cc = e & (T - 1);
        const int k = e >> LOGT;
        const int64_t X = g0 + cc + Tail * k;
        const cplx<R> v = sm[k * PT + cc];
        if (X < nf) z0[X] = v;
        const int64_t Xm = (L - X) & (L - 1);
        if (Xm < nf) z1[Xm] = v;
      }
    } else {
      const int64_t E = pair_extent(mo, g, p);
#pragma unroll 4
      for (int it = 0; it < ELEMS / kNT; ++it) {
        const int e = tid + it * kNT;
        const int cc = e & (T - 1);
        const int k = e >> LOGT;
        const int64_t X = g0 + cc + Tail * k;
        if (X < E) ((cplx<R>*)a.grid_out)[grid_off + X] = sm[k * PT + cc];
      }
    }
  }
}

template <typename R, int LOGN, int LOGT>
hipError_t launch_one(const FftPassArgs& a, const void* in, void* out, const Moments* mom,
                      const Geom& g, const void* tws, const void* twl, const void* twh,
                      int n_curves, int64_t ncols, hipStream_t st) {
  dim3 grid((unsigned)(ncols >> LOGT), (unsigned)g.P, (unsigned)n_curves);
  hipLaunchKernelGGL((k_fft_pass<R, LOGN, LOGT>), grid, dim3(kNT), 0, st, a,
                     (const cplx<R>*)in, (cplx<R>*)out, mom, g, (const cplx<R>*)tws,
                     (const cplx<R>*)twl, (const cplx<R>*)twh);
  return hipGetLastError();
}

template <typename R>
hipError_t dispatch(const FftPassArgs& a, int logn, int logt, const void* in, void* out,
                    const Moments* mom, const Geom& g, const void* tws, const void* twl,
                    const void* twh, int n_curves, int64_t ncols, hipStream_t st) {
  constexpr int LE = TileElems<R>::log;
  if (logt == 0) {
    // Single-pass tile: the whole grid in one workgroup.
    if (logn == LE) return launch_one<R, LE, 0>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    if constexpr (LE - 1 >= 12) {
      if (logn == LE - 1) return launch_one<R, LE - 1, 0>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    }
    return hipErrorInvalidValue;
  }
  if (logn + logt != LE) return hipErrorInvalidValue;
  switch (logn) {
    case 4: return launch_one<R, 4, LE - 4>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 5: return launch_one<R, 5, LE - 5>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 6: return launch_one<R, 6, LE - 6>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 7: return launch_one<R, 7, LE - 7>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 8: return launch_one<R, 8, LE - 8>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 9: return launch_one<R, 9, LE - 9>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    case 10: return launch_one<R, 10, LE - 10>(a, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int fft_tile_log(bool fp64) { return fp64 ? TileElems<double>::log : TileElems<float>::log; }

hipError_t launch_fft_pass(bool fp64, const FftPassArgs& a, int logn, int logt, const void* in,
                           void* out, const Moments* mom, const Geom& g, const void* tws,
                           const void* twl, const void* twh, int n_curves, int64_t ncols,
                           hipStream_t st) {
  if (fp64)
    return dispatch<double>(a, logn, logt, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
  return dispatch<float>(a, logn, logt, in, out, mom, g, tws, twl, twh, n_curves, ncols, st);
}

}  // namespace fchi2
