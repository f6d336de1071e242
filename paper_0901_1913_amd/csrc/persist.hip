// Persistent batched search: one launch over all curves of a plan.
//
// The workgroups of the launch take curves from a device-side work queue (a
// counter in the workspace, claimed with a global atomic add) until it runs
// dry.  Each workgroup runs the whole chain of its curve itself, in its own
// scratch slot: the tile table of every harmonic, then pair by pair the
// spreading of the pair's grid and every FFT pass over it (the pruned spectra
// of all pairs accumulate in the slot), then the per-bin solve, which writes
// the curve's Delta chi2 rows and bin flags.  Nothing is shared between
// workgroups except the queue counter, so no workgroup ever waits for
// another; stages within a workgroup are separated by its barriers.  Curves
// of uneven length simply take more or less time: the queue balances them.
// Every stage is the same tile code as the per-stage kernels (spread_tile.h,
// fft_tile.h, solve_bin.h) on the same schedule, so each curve's results are
// identical bit for bit to the per-stage search's.
#include "fchi2_internal.h"
#include "launch.h"
#include "fft_tile.h"
#include "spread_tile.h"
#include "solve_bin.h"

namespace fchi2 {

namespace {

using namespace solve_detail;

template <typename T>
constexpr size_t cmax(T a, T b) {
  return a > b ? a : b;
}

// LDS of the largest stage: FFT tiles of 4096 FP32 elements (N = 2^5..2^9
// rows) and spreading tiles of 1024 or 2048 cells.
constexpr size_t kSmemBytes =
    cmax(cmax(cmax(sizeof(FftSmem<float, 5, 7>), sizeof(FftSmem<float, 6, 6>)),
              cmax(sizeof(FftSmem<float, 7, 5>), sizeof(FftSmem<float, 8, 4>))),
         cmax(sizeof(FftSmem<float, 9, 3>),
              cmax(sizeof(SpreadSmem<10>), sizeof(SpreadSmem<11>))));

template <typename T>
__device__ __forceinline__ T& smem_as(unsigned char* p) {
  return *reinterpret_cast<T*>(p);
}

// The thread index, hidden from the optimiser.  Every address a tile forms
// from the thread index is the same for every tile of a loop; left to itself
// the compiler hoists them all out of the tile loop and keeps them live across
// it, which takes the kernel to the whole register file (one wave per SIMD).
// An opaque copy per tile keeps the address arithmetic per tile, as in the
// per-stage kernels.
__device__ __forceinline__ int opaque_tid() {
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  return tid;
}

// One FFT pass over pair p of the curve in the slot: every column tile in
// turn (4096-element tiles, 2^LOGN rows).  The stages are functions of their
// own (not inlined), so that each gets the register allocation of its own
// kernel rather than that of all stages merged.
template <int LOGN>
__device__ __forceinline__ void slot_pass(const PersistArgs& a, const FftPassArgs& fa,
                                          const cplx<float>* in, cplx<float>* out, int p, int c,
                                          cplx<float>* zpair, unsigned char* smem) {
  constexpr int LOGT = 12 - LOGN;
  const int64_t tiles = (a.g.L >> LOGN) >> LOGT;
  for (int64_t bx = 0; bx < tiles; ++bx) {
    fft_pass_tile<float, LOGN, LOGT, false>(fa, in, out, a.mom, a.g, a.tws, a.twsm, (int)bx, p,
                                            c, 0, zpair, smem_as<FftSmem<float, LOGN, LOGT>>(smem),
                                            opaque_tid());
    __syncthreads();  // the next tile rewrites the twiddles and the tile in LDS
  }
}

template <int LOGB>
__device__ __forceinline__ void slot_spread(const PersistArgs& a, const Moments& mo, int p,
                                            const int32_t* tb, cplx<float>* gA,
                                            unsigned char* smem) {
  const int64_t nt = pair_extent(mo, a.g, p) >> LOGB;
  for (int64_t tile = 0; tile < nt; ++tile)
    spread_tile<float, LOGB, false>(a.t, a.x, a.sigma, mo, a.g, 0, tb, a.ntb, 0, p, tile,
                                    gA + (tile << LOGB), smem_as<SpreadSmem<LOGB>>(smem), opaque_tid());
}

template <int H>
__device__ __forceinline__ void slot_tables(const PersistArgs& a, const Moments& mo, int32_t* tb) {
  for (int m = 1; m <= 2 * a.g.H; ++m)
    for (int64_t il = opaque_tid(); il <= mo.n; il += kNT)
      tile_bounds_point(a.t, mo, a.g, 0, m, il, a.log_tile, a.ntb, tb);
}

template <int H>
__device__ __forceinline__ void slot_solve(const PersistArgs& a, int c, const cplx<float>* zc) {
  const int64_t nf = a.g.n_freq;
  const Moments mo = a.mom[c];
  for (int64_t k = opaque_tid(); k < nf; k += kNT) {
    float d[H];
    const uint8_t fl = solve_bin<H, float, float, false>(zc, a.D, mo, a.g, 0, k, a.eps, d);
    float* o = a.out + (int64_t)c * H * nf + k;
#pragma unroll
    for (int h = 0; h < H; ++h) o[h * nf] = d[h];
    if (a.flags) a.flags[(int64_t)c * nf + k] = fl;
  }
}

// Waves per SIMD the kernel is compiled for: the solve's registers grow with
// H; up to H = 3 every stage fits 168 registers (three workgroups per CU).
template <int H>
constexpr int persist_waves() {
  return H <= 3 ? 3 : (H <= 5 ? 2 : 1);
}

template <int H>
__global__ __launch_bounds__(kNT, persist_waves<H>()) void k_search_persistent(PersistArgs a) {
  __shared__ __align__(16) unsigned char smem[kSmemBytes];
  __shared__ int s_c;
  const int tid = threadIdx.x;
  const Geom& g = a.g;
  char* slot = a.slots + (size_t)blockIdx.x * a.slot_bytes;
  cplx<float>* gA = (cplx<float>*)slot;
  cplx<float>* gB = (cplx<float>*)(slot + a.off_gB);
  cplx<float>* zc = (cplx<float>*)(slot + a.off_zc);
  int32_t* tb = (int32_t*)(slot + a.off_tb);
  const int64_t nf = g.n_freq;
  for (;;) {
    if (tid == 0) s_c = atomicAdd(a.next, 1);
    __syncthreads();
    const int cq = __builtin_amdgcn_readfirstlane(s_c);
    __syncthreads();  // every thread has read s_c before it is written again
    if (cq >= a.n_curves) break;  // the queue is dry: every wave leaves here
    const int c = a.curve_base + cq;
    const Moments mo = a.mom[c];
    if (!(mo.flags & kCurveFatal)) {
      slot_tables<H>(a, mo, tb);
      __syncthreads();
      for (int p = 0; p < g.P; ++p) {
        if (a.log_tile == 10)
          slot_spread<10>(a, mo, p, tb, gA, smem);
        else
          slot_spread<11>(a, mo, p, tb, gA, smem);
        __syncthreads();
        for (int q = a.fa[1].np; q >= 1; --q) {
          const FftPassArgs& fa = a.fa[q];
          const cplx<float>* in = (q == fa.np) ? gA : gB;
          cplx<float>* zpair = zc + (int64_t)p * 2 * nf;
          switch (fa.logn[q]) {
            case 5: slot_pass<5>(a, fa, in, gB, p, c, zpair, smem); break;
            case 6: slot_pass<6>(a, fa, in, gB, p, c, zpair, smem); break;
            case 7: slot_pass<7>(a, fa, in, gB, p, c, zpair, smem); break;
            case 8: slot_pass<8>(a, fa, in, gB, p, c, zpair, smem); break;
            default: slot_pass<9>(a, fa, in, gB, p, c, zpair, smem); break;
          }
          __syncthreads();
        }
      }
    }
    // The solve (a rejected curve gets NaN rows and its flags, as in the
    // per-stage search).
    slot_solve<H>(a, c, zc);
  }
}

__global__ void k_queue_reset(int* next) { *next = 0; }

}  // namespace

size_t persist_smem_bytes() { return kSmemBytes; }

hipError_t persist_occupancy(int H, int* blocks_per_cu) {
  hipError_t e = hipErrorInvalidValue;
  switch (H) {
#define FCHI2_OCC(h)                                                                        \
  case h:                                                                                   \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_search_persistent<h>, \
                                                     kNT, 0);                               \
    break;
    FCHI2_OCC(1)
    FCHI2_OCC(2)
    FCHI2_OCC(3)
    FCHI2_OCC(4)
    FCHI2_OCC(5)
    FCHI2_OCC(6)
    FCHI2_OCC(7)
    FCHI2_OCC(8)
#undef FCHI2_OCC
    default: break;
  }
  return e;
}

hipError_t launch_persistent(const PersistArgs& a, int n_slots, hipStream_t st) {
  // A fill kernel, not a memset, so the reset can be captured in a graph.
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, st, a.next);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (a.g.H) {
#define FCHI2_LAUNCH(h)                                                                      \
  case h:                                                                                    \
    hipLaunchKernelGGL(k_search_persistent<h>, dim3((unsigned)n_slots), dim3(kNT), 0, st, a); \
    break;
    FCHI2_LAUNCH(1)
    FCHI2_LAUNCH(2)
    FCHI2_LAUNCH(3)
    FCHI2_LAUNCH(4)
    FCHI2_LAUNCH(5)
    FCHI2_LAUNCH(6)
    FCHI2_LAUNCH(7)
    FCHI2_LAUNCH(8)
#undef FCHI2_LAUNCH
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fchi2
