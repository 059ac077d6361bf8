// Lateral gridding of the non-equispaced-data NUFFT over the sensor plane
// (Section 3.2), one chunk of temporal bins at a time.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
// Stage 1: lateral spreading (the gridding of eq. NED_NUFFT), one chunk of
// temporal bins at a time. Output-driven and atomic-free: every lane owns one
// grid point and accumulates in registers the contributions of its sensors in
// a fixed order (deterministic).
// ---------------------------------------------------------------------------
constexpr int kSpreadBins = 16;  // bins per group: a lane's accumulators
constexpr int kMaxW = 16;

template <typename T, bool KAHAN>
__device__ __forceinline__ void accum(cx<T>& a, cx<T>& c, T wt, cx<T> g) {
  if (KAHAN) {
    const T yr = wt * g.x - c.x;
    const T tr = a.x + yr;
    c.x = (tr - a.x) - yr;
    a.x = tr;
    const T yi = wt * g.y - c.y;
    const T ti = a.y + yi;
    c.y = (ti - a.y) - yi;
    a.y = ti;
  } else {
    a.x += wt * g.x;
    a.y += wt * g.y;
  }
}

// A 64-thread work-group owns a
// 16 x kPatchRows patch of the grid and walks the patch's slots. A slot holds
// up to kSlotK sensors whose footprints share no point of the patch (packed
// at plan time, first fit in list order), so one pass over a slot serves
// every lane from the one sensor that covers it: with 8-point footprints on a
// 16 x 4 patch most sensors cover a quarter of the lanes or less, and a pass
// per sensor left most lanes multiplying by zero (2.6 times fewer passes on
// the warped 128 x 128 layout over a 384^2 grid). The plan also stores every
// lane's weight wx*wy and which of the slot's sensors it reads, so the inner
// loop is the LDS row reads and the FMAs. The bin values of a round's slots
// go from global memory straight into LDS (16-byte loads to LDS, no staging
// registers), laid out load-major: load i of lane L lands at i*1024 + 16*L,
// which puts the up to four rows of one slot in different banks. The plan
// keeps an even number of band bins, so every sensor's row starts on a
// 16-byte boundary and every load starts on a whole 16-byte unit of it; a
// load starting past the band's last unit is moved onto that unit (the bins
// it then holds are never stored), so no load leaves its row. Each
// grid point sums its sensors in slot order
// (deterministic). A work-group takes kSpreadGroups consecutive bin groups of
// its patch, so a patch with one round of slots (the usual case) reads its
// lane tables once. Measured on MI355X at the headline size: 8 slots per
// round beat 16; two bin groups per work-group beat one, four and nine;
// splitting a group's bins over two or four passes (fewer live accumulators)
// and XCD-contiguous or patch-major block orders were slower.

template <typename T, bool KAHAN>
__device__ __forceinline__ void spread_slot_body(const cx<T>* __restrict__ Gt, int nb,
                                                 const int* __restrict__ slot_off,
                                                 const int* __restrict__ slot_sens, const T* __restrict__ slot_w,
                                                 const unsigned* __restrict__ slot_k, int n_x, int n_y,
                                                 int tiles_x, int nchunks, int b_begin, int b_end,
                                                 cx<T>* __restrict__ U, int bx) {
  constexpr int BC = kSpreadBins, K = kSlotK, SB = kSlotBatch;
  constexpr int ROWS = SB * K;
  constexpr int LPR = 64 / ROWS;  // lanes staging one row
  constexpr int EPL = BC / LPR;   // bins staged per lane
  constexpr int EL = 16 / int(sizeof(cx<T>));  // bins per 16-byte load
  constexpr int NLD = EPL / EL;                  // loads per lane per round
  constexpr int LSTRIDE = 64 * EL;               // elements between two loads' blocks
  static_assert(ROWS * LPR == 64 && BC % LPR == 0 && EPL % EL == 0 && SB * 2 <= 32 && K <= 4, "staging layout");
  __shared__ __align__(16) cx<T> s_g[NLD * LSTRIDE];
  const int ngroups = (nchunks + kSpreadGroups - 1) / kSpreadGroups;
  const int grp = bx % ngroups;  // bin groups vary fastest: neighbours share the patch's slots
  const int patch = bx / ngroups;
  const int prg = patch / tiles_x;
  const int pcol = patch - prg * tiles_x;
  const int lane = threadIdx.x;
  const int px = pcol * kSpreadTile + (lane & 15);
  const int py = prg * kPatchRows + (lane >> 4);
  const int q_begin = slot_off[patch];
  const int q_end = slot_off[patch + 1];
  const bool one_round = q_end - q_begin <= SB;
  const int row = lane / LPR, part = lane - (lane / LPR) * LPR;
  T wq[SB];
  unsigned kq = 0;  // 2-bit places of the round's slots
  const int c_first = grp * kSpreadGroups;
  const int c_end = min(nchunks, c_first + kSpreadGroups);
  for (int c = c_first; c < c_end; ++c) {
    const int b0 = b_begin + c * BC;
    const int nbc = min(BC, b_end - b0);
    cx<T> acc[BC];
    cx<T> cmp[KAHAN ? BC : 1];
#pragma unroll
    for (int b = 0; b < BC; ++b) acc[b] = cx<T>{T(0), T(0)};
#pragma unroll
    for (int b = 0; b < (KAHAN ? BC : 1); ++b) cmp[b] = cx<T>{T(0), T(0)};
    for (int qb = q_begin; qb < q_end; qb += SB) {
      const int nq = min(SB, q_end - qb);
      if (!one_round || c == c_first) {
        // lane tables, read unconditionally (slots past the round's end
        // repeat its last one and go unused), so no load waits on a branch
#pragma unroll
        for (int q = 0; q < SB; ++q) wq[q] = slot_w[size_t(qb + min(q, nq - 1)) * 64 + lane];
        kq = slot_k[size_t(qb) * 64 + lane];
      }
      // an empty place loads sensor 0's row: no lane reads it
      const int rq = min(row / K, nq - 1);
      const int sid = row / K < nq ? max(0, slot_sens[size_t(qb + rq) * K + (row - (row / K) * K)]) : 0;
      const cx<T>* gs = Gt + size_t(sid) * nb;
      __syncthreads();  // the previous round has been consumed
#pragma unroll
      for (int i = 0; i < NLD; ++i) {
        const int e = min(b0 + part * EPL + i * EL, nb - EL);  // nb is a multiple of EL
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(gs + e),
                                         (__attribute__((address_space(3))) void*)(s_g + i * LSTRIDE), 16, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);  // the loads have landed in LDS
      __syncthreads();
#pragma unroll
      for (int q = 0; q < SB; ++q) {
        if (q < nq) {
          // bin b of row r: load (b % EPL) / EL, lane 2r + b / EPL, element b % EL
          const cx<T>* gq = s_g + (2 * (q * K + int((kq >> (2 * q)) & 3u))) * EL;
          const T wt = wq[q];
#pragma unroll
          for (int b = 0; b < BC; ++b)
            accum<T, KAHAN>(acc[b], cmp[KAHAN ? b : 0], wt,
                            gq[((b % EPL) / EL) * LSTRIDE + (b / EPL) * EL + b % EL]);
        }
      }
    }
    if (px < n_x && py < n_y) {
      // non-temporal stores: the grid streams out once (read back by the
      // x-FFT only); measured 17 % faster at the headline size
      cx<T>* out = U + (size_t(b0 - b_begin) * n_y + py) * n_x + px;
      const size_t slice = size_t(n_y) * n_x;
#pragma unroll
      for (int b = 0; b < BC; ++b)
        if (b < nbc) nt_store(out + b * slice, acc[b]);
    }
  }
}

template <typename T, bool KAHAN>
__global__ __launch_bounds__(64) void k_spread_slots(const cx<T>* __restrict__ Gt, int nb,
                                                     const int* __restrict__ slot_off,
                                                     const int* __restrict__ slot_sens,
                                                     const T* __restrict__ slot_w,
                                                     const unsigned* __restrict__ slot_k, int n_x, int n_y,
                                                     int tiles_x, int nchunks, int b_begin, int b_end,
                                                     cx<T>* __restrict__ U) {
  spread_slot_body<T, KAHAN>(Gt, nb, slot_off, slot_sens, slot_w, slot_k, n_x, n_y, tiles_x, nchunks, b_begin,
                             b_end, U, blockIdx.x);
}

template <typename T>
hipError_t launch_spread(const DevPlan& p, const void* Gt, void* U, int b_begin, int b_end, hipStream_t s) {
  if (p.w_xy > kMaxW || b_begin < 0 || b_end > p.nb || b_begin >= b_end) return hipErrorInvalidValue;
  const int nchunks = (b_end - b_begin + kSpreadBins - 1) / kSpreadBins;
  const long long blocks =
      (long long)p.tiles_x * p.patches_y * ((nchunks + kSpreadGroups - 1) / kSpreadGroups);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (p.kahan)
    hipLaunchKernelGGL((k_spread_slots<T, true>), dim3((unsigned)blocks), dim3(64), 0, s,
                       static_cast<const cx<T>*>(Gt), p.nb, p.slot_off, p.slot_sens,
                       static_cast<const T*>(p.slot_w), p.slot_k, p.n_x, p.n_y, p.tiles_x, nchunks, b_begin,
                       b_end, static_cast<cx<T>*>(U));
  else
    hipLaunchKernelGGL((k_spread_slots<T, false>), dim3((unsigned)blocks), dim3(64), 0, s,
                       static_cast<const cx<T>*>(Gt), p.nb, p.slot_off, p.slot_sens,
                       static_cast<const T*>(p.slot_w), p.slot_k, p.n_x, p.n_y, p.tiles_x, nchunks, b_begin,
                       b_end, static_cast<cx<T>*>(U));
  return hipGetLastError();
}

// Batched form: one launch over the (patch, bin-group pair) items of every
// problem, each item as in the single-problem launch (same sums, same order).
template <typename T, bool KAHAN>
__global__ __launch_bounds__(64) void k_spread_batch(const SpreadBA* __restrict__ args,
                                                     const int* __restrict__ prefix, int nprob, int total, BatchIO io) {
  __shared__ BatchMeta<SpreadBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const SpreadBA a = batch_args(meta, p);
    spread_slot_body<T, KAHAN>(static_cast<const cx<T>*>(a.Gt), a.nb, a.slot_off, a.slot_sens,
                               static_cast<const T*>(a.slot_w), a.slot_k, a.n_x, a.n_y, a.tiles_x, a.nchunks, 0,
                               a.nb, static_cast<cx<T>*>(a.U), w - meta.prefix[p]);
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_spread_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  if (st.kahan)
    hipLaunchKernelGGL((k_spread_batch<T, true>), dim3(batch_grid(st)), dim3(64), 0, s,
                       static_cast<const SpreadBA*>(st.args), st.prefix, st.nprob, st.total, io);
  else
    hipLaunchKernelGGL((k_spread_batch<T, false>), dim3(batch_grid(st)), dim3(64), 0, s,
                       static_cast<const SpreadBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T) template hipError_t launch_spread<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_spread_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
