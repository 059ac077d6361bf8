// Lateral gridding of the non-equispaced-data NUFFT over the sensor plane
// (Section 3.2), one chunk of temporal bins at a time.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
// Stage 1: lateral spreading (the gridding of eq. NED_NUFFT), one chunk of
// temporal bins at a time. Output-driven and atomic-free: every lane owns one
// grid point and accumulates in registers the contributions of a sensor list
// in list order (deterministic). Tile form (used by batched launches): a
// work-group owns a 16x16 tile of the oversampled grid (four waves, each a
// 16x4 patch) and the tile's sensor list.
// The list is staged through LDS in batches (sensor footprint origin,
// per-axis weights, the chunk's bin values), so the inner loop reads only
// LDS: the bin values are wave-uniform broadcasts and the lane's weight is
// wx[tx]*wy[ty] (0 outside the footprint).
// ---------------------------------------------------------------------------
constexpr int kSpreadBins = 16;
constexpr int kSpreadBatch = 64;
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

template <typename T, bool KAHAN, int BC = kSpreadBins>
__device__ __forceinline__ void spread_body(const cx<T>* __restrict__ Gt, int nb, const int* __restrict__ tile_off,
                                            const int* __restrict__ tile_sens, const int* __restrict__ sbx,
                                            const int* __restrict__ sby, const T* __restrict__ swx,
                                            const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                            int nchunks, int b_begin, int b_end, cx<T>* __restrict__ U, int bx) {
  constexpr int SB = kSpreadBatch;
  constexpr int BPT = BC / 4;  // bins staged per thread
  __shared__ int s_bx[SB], s_by[SB];
  __shared__ T s_wx[SB * kMaxW], s_wy[SB * kMaxW];
  __shared__ cx<T> s_g[SB * BC];
  // bin groups vary fastest: groups running together share one tile's sensor
  // list and read whole per-sensor rows of Gt (measured faster on MI355X than
  // ordering by tile)
  const int chunk = bx % nchunks;
  const int tile = bx / nchunks;
  const int tyi = tile / tiles_x;
  const int txi = tile - tyi * tiles_x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int px = txi * kSpreadTile + (lane & 15);
  const int prow0 = tyi * kSpreadTile + wave * 4;
  const int py = prow0 + (lane >> 4);
  const int b0 = b_begin + chunk * BC;  // first bin of this group; U holds bins from b_begin on
  const int nbc = min(BC, b_end - b0);
  cx<T> acc[BC];
  cx<T> cmp[KAHAN ? BC : 1];
#pragma unroll
  for (int b = 0; b < BC; ++b) acc[b] = cx<T>{T(0), T(0)};
#pragma unroll
  for (int b = 0; b < (KAHAN ? BC : 1); ++b) cmp[b] = cx<T>{T(0), T(0)};
  const int q_begin = tile_off[tile];
  const int q_end = tile_off[tile + 1];
  for (int qb = q_begin; qb < q_end; qb += SB) {
    const int nq = min(SB, q_end - qb);
    __syncthreads();  // the previous batch has been consumed
    {
      // four threads per staged sensor: one read of the sensor index, then every
      // table and bin load of that sensor issued together
      static_assert(SB * 4 == 256 && kMaxW == 16 && BC % 4 == 0, "staging layout");
      const int qi = tid >> 2, r = tid & 3;
      if (qi < nq) {
        const int sidx = tile_sens[qb + qi];
        const T* wxs = swx + size_t(sidx) * w;
        const T* wys = swy + size_t(sidx) * w;
        const cx<T>* gs = Gt + size_t(sidx) * nb + b0;
        T vx[4], vy[4];
        cx<T> vg[BPT];
        int bxv = 0, byv = 0;
        if (r == 0) {
          bxv = sbx[sidx];
          byv = sby[sidx];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = r * 4 + i;
          vx[i] = e < w ? wxs[e] : T(0);
          vy[i] = e < w ? wys[e] : T(0);
        }
#pragma unroll
        for (int i = 0; i < BPT; ++i) {
          const int e = r * BPT + i;
          vg[i] = e < nbc ? gs[e] : cx<T>{T(0), T(0)};
        }
        if (r == 0) {
          s_bx[qi] = bxv;
          s_by[qi] = byv;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          s_wx[qi * kMaxW + r * 4 + i] = vx[i];
          s_wy[qi * kMaxW + r * 4 + i] = vy[i];
        }
#pragma unroll
        for (int i = 0; i < BPT; ++i) s_g[qi * BC + r * BPT + i] = vg[i];
      }
    }
    __syncthreads();
    for (int qi = 0; qi < nq; ++qi) {
      const int by = s_by[qi];
      int d0 = prow0 - by;
      if (d0 < 0) d0 += n_y;
      if (!(d0 < w || d0 + 3 >= n_y)) continue;  // footprint misses this wave's four rows
      int tx = px - s_bx[qi];
      if (tx < 0) tx += n_x;
      int ty = py - by;
      if (ty < 0) ty += n_y;
      const T wt = (tx < w && ty < w) ? s_wx[qi * kMaxW + tx] * s_wy[qi * kMaxW + ty] : T(0);
      const cx<T>* gq = s_g + qi * BC;
#pragma unroll
      for (int b = 0; b < BC; ++b) accum<T, KAHAN>(acc[b], cmp[KAHAN ? b : 0], wt, gq[b]);
    }
  }
  if (px < n_x && py < n_y) {
    cx<T>* out = U + (size_t(b0 - b_begin) * n_y + py) * n_x + px;
    const size_t slice = size_t(n_y) * n_x;
#pragma unroll
    for (int b = 0; b < BC; ++b)
      if (b < nbc) out[b * slice] = acc[b];
  }
}

// One-wave form: a 64-thread work-group owns a 16 x kPatchRows patch of the
// grid for one bin group and walks only the sensors whose footprint meets
// that patch (its own list), so no wave iterates over sensors that miss its
// rows. Per grid point the contributing sensors and their order are those of
// spread_body, so the results are identical. Measured on MI355X (headline
// size) about 1 % faster than the tile form; staging 32 or 64 sensors per
// round, or an XCD-contiguous block order, measured slower.
constexpr int kWaveBatch = 16;  // sensors staged per round (four threads each)

template <typename T, bool KAHAN, int SB>
__device__ __forceinline__ void spread_wave_body(const cx<T>* __restrict__ Gt, int nb,
                                                 const int* __restrict__ patch_off,
                                                 const int* __restrict__ patch_sens, const int* __restrict__ sbx,
                                                 const int* __restrict__ sby, const T* __restrict__ swx,
                                                 const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                                 int nchunks, int b_begin, int b_end, cx<T>* __restrict__ U, int bx) {
  constexpr int BC = kSpreadBins;
  constexpr int SPT = SB / 16;  // sensors staged per group of four threads
  static_assert(SB % 16 == 0 && kMaxW == 16 && BC == 16, "staging layout");
  __shared__ int s_bx[SB], s_by[SB];
  __shared__ T s_wx[SB * kMaxW], s_wy[SB * kMaxW];
  __shared__ cx<T> s_g[SB * BC];
  const int chunk = bx % nchunks;  // bin groups vary fastest, as in spread_body
  const int patch = bx / nchunks;
  const int prg = patch / tiles_x;
  const int pcol = patch - prg * tiles_x;
  const int lane = threadIdx.x;
  const int px = pcol * kSpreadTile + (lane & 15);
  const int py = prg * kPatchRows + (lane >> 4);
  const int b0 = b_begin + chunk * BC;
  const int nbc = min(BC, b_end - b0);
  cx<T> acc[BC];
  cx<T> cmp[KAHAN ? BC : 1];
#pragma unroll
  for (int b = 0; b < BC; ++b) acc[b] = cx<T>{T(0), T(0)};
#pragma unroll
  for (int b = 0; b < (KAHAN ? BC : 1); ++b) cmp[b] = cx<T>{T(0), T(0)};
  const int q_begin = patch_off[patch];
  const int q_end = patch_off[patch + 1];
  const int qi = lane >> 2, r = lane & 3;
  for (int qb = q_begin; qb < q_end; qb += SB) {
    const int nq = min(SB, q_end - qb);
    __syncthreads();  // the previous batch has been consumed
    // every thread issues the loads of its SPT sensors before any LDS store
    int sidx[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) sidx[k] = qi + 16 * k < nq ? patch_sens[qb + qi + 16 * k] : 0;
    T vx[SPT][4], vy[SPT][4];
    cx<T> vg[SPT][4];
    int bxv[SPT], byv[SPT];
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const bool ok = qi + 16 * k < nq;
      const T* wxs = swx + size_t(sidx[k]) * w;
      const T* wys = swy + size_t(sidx[k]) * w;
      const cx<T>* gs = Gt + size_t(sidx[k]) * nb + b0;
      bxv[k] = ok && r == 0 ? sbx[sidx[k]] : 0;
      byv[k] = ok && r == 0 ? sby[sidx[k]] : 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = r * 4 + i;
        vx[k][i] = ok && e < w ? wxs[e] : T(0);
        vy[k][i] = ok && e < w ? wys[e] : T(0);
        vg[k][i] = ok && e < nbc ? gs[e] : cx<T>{T(0), T(0)};
      }
    }
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const int qk = qi + 16 * k;
      if (qk < nq) {
        if (r == 0) {
          s_bx[qk] = bxv[k];
          s_by[qk] = byv[k];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          s_wx[qk * kMaxW + r * 4 + i] = vx[k][i];
          s_wy[qk * kMaxW + r * 4 + i] = vy[k][i];
          s_g[qk * BC + r * 4 + i] = vg[k][i];
        }
      }
    }
    __syncthreads();
    for (int q = 0; q < nq; ++q) {
      int tx = px - s_bx[q];
      if (tx < 0) tx += n_x;
      int ty = py - s_by[q];
      if (ty < 0) ty += n_y;
      const T wt = (tx < w && ty < w) ? s_wx[q * kMaxW + tx] * s_wy[q * kMaxW + ty] : T(0);
      const cx<T>* gq = s_g + q * BC;
#pragma unroll
      for (int b = 0; b < BC; ++b) accum<T, KAHAN>(acc[b], cmp[KAHAN ? b : 0], wt, gq[b]);
    }
  }
  if (px < n_x && py < n_y) {
    cx<T>* out = U + (size_t(b0 - b_begin) * n_y + py) * n_x + px;
    const size_t slice = size_t(n_y) * n_x;
#pragma unroll
    for (int b = 0; b < BC; ++b)
      if (b < nbc) out[b * slice] = acc[b];
  }
}

template <typename T, bool KAHAN, int SB>
__global__ __launch_bounds__(64) void k_spread_wave(const cx<T>* __restrict__ Gt, int nb,
                                                    const int* __restrict__ patch_off,
                                                    const int* __restrict__ patch_sens, const int* __restrict__ sbx,
                                                    const int* __restrict__ sby, const T* __restrict__ swx,
                                                    const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                                    int nchunks, int b_begin, int b_end, cx<T>* __restrict__ U) {
  spread_wave_body<T, KAHAN, SB>(Gt, nb, patch_off, patch_sens, sbx, sby, swx, swy, w, n_x, n_y, tiles_x, nchunks,
                             b_begin, b_end, U, blockIdx.x);
}

template <typename T, int SB>
static hipError_t launch_spread_wave(const DevPlan& p, const void* Gt, void* U, int b_begin, int b_end,
                                     hipStream_t s) {
  const int nchunks = (b_end - b_begin + kSpreadBins - 1) / kSpreadBins;
  const long long blocks = (long long)p.tiles_x * p.patches_y * nchunks;
  if (p.kahan)
    hipLaunchKernelGGL((k_spread_wave<T, true, SB>), dim3((unsigned)blocks), dim3(64), 0, s,
                       static_cast<const cx<T>*>(Gt), p.nb, p.patch_off, p.patch_sens, p.sbx, p.sby,
                       static_cast<const T*>(p.swx), static_cast<const T*>(p.swy), p.w_xy, p.n_x, p.n_y, p.tiles_x,
                       nchunks, b_begin, b_end, static_cast<cx<T>*>(U));
  else
    hipLaunchKernelGGL((k_spread_wave<T, false, SB>), dim3((unsigned)blocks), dim3(64), 0, s,
                       static_cast<const cx<T>*>(Gt), p.nb, p.patch_off, p.patch_sens, p.sbx, p.sby,
                       static_cast<const T*>(p.swx), static_cast<const T*>(p.swy), p.w_xy, p.n_x, p.n_y, p.tiles_x,
                       nchunks, b_begin, b_end, static_cast<cx<T>*>(U));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spread(const DevPlan& p, const void* Gt, void* U, int b_begin, int b_end, hipStream_t s) {
  if (p.w_xy > kMaxW || b_begin < 0 || b_end > p.nb || b_begin >= b_end) return hipErrorInvalidValue;
  return launch_spread_wave<T, kWaveBatch>(p, Gt, U, b_begin, b_end, s);
}

// Batched form: one launch over the (tile, bin group) items of every problem.
template <typename T, bool KAHAN>
__global__ __launch_bounds__(256) void k_spread_batch(const SpreadBA* __restrict__ args, const int* __restrict__ prefix,
                             int nprob, int total, BatchIO io) {
  __shared__ BatchMeta<SpreadBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int w = blockIdx.x; w < total; w += gridDim.x) {
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const SpreadBA a = batch_args(meta, p);
    spread_body<T, KAHAN>(static_cast<const cx<T>*>(a.Gt), a.nb, a.tile_off, a.tile_sens, a.sbx, a.sby,
                          static_cast<const T*>(a.swx), static_cast<const T*>(a.swy), a.w, a.n_x, a.n_y, a.tiles_x,
                          a.nchunks, 0, a.nb, static_cast<cx<T>*>(a.U), w - meta.prefix[p]);
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_spread_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  if (st.kahan)
    hipLaunchKernelGGL((k_spread_batch<T, true>), dim3(batch_grid(st)), dim3(256), 0, s,
                       static_cast<const SpreadBA*>(st.args), st.prefix, st.nprob, st.total, io);
  else
    hipLaunchKernelGGL((k_spread_batch<T, false>), dim3(batch_grid(st)), dim3(256), 0, s,
                       static_cast<const SpreadBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T) template hipError_t launch_spread<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_spread_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
