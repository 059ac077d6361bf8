// Temporal stage of the reconstruction: the equispaced part of the
// non-equispaced-range NUFFT in time (Section 3.1), per sensor.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
// Stage 0: temporal FFT per sensor (the equispaced half of eq. NER_NUFFT).
// Two real traces share one complex FFT (re = sensor m0, im = sensor m1).
// Sample n sits at index (n - n0) mod n_t after multiplication by
// h_m*dt/phihat_t((n - n0)/n_t) (hw == nullptr: unit weight instead of
// h_m*dt); bins b_lo .. b_lo+nb-1 are kept per sensor. The transform's
// twiddles come from the split tables (TwSplit) in LDS behind the sequence:
// the full 2560-point table in LDS cost work-groups per CU, read from global
// memory it left every pass waiting on it (0.096 -> 0.083 ms at 2560 points).
// ---------------------------------------------------------------------------

constexpr int kTemporalThreads = 512;
// compile-time lengths (at most 4096 points): 256 threads, 16 values each,
// measured 5 % faster than 512 at 2560 points
constexpr int kTemporalCtThreads = 256;
template <int NCT>
constexpr int temporal_threads() { return NCT > 0 ? kTemporalCtThreads : kTemporalThreads; }

template <typename T, int NCT = 0>
__device__ __forceinline__ void temporal_body(const T* __restrict__ g, int M, int Nt, int n0,
                                              const T* __restrict__ hw, const T* __restrict__ deap,
                                              FftDesc<T> fd, int b_lo, int nb, cx<T>* __restrict__ Gt, int bx,
                                              int tid = threadIdx.x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nthr = blockDim.x;
  const int n_t = fd.n;
  const int m0 = 2 * bx;  // the pair's first sensor (one pair per group measured fastest on MI355X)
  const bool has1 = m0 + 1 < M;
  // zero padding: only the slots no sample lands in, (n - n0) mod n_t for
  // n = Nt .. n_t-1; they are disjoint from the samples' slots, so the fill
  // and the sample stores need no barrier between them
  for (int i = tid; i < n_t - Nt; i += nthr) {
    int pos = Nt + i - n0;
    if (pos < 0) pos += n_t;
    buf[lpos(pos)] = cx<T>{T(0), T(0)};
  }
  const TwSplit<T> tw = tw_split_fill(buf + lseq(n_t), fd.tw, n_t, tid, nthr);
  const T w0 = hw ? hw[m0] : T(1);
  const T w1 = has1 ? (hw ? hw[m0 + 1] : T(1)) : T(0);
  const T* g0 = g + size_t(m0) * Nt;
  const T* g1 = g + size_t(has1 ? m0 + 1 : m0) * Nt;
  staged_copy<kFftMaxV>(
      Nt, tid, nthr,
      [&](int n) {
        const T d = deap[n];
        const T a = g0[n] * w0 * d;
        const T b = has1 ? g1[n] * w1 * d : T(0);
        return cx<T>{a, b};
      },
      [&](int n, cx<T> v) {
        int pos = n - n0;
        if (pos < 0) pos += n_t;
        buf[lpos(pos)] = v;
      });
  __syncthreads();
  if constexpr (NCT > 0)
    fft_ct_tw<T, NCT, temporal_threads<NCT>(), 1, false>(buf, 1, tw, tid);
  else
    fft_lds_tw<T, kFftMaxV, false, false>(buf, fd, tw, 1, lseq(n_t), tid, nthr);
  for (int i = tid; i < nb; i += nthr) {
    const int b = b_lo + i;  // -n_t < b < n_t (the band fits in n_t bins)
    const int pb = b < 0 ? b + n_t : b;
    const int mb = b > 0 ? n_t - b : -b;
    const cx<T> z = buf[lpos(pb)];
    const cx<T> zm = buf[lpos(mb)];
    // transform of the real part: (Z_b + conj Z_-b)/2; of the imaginary part: (Z_b - conj Z_-b)/(2i)
    Gt[size_t(m0) * nb + i] = cx<T>{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
    if (has1) Gt[size_t(m0 + 1) * nb + i] = cx<T>{T(0.5) * (z.y + zm.y), T(-0.5) * (z.x - zm.x)};
  }
}

template <typename T, int NCT>
__global__ __launch_bounds__(temporal_threads<NCT>()) void k_temporal(const T* __restrict__ g, int M, int Nt, int n0,
                                                             const T* __restrict__ hw, const T* __restrict__ deap,
                                                             FftDesc<T> fd, int b_lo, int nb,
                                                             cx<T>* __restrict__ Gt) {
  temporal_body<T, NCT>(g, M, Nt, n0, hw, deap, fd, b_lo, nb, Gt, blockIdx.x);
}

template <typename T>
hipError_t launch_temporal(const DevPlan& p, const T* g, void* Gt, bool weighted, hipStream_t s) {
  if (p.n_t > kFftMaxV * kTemporalThreads || p.Nt > p.n_t) return hipErrorInvalidValue;
  const int blocks = (p.M + 1) / 2;  // one sensor pair per group
  const size_t lds = size_t(temporal_lds_slots(p.n_t)) * sizeof(cx<T>);
  return ct_pick(CtTemporal{}, p.n_t, [&](auto c) {
    constexpr int NCT = decltype(c)::value, NT = temporal_threads<NCT>();
    static_assert(NCT <= kFftMaxV * NT, "a thread holds at most kFftMaxV values");
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_temporal<T, NCT>), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_temporal<T, NCT>), dim3(blocks), dim3(NT), lds, s, g, p.M,
                       p.Nt, p.n0, weighted ? static_cast<const T*>(p.hw) : nullptr, static_cast<const T*>(p.deap),
                       as_desc<T>(p.f_nt), p.b_lo, p.nb, static_cast<cx<T>*>(Gt));
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------------------
// Transpose of k_temporal with unit weights (the forward model's last step):
//   g[m][n] = a_n Re sum_b Gt'[m][b] exp(+2 pi i b (n - n0)/n_t),
// a_n = 1/phihat_t((n - n0)/n_t). Two sensors share one inverse FFT: the
// spectrum Z[k] = (X0[k] + conj X0[-k])/2 + i (X1[k] + conj X1[-k])/2 (band
// bins placed at b mod n_t) transforms to Re x0 + i Re x1. The band never
// covers a bin twice (nb <= n_t), so each of the two placement passes
// writes distinct slots.
// ---------------------------------------------------------------------------
template <typename T, int NCT>
__global__ __launch_bounds__(temporal_threads<NCT>()) void k_temporal_t(const cx<T>* __restrict__ Gt, int M, int Nt, int n0,
                                                               const T* __restrict__ deap, FftDesc<T> fd, int b_lo,
                                                               int nb, T* __restrict__ g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_t = fd.n;
  const int m0 = 2 * blockIdx.x;
  const bool has1 = m0 + 1 < M;
  for (int q = tid; q < n_t; q += nthr) buf[lpos(q)] = cx<T>{T(0), T(0)};
  const TwSplit<T> tw = tw_split_fill(buf + lseq(n_t), fd.tw, n_t, tid, nthr);
  __syncthreads();
  const cx<T>* x0 = Gt + size_t(m0) * nb;
  const cx<T>* x1 = Gt + size_t(m0 + 1) * nb;
  const cx<T> zero{T(0), T(0)};
  for (int i = tid; i < nb; i += nthr) {
    const int b = b_lo + i;
    const int pb = b < 0 ? b + n_t : b;
    const cx<T> a = x0[i], c = has1 ? x1[i] : zero;
    buf[lpos(pb)] = cx<T>{T(0.5) * (a.x - c.y), T(0.5) * (a.y + c.x)};
  }
  __syncthreads();
  for (int i = tid; i < nb; i += nthr) {
    const int b = b_lo + i;
    const int mb = b > 0 ? n_t - b : -b;
    const cx<T> a = x0[i], c = has1 ? x1[i] : zero;
    cx<T>& z = buf[lpos(mb)];
    z = cx<T>{z.x + T(0.5) * (a.x + c.y), z.y + T(0.5) * (c.x - a.y)};
  }
  __syncthreads();
  if constexpr (NCT > 0)
    fft_ct_tw<T, NCT, temporal_threads<NCT>(), 1, true>(buf, 1, tw, tid);
  else
    fft_lds_tw<T, kFftMaxV, true, false>(buf, fd, tw, 1, lseq(n_t), tid, nthr);
  __syncthreads();
  for (int n = tid; n < Nt; n += nthr) {
    int pos = n - n0;
    if (pos < 0) pos += n_t;
    const cx<T> z = buf[lpos(pos)];
    const T d = deap[n];
    // the caller's traces: non-temporal stores (measured faster)
    __builtin_nontemporal_store(z.x * d, g + size_t(m0) * Nt + n);
    if (has1) __builtin_nontemporal_store(z.y * d, g + size_t(m0 + 1) * Nt + n);
  }
}

template <typename T>
hipError_t launch_temporal_t(const DevPlan& p, const void* Gt, T* g, hipStream_t s) {
  if (p.n_t > kFftMaxV * kTemporalThreads || p.Nt > p.n_t || p.nb > p.n_t) return hipErrorInvalidValue;
  const size_t lds = size_t(temporal_lds_slots(p.n_t)) * sizeof(cx<T>);
  return ct_pick(CtTemporal{}, p.n_t, [&](auto c) {
    constexpr int NCT = decltype(c)::value, NT = temporal_threads<NCT>();
    static_assert(NCT <= kFftMaxV * NT, "a thread holds at most kFftMaxV values");
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_temporal_t<T, NCT>), lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_temporal_t<T, NCT>), dim3((p.M + 1) / 2), dim3(NT), lds, s,
                       static_cast<const cx<T>*>(Gt), p.M, p.Nt, p.n0, static_cast<const T*>(p.deap),
                       as_desc<T>(p.f_nt), p.b_lo, p.nb, g);
    return hipGetLastError();
  });
}

// Batched form: one launch over the sensor pairs of every problem.
template <typename T>
__global__ __launch_bounds__(kTemporalThreads) void k_temporal_batch(const TemporalBA* __restrict__ args,
                                                                     const int* __restrict__ prefix, int nprob, int total,
                                                                     BatchIO io) {
  __shared__ BatchMeta<TemporalBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const TemporalBA a = batch_args(meta, p);
    temporal_body<T>(static_cast<const T*>(io.in[p]), a.M, a.Nt, a.n0, static_cast<const T*>(a.hw),
                     static_cast<const T*>(a.deap), view_desc<T>(a.fd), a.b_lo, a.nb, static_cast<cx<T>*>(a.Gt),
                     w - meta.prefix[p], loop_lane());
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_temporal_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_temporal_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_temporal_batch<T>), dim3(batch_grid(st)), dim3(kTemporalThreads), st.lds, s,
                     static_cast<const TemporalBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T)                                                                      \
  template hipError_t launch_temporal<T>(const DevPlan&, const T*, void*, bool, hipStream_t); \
  template hipError_t launch_temporal_t<T>(const DevPlan&, const void*, T*, hipStream_t); \
  template hipError_t launch_temporal_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
