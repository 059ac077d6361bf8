// Helpers shared by the gfx950 stage kernels: FFT work-group shape, the
// in-LDS transform of a batch of sequences, dynamic-LDS opt-in and the
// device view of an FFT plan.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <utility>

#include "fft_device.hpp"
#include "kernels.hpp"

namespace patk {

constexpr int kFftMaxV = 16;    // values per thread in the FFT kernels
constexpr int kFftThreads = 256; // threads per FFT work-group

// Sequences of length n per FFT work-group of nthr threads: at most kFftMaxV
// values per thread, at most `cap`, and (when possible) within 80 KiB of LDS
// so two work-groups share a CU.
template <typename T>
static inline int fft_batch(int n, int nthr, int cap) {
  int b = kFftMaxV * nthr / n;
  const int by_lds = int(81920 / (size_t(lseq(n)) * 2 * sizeof(T)));
  if (b > by_lds) b = by_lds;
  if (b > cap) b = cap;
  return b < 1 ? 1 : b;
}

// Transform the nseq sequences of length fd.n in LDS. Sequences of at most
// 1024 points are each owned by one wave (no work-group barriers inside the
// transform); longer ones use the whole work-group. Callers synchronise the
// work-group before (after filling) and after (before reading).
constexpr int kWaveFftMax = 1024;

// FFT work-group shape: 256 threads, at most 8 sequences per group (measured
// best on MI355X among 128-512 threads and 4-16 sequences, block or wave mode)
constexpr int kFftCap = 8;
struct FftCfg {
  int threads = 256, cap = kFftCap, wave = 0;
};
static inline FftCfg fft_cfg() { return FftCfg{}; }
// The inverse 3-D FFT's x and y passes read and write the half spectrum in
// runs of `cap` consecutive z modes: 16 per group measured faster there.
constexpr int kInvCap = 16;
// z modes per work-group of the gather fused with the inverse x pass: 8
// (19.5 KiB of LDS at 256 points) fits 6 work-groups per CU where 16 fit 4,
// and the gather is bound by instruction issue (0.083 -> 0.077 ms for a
// 256^3 image from 576 band bins; 4 measured 0.088 ms)
constexpr int kGatherCap = 8;
static inline FftCfg inv_cfg() { return FftCfg{256, kInvCap, 0}; }

// Lengths with compile-time FFT instantiations (fft_ct); a launcher calls
// f(std::integral_constant<int, N>) for a listed length and
// f(std::integral_constant<int, 0>) (the runtime plan) otherwise.
template <int... Ns>
struct CtList {};
// sequences of length n a 256-thread group can hold, capped
__host__ __device__ constexpr int ct_maxb(int n, int cap) {
  return n > 0 && kFftMaxV * kFftThreads / n < cap ? kFftMaxV * kFftThreads / n : cap;
}
// 256 / 384 / 512 points: 128^3 .. 256^3 images at oversampling 1.5 or 2;
// 288 / 192 / 1920: a 192^3 image at oversampling 1.5 with 1536 samples
using CtLateral = CtList<256, 288, 384, 512>;
using CtInverse = CtList<128, 192, 256, 512>;
using CtTemporal = CtList<1920, 2048, 2560, 4096>;
// the forward model's fused x-FFT + interpolation (instantiated per footprint
// width and strip height as well) keeps the shorter list
using CtFused = CtList<256, 384, 512>;

template <class F>
static inline hipError_t ct_pick(CtList<>, int, F&& f) {
  return f(std::integral_constant<int, 0>{});
}
template <int N0, int... Ns, class F>
static inline hipError_t ct_pick(CtList<N0, Ns...>, int n, F&& f) {
  if (n == N0) return f(std::integral_constant<int, N0>{});
  return ct_pick(CtList<Ns...>{}, n, f);
}

template <typename T, bool INV>
__device__ __forceinline__ void fft_group(cx<T>* buf, const FftDesc<T>& fd, int nseq, int bstride, int tid, int nthr,
                                          int wave_mode) {
  if (wave_mode && fd.n <= kWaveFftMax) {
    const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
    for (int q = wave; q < nseq; q += nwaves) fft_lds<T, 16, INV, true>(buf + q * bstride, fd, 1, bstride, lane, 64);
  } else {
    fft_lds<T, kFftMaxV, INV, false>(buf, fd, nseq, bstride, tid, nthr);
  }
}

// The same transform with its twiddle table read from a copy in LDS (every
// pass reads the table between two barriers; from LDS the reads cost a few
// dozen cycles instead of a cache round trip).
template <typename T>
__device__ __forceinline__ FftDesc<T> lds_twiddles(FftDesc<T> fd, const cx<T>* twl) {
  fd.tw = twl;
  return fd;
}

// Allow a kernel more than the default dynamic LDS when a launch needs it.
// The largest size granted per (kernel, device) is remembered in a fixed
// table, so repeated launches (also inside a stream capture) make no runtime
// call and no host allocation.
static inline hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return hipGetLastError();
  struct Grant {
    const void* fn;
    int dev;
    size_t bytes;
  };
  constexpr int kGrants = 256;
  static Grant granted[kGrants];
  static int used = 0;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  int i = 0;
  while (i < used && !(granted[i].fn == fn && granted[i].dev == dev)) ++i;
  if (i < used && bytes <= granted[i].bytes) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  if (e != hipSuccess) return e;
  if (i == used && used < kGrants) granted[used++] = Grant{fn, dev, 0};
  if (i < used) granted[i].bytes = bytes;  // a full table only means the attribute is set again next time
  return hipSuccess;
}

template <typename T>
static inline FftDesc<T> as_desc(const FftRaw& r) {
  FftDesc<T> d;
  static_assert(sizeof(FftPass) == sizeof(FftPassRaw), "pass layout");
  d.n = r.n;
  d.npass = r.npass;
  d.pass = static_cast<const FftPass*>(r.dpass);
  d.tw = static_cast<const cx<T>*>(r.tw);
  return d;
}

static inline FftView as_view(const FftRaw& r) {
  FftView v;
  v.n = r.n;
  v.npass = r.npass;
  v.pass = r.dpass;
  v.tw = r.tw;
  return v;
}

template <typename T>
__host__ __device__ inline FftDesc<T> view_desc(const FftView& v) {
  FftDesc<T> d;
  d.n = v.n;
  d.npass = v.npass;
  d.pass = static_cast<const FftPass*>(v.pass);
  d.tw = static_cast<const cx<T>*>(v.tw);
  return d;
}

// A batched launch's per-problem arguments and work-item prefix sums, copied
// into LDS once per work-group; each work item then finds its problem with
// an LDS search and takes the arguments into scalar registers (as kernel
// arguments would be), so no work item waits on dependent global loads.
template <class A>
struct BatchMeta {
  int prefix[kGroupMax + 1];
  A args[kGroupMax];
};

template <class A>
__device__ __forceinline__ void batch_meta_load(BatchMeta<A>& m, const A* __restrict__ args,
                                                const int* __restrict__ prefix, int nprob) {
  static_assert(sizeof(A) % 4 == 0, "argument words");
  const int nw = nprob * int(sizeof(A) / 4);
  const int* src = reinterpret_cast<const int*>(args);
  int* dst = reinterpret_cast<int*>(m.args);
  for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i <= nprob; i += blockDim.x) m.prefix[i] = prefix[i];
  __syncthreads();
}

template <class A>
__device__ __forceinline__ A batch_args(const BatchMeta<A>& m, int p) {
  A a;
  const int* src = reinterpret_cast<const int*>(&m.args[p]);
  int* dst = reinterpret_cast<int*>(&a);
#pragma unroll
  for (int i = 0; i < int(sizeof(A) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return a;
}

// Linear index of this work-group in a 2-D grid with the hardware's
// round-robin placement over the 8 XCDs undone: work-groups with consecutive
// results run on the same XCD and share its L2 (a partial tail keeps its
// own order).
__device__ __forceinline__ int xcd_linear() {
  const int b = blockIdx.x + gridDim.x * blockIdx.y;
  const int per = int(gridDim.x * gridDim.y) / 8;
  return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

// Problem of batched work item w: the largest p with prefix[p] <= w.
__device__ __forceinline__ int batch_locate(const int* prefix, int nprob, int w) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// LDS slots of a complex-to-real z work-group of `rows` real rows: two rows
// share one complex sequence, then the n twiddles.
__host__ __device__ constexpr int c2r_lds_slots(int rows, int n) { return (rows + 1) / 2 * lseq(n) + n; }
// complex pairs staged per thread in a runtime-length complex-to-real z pass:
// (rows + 1) / 2 pairs of n / 2 + 1 values with rows * n <= kFftMaxV * 256
// stay within 8 * 256 for every n <= 2048 (at most 1366; 1032 at n = 256)
constexpr int kC2rStage = 8;

// LDS slots of one temporal work-group (a sensor pair): the sequence, then
// the split twiddle tables (single-problem and batched launches).
__host__ __device__ constexpr int temporal_lds_slots(int n_t) { return lseq(n_t) + tw_split_slots(n_t); }

// The lane index, re-read inside a batched stage's persistent loop: values
// computed from it are then not hoisted out of the loop, where they stayed
// live across every work item (the batched temporal FFT held 94 registers
// against 72 for one item, 2 instead of 3 work-groups per CU).
__device__ __forceinline__ int loop_lane() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Work item of a batched launch's slot L = blockIdx.x + i * gridDim.x (the
// i-th pass of a persistent grid). The hardware places work-groups on the 8
// XCDs round-robin, so with a grid that is a multiple of 8 slots L and L + 8
// share an XCD; items 2m and 2m + 1 (neighbouring blocks of one problem,
// which write the two halves of the same 128-byte lines) are given such a
// pair of slots, so that XCD's L2 merges the halves. A bijection on
// [0, total): the last total mod 16 items keep their slots.
__device__ __forceinline__ int batch_item(int L, int total) {
  if (L >= (total & ~15)) return L;
  const int r = L & 15;
  return (L & ~15) + 2 * (r & 7) + (r >> 3);
}

// Grid of a batched launch: one block per work item, or `st.grid` blocks
// striding over the items.
static inline unsigned batch_grid(const BatchStage& st) {
  return unsigned(st.grid > 0 && st.grid < st.total ? st.grid : st.total);
}

}  // namespace patk
