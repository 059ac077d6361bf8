// Interpolation from the oversampled lateral grid to the sensors: the
// transpose of the lateral gridding (the type-2 counterpart of
// eq. NED_NUFFT), used by the forward model.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
//   Gt'[m][b] = sum_{ty,tx < w} wy_m[ty] wx_m[tx] U'[b][(by_m + ty) mod n_y][(bx_m + tx) mod n_x]
// with the spread's footprint origin and weights. A work-group owns one
// 16x16 home tile (the tile holding the footprint origins of its sensors)
// and `bc` bins: it stages the tile plus a (w-1) halo of those bins in LDS
// (periodic wrap), then one thread per (sensor, bin) pair sums the footprint
// from LDS. Each output is written once; no atomics.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_interp(const cx<T>* __restrict__ U, int nb, const int* __restrict__ home_off,
                                                const int* __restrict__ home_sens, const int* __restrict__ sbx,
                                                const int* __restrict__ sby, const T* __restrict__ swx,
                                                const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                                int nchunks, int bc, int b_begin, int b_end, cx<T>* __restrict__ Gt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* patch = reinterpret_cast<cx<T>*>(smem_raw);
  const int chunk = blockIdx.x % nchunks;
  const int tile = blockIdx.x / nchunks;
  const int q0 = home_off[tile], q1 = home_off[tile + 1];
  if (q0 == q1) return;
  const int tyi = tile / tiles_x;
  const int txi = tile - tyi * tiles_x;
  const int tx0 = txi * kSpreadTile, ty0 = tyi * kSpreadTile;
  const int P = kSpreadTile + w - 1;  // patch edge
  const int PR = P | 1;               // odd row pitch
  const int plane = P * PR;
  const int b0 = b_begin + chunk * bc;
  const int nbc = min(bc, b_end - b0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const size_t slice = size_t(n_y) * n_x;
  const FastDiv div_p(P), div_pp(P * P);
  // stage the patch: each thread issues up to kStage loads before its LDS stores
  constexpr int kStage = 8;
  const int total = nbc * P * P;
  for (int q0s = 0; q0s < total; q0s += kStage * nthr) {
    cx<T> v[kStage];
    int dst[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int q = q0s + tid + u * nthr;
      dst[u] = -1;
      if (q < total) {
        const int bi = div_pp(q);
        const int rem = q - bi * P * P;
        const int r = div_p(rem);
        const int cc = rem - r * P;
        int py = ty0 + r;
        while (py >= n_y) py -= n_y;
        int px = tx0 + cc;
        while (px >= n_x) px -= n_x;
        v[u] = U[size_t(b0 - b_begin + bi) * slice + size_t(py) * n_x + px];
        dst[u] = bi * plane + r * PR + cc;
      }
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u)
      if (dst[u] >= 0) patch[dst[u]] = v[u];
  }
  __syncthreads();
  const int npairs = (q1 - q0) * nbc;  // may exceed 2^16: plain division below
  for (int pq = tid; pq < npairs; pq += nthr) {
    const int qi = pq / nbc;
    const int bi = pq - qi * nbc;
    const int m = home_sens[q0 + qi];
    const int ox = sbx[m] - tx0, oy = sby[m] - ty0;
    const T* wx = swx + size_t(m) * w;
    const T* wy = swy + size_t(m) * w;
    const cx<T>* pp = patch + bi * plane + oy * PR + ox;
    cx<T> acc{T(0), T(0)};
    for (int ty = 0; ty < w; ++ty) {
      cx<T> row{T(0), T(0)};
      for (int tx = 0; tx < w; ++tx) {
        const cx<T> v = pp[ty * PR + tx];
        row.x += wx[tx] * v.x;
        row.y += wx[tx] * v.y;
      }
      acc.x += wy[ty] * row.x;
      acc.y += wy[ty] * row.y;
    }
    Gt[size_t(m) * nb + b0 + bi] = acc;
  }
}

// bins per work-group: the largest of 8, 4, 2, 1 whose patch fits 40 KiB
// (four work-groups per CU)
template <typename T>
static int interp_bins(int w) {
  const int P = kSpreadTile + w - 1;
  const size_t plane = size_t(P) * (P | 1) * sizeof(cx<T>);
  int bc = 8;
  while (bc > 1 && plane * bc > 40960) bc >>= 1;
  return bc;
}

template <typename T>
hipError_t launch_interp(const DevPlan& p, const void* U, void* Gt, int b_begin, int b_end, hipStream_t s) {
  if (p.w_xy > 16 || b_begin < 0 || b_end > p.nb || b_begin >= b_end) return hipErrorInvalidValue;
  const int bc = interp_bins<T>(p.w_xy);
  const int P = kSpreadTile + p.w_xy - 1;
  const size_t lds = size_t(P) * (P | 1) * sizeof(cx<T>) * bc;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_interp<T>), lds);
  if (e != hipSuccess) return e;
  const int nchunks = (b_end - b_begin + bc - 1) / bc;
  const long long blocks = (long long)p.tiles_x * p.tiles_y * nchunks;
  hipLaunchKernelGGL(k_interp<T>, dim3((unsigned)blocks), dim3(256), lds, s, static_cast<const cx<T>*>(U), p.nb,
                     p.home_off, p.home_sens, p.sbx, p.sby, static_cast<const T*>(p.swx), static_cast<const T*>(p.swy),
                     p.w_xy, p.n_x, p.n_y, p.tiles_x, nchunks, bc, b_begin, b_end, static_cast<cx<T>*>(Gt));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused form of k_fft_x_t followed by k_interp: the oversampled grid U' never
// goes to memory. A work-group owns one strip of FS*kSpreadTile grid rows (FS
// rows of home tiles; two where the LDS holds them, with 1024 threads, else
// one with 512) and a run of bins. Per bin it loads the strip's rows plus a
// (W-1)-row halo of V' (periodic in y), embeds the Nx kept modes of every row
// into n_x slots, inverse-FFTs the rows in LDS (one wave per row), then
// interpolates every sensor whose footprint origin lies in the strip straight
// from LDS. Per sensor the footprint sum runs in the same order as k_interp
// and the row transforms take the same passes as k_fft_x_t, so the two forms
// agree to rounding.
// ---------------------------------------------------------------------------
constexpr int kFusedThreads = 512;  // per home-tile row of the strip
constexpr int kFusedBins = 8;       // most bins per work-group
// sensors per thread whose bins are held in registers: as many as fit the
// register budget without spills (FP32 footprints up to 8 or 12 points)
template <typename T, int W>
__host__ __device__ constexpr int fused_held() {
  return sizeof(T) == 4 ? (W <= 8 ? 2 : (W <= 12 ? 1 : 0)) : 0;
}

template <int W, int FS>
__host__ __device__ constexpr int fused_rows() { return FS * kSpreadTile + W - 1; }

// One sensor of the strip: footprint origin row within the strip, the LDS
// slots of its footprint columns, and its weights.
template <typename T, int W>
struct FusedSensor {
  int m, oy;
  int col[W];
  T wx[W], wy[W];
};

template <typename T, int W>
__device__ __forceinline__ void fused_sensor_load(FusedSensor<T, W>& f, int m, int py0, int n_x,
                                                  const int* __restrict__ sbx, const int* __restrict__ sby,
                                                  const T* __restrict__ swx, const T* __restrict__ swy) {
  f.m = m;
  const int ox = sbx[m];
  f.oy = sby[m] - py0;
#pragma unroll
  for (int t = 0; t < W; ++t) {
    f.wx[t] = swx[size_t(m) * W + t];
    f.wy[t] = swy[size_t(m) * W + t];
    int c = ox + t;
    if (c >= n_x) c -= n_x;
    f.col[t] = lpos(c);
  }
}

// footprint sum in k_interp's order: rows of x-weighted sums, then y weights
template <typename T, int W>
__device__ __forceinline__ cx<T> fused_sensor_sum(const FusedSensor<T, W>& f, const cx<T>* buf, int bstride) {
  const cx<T>* rows = buf + f.oy * bstride;
  cx<T> acc{T(0), T(0)};
#pragma unroll
  for (int ty = 0; ty < W; ++ty) {
    cx<T> row{T(0), T(0)};
#pragma unroll
    for (int tx = 0; tx < W; ++tx) {
      const cx<T> v = rows[ty * bstride + f.col[tx]];
      row.x += f.wx[tx] * v.x;
      row.y += f.wx[tx] * v.y;
    }
    acc.x += f.wy[ty] * row.x;
    acc.y += f.wy[ty] * row.y;
  }
  return acc;
}

template <typename T, int W, int MAXV, int NCT, int FS>
__global__ __launch_bounds__(kFusedThreads * FS) void k_fft_x_interp(
    const cx<T>* __restrict__ V, int nb, int Nx, int n_y, int tiles_x, int nchunks, int bins,
    const int* __restrict__ home_off, const int* __restrict__ home_sens, const int* __restrict__ sbx,
    const int* __restrict__ sby, const T* __restrict__ swx, const T* __restrict__ swy, FftDesc<T> fd,
    const int* __restrict__ brange, cx<T>* __restrict__ Gt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int R = fused_rows<W, FS>();
  const int chunk = blockIdx.x % nchunks;  // bins vary fastest: neighbouring groups share the strip's sensors
  const int strip = blockIdx.x / nchunks;
  const int tiles_y = (n_y + kSpreadTile - 1) / kSpreadTile;
  const int q0 = home_off[strip * FS * tiles_x], q1 = home_off[min(strip * FS + FS, tiles_y) * tiles_x];
  if (q0 == q1) return;
  const int n_x = fd.n;
  const int bstride = lseq(n_x);
  const int py0 = strip * FS * kSpreadTile;
  const int b0 = chunk * bins, b1 = min(nb, b0 + bins);
  const int gap = n_x - Nx;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nthr >> 6;
  const FastDiv div_gap(gap > 0 ? gap : 1), div_r(R);
  const size_t plane = size_t(Nx) * n_y;
  const int total = R * Nx;
  // grid row of each strip row (periodic in y; short axes wrap more than once)
  constexpr int HELD = fused_held<T, W>();
  cx<T> held[HELD > 0 ? HELD : 1][kFusedBins];
  __shared__ int s_row[R];
  for (int r = tid; r < R; r += nthr) s_row[r] = (py0 + r) % n_y;
  __syncthreads();  // every wave reads the table in the first bin's staging loop
  for (int b = b0; b < b1; ++b) {
    for (int q = tid; q < R * gap; q += nthr) {
      const int r = div_gap(q);
      buf[r * bstride + lpos(Nx / 2 + (q - r * gap))] = cx<T>{T(0), T(0)};
    }
    // element q of the strip: mode jj = q / R of grid row py0 + q mod R (periodic
    // in y); x-modes outside [J0, J1] for this bin are zero (not written)
    const cx<T>* src = V + size_t(b) * plane;
    const int J0 = brange ? brange[2 * b] : 0, J1 = brange ? brange[2 * b + 1] : Nx;
    constexpr int kStage = 8;
    for (int qs = 0; qs < total; qs += kStage * nthr) {
      cx<T> v[kStage];
      int dst[kStage];
      bool ok[kStage];
      // every lane loads (lanes outside the window all read element 0, one
      // line), so the loads stay in flight together; zeros are chosen at the store
#pragma unroll
      for (int u = 0; u < kStage; ++u) {
        const int q = qs + tid + u * nthr;
        const bool in = q < total;
        const int qc = in ? q : 0;  // straight-line code: the loads stay back to back
        const int jj = div_r(qc);
        const int r = qc - jj * R;
        const int py = s_row[r];
        const int j = jj < Nx / 2 ? jj : jj - Nx;
        const int aj = j < 0 ? -j : j;
        ok[u] = in && aj >= J0 && aj <= J1;
        v[u] = src[ok[u] ? size_t(jj) * n_y + py : 0];
        dst[u] = in ? r * bstride + lpos(j < 0 ? j + n_x : j) : -1;
      }
#pragma unroll
      for (int u = 0; u < kStage; ++u)
        if (dst[u] >= 0) buf[dst[u]] = ok[u] ? v[u] : cx<T>{T(0), T(0)};
    }
    __syncthreads();
    for (int r = wave; r < R; r += nwaves) {
      if constexpr (NCT > 0)
        fft_ct<T, NCT, 64, 1, true, true>(buf + r * bstride, 1, fd.tw, lane);
      else
        fft_lds<T, MAXV, true, true>(buf + r * bstride, fd, 1, bstride, lane, 64);
    }
    __syncthreads();
    // the first HELD sensors of every thread keep their values in
    // registers until the group's last bin (shifted one place per bin), so
    // each sensor's run of bins goes out in one burst instead of as single
    // 8-byte writes to lines the L2 has evicted in between
#pragma unroll
    for (int k = 0; k < HELD; ++k) {
      const int q = q0 + tid + k * nthr;
      cx<T> val{T(0), T(0)};
      if (q < q1) {
        FusedSensor<T, W> f;
        fused_sensor_load<T, W>(f, home_sens[q], py0, n_x, sbx, sby, swx, swy);
        val = fused_sensor_sum<T, W>(f, buf, bstride);
      }
#pragma unroll
      for (int j = 0; j + 1 < kFusedBins; ++j) held[k][j] = held[k][j + 1];
      held[k][kFusedBins - 1] = val;
    }
    for (int q = q0 + tid + HELD * nthr; q < q1; q += nthr) {
      FusedSensor<T, W> f;
      fused_sensor_load<T, W>(f, home_sens[q], py0, n_x, sbx, sby, swx, swy);
      Gt[size_t(f.m) * nb + b] = fused_sensor_sum<T, W>(f, buf, bstride);
    }
    __syncthreads();
  }
  // held[k][j] is bin b0 + j - (kFusedBins - nbin)
  const int nbin = b1 - b0;
#pragma unroll
  for (int k = 0; k < HELD; ++k) {
    const int q = q0 + tid + k * nthr;
    if (q < q1) {
      cx<T>* g = Gt + size_t(home_sens[q]) * nb + b0;  // bin b0 + i is held[k][i + kFusedBins - nbin]
#pragma unroll
      for (int j = 0; j < kFusedBins; ++j)
        if (j >= kFusedBins - nbin) g[j - (kFusedBins - nbin)] = held[k][j];
    }
  }
}

template <typename T>
size_t fused_interp_lds(const DevPlan& p, int strip_tiles) {
  return size_t(strip_tiles * kSpreadTile + p.w_xy - 1) * lseq(p.n_x) * sizeof(cx<T>);
}

template <typename T>
bool fused_interp_ok(const DevPlan& p, size_t lds_limit) {
  return p.n_x <= kWaveFftMax && p.w_xy >= 2 && p.w_xy <= 16 && (p.w_xy % 2) == 0 && p.Nx <= p.n_x &&
         fused_interp_lds<T>(p, 1) <= lds_limit;
}

template <typename T, int W, int MAXV, int NCT, int FS>
static hipError_t launch_fused_wvs(const DevPlan& p, const void* V, void* Gt, hipStream_t s) {
  const size_t lds = fused_interp_lds<T>(p, FS);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_x_interp<T, W, MAXV, NCT, FS>), lds);
  if (e != hipSuccess) return e;
  // bins per work-group: enough groups to fill the device several times over
  const long long strips = (p.tiles_y + FS - 1) / FS;
  int bins = int(std::min<long long>(kFusedBins, std::max<long long>(1, p.tiles_y * p.nb / 2048)));
  // where even 4 bins per group fill every resident slot at least twice, the
  // count in 4..kFusedBins whose last wave of work-groups is fullest (the
  // groups take about equal time, and a part-filled last wave idles the
  // rest of the device: 0.98 -> 0.965 ms per forward call with 576 bins
  // on a 384^2 grid, 7 bins instead of 6)
  static int slots_cache[64] = {};  // resident groups on the device, per device
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64) {
    if (slots_cache[dev] == 0) {
      int per_cu = 0, cus = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &per_cu, reinterpret_cast<const void*>(&k_fft_x_interp<T, W, MAXV, NCT, FS>), kFusedThreads * FS,
              lds) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        slots_cache[dev] = std::max(1, per_cu * cus);
      else
        slots_cache[dev] = -1;
    }
    const long long slots = slots_cache[dev];
    if (slots > 0 && strips * ((p.nb + 3) / 4) >= 2 * slots) {
      double best = -1.0;
      for (int bb = 4; bb <= kFusedBins; ++bb) {
        const double waves = double(strips * ((p.nb + bb - 1) / bb)) / double(slots);
        const double fill = waves / std::ceil(waves);
        if (fill >= best - 1e-9) {
          best = fill;
          bins = bb;
        }
      }
    }
  }
  const int nchunks = (p.nb + bins - 1) / bins;
  const long long blocks = strips * nchunks;
  hipLaunchKernelGGL((k_fft_x_interp<T, W, MAXV, NCT, FS>), dim3((unsigned)blocks), dim3(kFusedThreads * FS), lds, s,
                     static_cast<const cx<T>*>(V), p.nb, p.Nx, p.n_y, p.tiles_x, nchunks, bins, p.home_off,
                     p.home_sens, p.sbx, p.sby, static_cast<const T*>(p.swx), static_cast<const T*>(p.swy),
                     as_desc<T>(p.f_nx), p.brange, static_cast<cx<T>*>(Gt));
  return hipGetLastError();
}

// strip height chosen by the plan (DevPlan::fused_strip)
template <typename T, int W, int MAXV, int NCT>
static hipError_t launch_fused_wv(const DevPlan& p, const void* V, void* Gt, hipStream_t s) {
  if (p.fused_strip == 2) return launch_fused_wvs<T, W, MAXV, NCT, 2>(p, V, Gt, s);
  return launch_fused_wvs<T, W, MAXV, NCT, 1>(p, V, Gt, s);
}

// rows of up to 512 points need 8 values per lane in the one-wave transform, longer ones 16
template <typename T, int W>
static hipError_t launch_fused_w(const DevPlan& p, const void* V, void* Gt, hipStream_t s) {
  return ct_pick(CtFused{}, p.n_x, [&](auto c) {
    constexpr int NCT = decltype(c)::value;
    if constexpr (NCT > 0)
      return launch_fused_wv<T, W, 8, NCT>(p, V, Gt, s);
    else
      return p.n_x <= 512 ? launch_fused_wv<T, W, 8, 0>(p, V, Gt, s) : launch_fused_wv<T, W, 16, 0>(p, V, Gt, s);
  });
}

template <typename T>
hipError_t launch_fft_x_interp(const DevPlan& p, const void* V, void* Gt, hipStream_t s) {
  if (p.n_x > kWaveFftMax || p.Nx > p.n_x) return hipErrorInvalidValue;
  switch (p.w_xy) {
    case 2: return launch_fused_w<T, 2>(p, V, Gt, s);
    case 4: return launch_fused_w<T, 4>(p, V, Gt, s);
    case 6: return launch_fused_w<T, 6>(p, V, Gt, s);
    case 8: return launch_fused_w<T, 8>(p, V, Gt, s);
    case 10: return launch_fused_w<T, 10>(p, V, Gt, s);
    case 12: return launch_fused_w<T, 12>(p, V, Gt, s);
    case 14: return launch_fused_w<T, 14>(p, V, Gt, s);
    case 16: return launch_fused_w<T, 16>(p, V, Gt, s);
    default: return hipErrorInvalidValue;
  }
}

#define PATK_INST(T) template hipError_t launch_interp<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_fft_x_interp<T>(const DevPlan&, const void*, void*, hipStream_t);                   \
  template size_t fused_interp_lds<T>(const DevPlan&, int);                                                        \
  template bool fused_interp_ok<T>(const DevPlan&, size_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
