// gfx950 kernels of the NEDNER-NUFFT reconstruction (Section 3: a
// non-equispaced-range NUFFT in time, a non-equispaced-data NUFFT over the
// sensor plane, then an equispaced inverse FFT).
//
// Order of the steps on the device. The temporal transform's equispaced part
// (deapodise, zero-pad, FFT) runs first, per sensor; the lateral NUFFT then
// runs once per kept temporal bin; the temporal interpolation at
// omega(K) = c|K| runs last, per lateral mode. This is the paper's
// composition with the two linear maps on different indices applied in the
// other order, which lets the lateral grid be built only for the band of
// temporal bins that the interpolation reads.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fft_device.hpp"
#include "kernels.hpp"

namespace patk {

constexpr int kFftMaxV = 16;  // values per thread in the FFT kernels

// Sequences of length n per FFT work-group of nthr threads: at most kFftMaxV
// values per thread, at most `cap`, and (when possible) within 80 KiB of LDS
// so two work-groups share a CU.
template <typename T>
static int fft_batch(int n, int nthr, int cap) {
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
struct FftCfg {
  int threads = 256, cap = 8, wave = 0;
};
static FftCfg fft_cfg() { return FftCfg{}; }

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

// Allow a kernel more than the default dynamic LDS when a launch needs it.
static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename T>
static FftDesc<T> as_desc(const FftRaw& r) {
  FftDesc<T> d;
  static_assert(sizeof(FftPass) == sizeof(FftPassRaw), "pass layout");
  d.n = r.n;
  d.npass = r.npass;
  d.pass = static_cast<const FftPass*>(r.dpass);
  d.tw = static_cast<const cx<T>*>(r.tw);
  return d;
}

// ---------------------------------------------------------------------------
// Stage 0: temporal FFT per sensor (the equispaced half of eq. NER_NUFFT).
// Two real traces share one complex FFT (re = sensor m0, im = sensor m1).
// Sample n sits at index (n - n0) mod n_t after multiplication by
// h_m*dt/phihat_t((n - n0)/n_t); bins b_lo .. b_lo+nb-1 are kept per sensor.
// ---------------------------------------------------------------------------
constexpr int kTemporalThreads = 512;

template <typename T>
__global__ __launch_bounds__(kTemporalThreads) void k_temporal(const T* __restrict__ g, int M, int Nt, int n0,
                                                             const T* __restrict__ hw, const T* __restrict__ deap,
                                                             FftDesc<T> fd, int b_lo, int nb, int pairs,
                                                             cx<T>* __restrict__ Gt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_t = fd.n;
  const int L = lseq(n_t);
  const int mbase = 2 * pairs * blockIdx.x;  // first sensor of this group
  const int np = min(pairs, (M - mbase + 1) / 2);
  for (int q = tid; q < np * L; q += nthr) buf[q] = cx<T>{T(0), T(0)};
  __syncthreads();
  const FastDiv div_nt(Nt);
  staged_copy<kFftMaxV>(
      np * Nt, tid, nthr,
      [&](int q) {
        const int pr = div_nt(q);
        const int n = q - pr * Nt;
        const int m0 = mbase + 2 * pr;
        const bool has1 = m0 + 1 < M;
        const T d = deap[n];
        const T a = g[size_t(m0) * Nt + n] * hw[m0] * d;
        const T b = has1 ? g[size_t(m0 + 1) * Nt + n] * hw[m0 + 1] * d : T(0);
        return cx<T>{a, b};
      },
      [&](int q, cx<T> v) {
        const int pr = div_nt(q);
        int pos = q - pr * Nt - n0;
        if (pos < 0) pos += n_t;
        buf[pr * L + lpos(pos)] = v;
      });
  __syncthreads();
  fft_lds<T, kFftMaxV, false>(buf, fd, np, L, tid, nthr);
  const FastDiv div_nb(nb);
  for (int q = tid; q < np * nb; q += nthr) {
    const int pr = div_nb(q);
    const int i = q - pr * nb;
    const int m0 = mbase + 2 * pr;
    const int b = b_lo + i;  // -n_t < b < n_t (the band fits in n_t bins)
    const int pb = b < 0 ? b + n_t : b;
    const int mb = b > 0 ? n_t - b : -b;
    const cx<T> z = buf[pr * L + lpos(pb)];
    const cx<T> zm = buf[pr * L + lpos(mb)];
    // transform of the real part: (Z_b + conj Z_-b)/2; of the imaginary part: (Z_b - conj Z_-b)/(2i)
    Gt[size_t(m0) * nb + i] = cx<T>{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
    if (m0 + 1 < M) Gt[size_t(m0 + 1) * nb + i] = cx<T>{T(0.5) * (z.y + zm.y), T(-0.5) * (z.x - zm.x)};
  }
}

template <typename T>
hipError_t launch_temporal(const DevPlan& p, const T* g, void* Gt, hipStream_t s) {
  if (p.n_t > kFftMaxV * kTemporalThreads || p.Nt > p.n_t) return hipErrorInvalidValue;
  const int pairs = 1;  // one sensor pair per group measured fastest on MI355X
  const int blocks = (p.M + 2 * pairs - 1) / (2 * pairs);
  const size_t lds = size_t(pairs) * lseq(p.n_t) * sizeof(cx<T>);
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_temporal<T>), lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_temporal<T>, dim3(blocks), dim3(kTemporalThreads), lds, s, g, p.M, p.Nt, p.n0,
                     static_cast<const T*>(p.hw), static_cast<const T*>(p.deap), as_desc<T>(p.f_nt), p.b_lo, p.nb,
                     pairs, static_cast<cx<T>*>(Gt));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage 1: lateral spreading (the gridding of eq. NED_NUFFT), one chunk of
// temporal bins at a time. Output-driven and atomic-free: a work-group owns a
// 16x16 tile of the oversampled grid (four waves, each a 16x4 patch) and
// every lane owns one grid point, accumulating in registers the
// contributions of the tile's sensor list in list order (deterministic).
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

template <typename T, bool KAHAN>
__global__ __launch_bounds__(256) void k_spread(const cx<T>* __restrict__ Gt, int nb, const int* __restrict__ tile_off,
                                                const int* __restrict__ tile_sens, const int* __restrict__ sbx,
                                                const int* __restrict__ sby, const T* __restrict__ swx,
                                                const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                                int nchunks, int b_begin, int b_end, cx<T>* __restrict__ U) {
  constexpr int BC = kSpreadBins;
  constexpr int SB = kSpreadBatch;
  __shared__ int s_bx[SB], s_by[SB];
  __shared__ T s_wx[SB * kMaxW], s_wy[SB * kMaxW];
  __shared__ cx<T> s_g[SB * BC];
  // bin groups vary fastest: groups running together share one tile's sensor
  // list and read whole per-sensor rows of Gt (measured faster on MI355X than
  // ordering by tile)
  const int chunk = blockIdx.x % nchunks;
  const int tile = blockIdx.x / nchunks;
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
      static_assert(SB * 4 == 256 && kMaxW == 16 && BC == 16, "staging layout");
      const int qi = tid >> 2, r = tid & 3;
      if (qi < nq) {
        const int sidx = tile_sens[qb + qi];
        const T* wxs = swx + size_t(sidx) * w;
        const T* wys = swy + size_t(sidx) * w;
        const cx<T>* gs = Gt + size_t(sidx) * nb + b0;
        T vx[4], vy[4];
        cx<T> vg[4];
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
          s_g[qi * BC + r * 4 + i] = vg[i];
        }
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

template <typename T>
hipError_t launch_spread(const DevPlan& p, const void* Gt, void* U, int b_begin, int b_end, hipStream_t s) {
  if (p.w_xy > kMaxW || b_begin < 0 || b_end > p.nb || b_begin >= b_end) return hipErrorInvalidValue;
  const int nchunks = (b_end - b_begin + kSpreadBins - 1) / kSpreadBins;
  const long long blocks = (long long)p.tiles_x * p.tiles_y * nchunks;
  if (p.kahan)
    hipLaunchKernelGGL((k_spread<T, true>), dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const cx<T>*>(Gt), p.nb,
                       p.tile_off, p.tile_sens, p.sbx, p.sby, static_cast<const T*>(p.swx),
                       static_cast<const T*>(p.swy), p.w_xy, p.n_x, p.n_y, p.tiles_x, nchunks, b_begin, b_end,
                       static_cast<cx<T>*>(U));
  else
    hipLaunchKernelGGL((k_spread<T, false>), dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const cx<T>*>(Gt),
                       p.nb, p.tile_off, p.tile_sens, p.sbx, p.sby, static_cast<const T*>(p.swx),
                       static_cast<const T*>(p.swy), p.w_xy, p.n_x, p.n_y, p.tiles_x, nchunks, b_begin, b_end,
                       static_cast<cx<T>*>(U));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage 2: FFT along x of every grid row, keeping the Nx centred modes.
// U[b][py][px] -> V[b][jj][py], jj = j mod Nx for j in [-Nx/2, Nx/2).
// ---------------------------------------------------------------------------
constexpr int kFftThreads = 256;

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_x(const cx<T>* __restrict__ U, int n_y, int Nx, int rows,
                                                     int b_begin, FftDesc<T> fd, cx<T>* __restrict__ V, int wm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_x = fd.n;
  const int bstride = lseq(n_x);
  const int b = b_begin + blockIdx.y;
  const int py0 = blockIdx.x * rows;
  const int nr = min(rows, n_y - py0);
  const cx<T>* src = U + (size_t(b - b_begin) * n_y + py0) * n_x;
  const FastDiv div_nx(n_x), div_nr(nr);
  staged_copy<kFftMaxV>(
      nr * n_x, tid, nthr, [&](int q) { return src[q]; },
      [&](int q, cx<T> v) {
        const int r = div_nx(q);
        buf[r * bstride + lpos(q - r * n_x)] = v;
      });
  __syncthreads();
  fft_group<T, false>(buf, fd, nr, bstride, tid, nthr, wm);
  __syncthreads();
  cx<T>* dst = V + size_t(b) * Nx * n_y + py0;
  staged_copy<kFftMaxV>(
      nr * Nx, tid, nthr,
      [&](int q) {
        const int jj = div_nr(q);
        const int r = q - jj * nr;
        const int j = jj < Nx / 2 ? jj : jj - Nx;
        return buf[r * bstride + lpos(j < 0 ? j + n_x : j)];
      },
      [&](int q, cx<T> v) {
        const int jj = div_nr(q);
        dst[size_t(jj) * n_y + (q - jj * nr)] = v;
      });
}

template <typename T>
hipError_t launch_fft_x(const DevPlan& p, const void* U, void* V, int b_begin, int b_end, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int rows = fft_batch<T>(p.n_x, cfg.threads, cfg.cap);
  const size_t lds = size_t(rows) * lseq(p.n_x) * sizeof(cx<T>);
  if (size_t(rows) * p.n_x > size_t(kFftMaxV) * cfg.threads || size_t(rows) * p.Nx > size_t(kFftMaxV) * cfg.threads ||
      b_begin < 0 || b_end > p.nb || b_begin >= b_end)
    return hipErrorInvalidValue;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_x<T>), lds);
  if (e != hipSuccess) return e;
  dim3 grid((p.n_y + rows - 1) / rows, b_end - b_begin);
  hipLaunchKernelGGL(k_fft_x<T>, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(U), p.n_y, p.Nx, rows,
                     b_begin, as_desc<T>(p.f_nx), static_cast<cx<T>*>(V), cfg.wave);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage 3: FFT along y, keep the Ny centred modes, divide by the window
// transform in x and y (eq. NED_NUFFT's 1/Psi_j), and transpose so the bins
// of each lateral mode are contiguous: V[b][jj][py] -> Gh[jj][kk][b].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_y(const cx<T>* __restrict__ V, int nb, int Nx, int Ny, int bins,
                                                     const T* __restrict__ dcx, const T* __restrict__ dcy,
                                                     FftDesc<T> fd, cx<T>* __restrict__ Gh, int wm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_y = fd.n;
  const int bstride = lseq(n_y);
  const int jj = blockIdx.y;
  const int b0 = blockIdx.x * bins;
  const int nbc = min(bins, nb - b0);
  const FastDiv div_ny(n_y), div_nbc(nbc);
  staged_copy<kFftMaxV>(
      nbc * n_y, tid, nthr,
      [&](int q) {
        const int bi = div_ny(q);
        return V[(size_t(b0 + bi) * Nx + jj) * n_y + (q - bi * n_y)];
      },
      [&](int q, cx<T> v) {
        const int bi = div_ny(q);
        buf[bi * bstride + lpos(q - bi * n_y)] = v;
      });
  __syncthreads();
  fft_group<T, false>(buf, fd, nbc, bstride, tid, nthr, wm);
  __syncthreads();
  const T cxj = dcx[jj];
  cx<T>* dst = Gh + size_t(jj) * Ny * nb + b0;
  staged_copy<kFftMaxV>(
      nbc * Ny, tid, nthr,
      [&](int q) {
        const int kk = div_nbc(q);
        const int bi = q - kk * nbc;
        const int k = kk < Ny / 2 ? kk : kk - Ny;
        const T sc = cxj * dcy[kk];
        const cx<T> v = buf[bi * bstride + lpos(k < 0 ? k + n_y : k)];
        return cx<T>{v.x * sc, v.y * sc};
      },
      [&](int q, cx<T> v) {
        const int kk = div_nbc(q);
        dst[size_t(kk) * nb + (q - kk * nbc)] = v;
      });
}

template <typename T>
hipError_t launch_fft_y(const DevPlan& p, const void* V, void* Gh, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int bins = fft_batch<T>(p.n_y, cfg.threads, cfg.cap);
  const size_t lds = size_t(bins) * lseq(p.n_y) * sizeof(cx<T>);
  if (size_t(bins) * p.n_y > size_t(kFftMaxV) * cfg.threads || size_t(bins) * p.Ny > size_t(kFftMaxV) * cfg.threads)
    return hipErrorInvalidValue;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_y<T>), lds);
  if (e != hipSuccess) return e;
  dim3 grid((p.nb + bins - 1) / bins, p.Nx);
  hipLaunchKernelGGL(k_fft_y<T>, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(V), p.nb, p.Nx, p.Ny,
                     bins, static_cast<const T*>(p.dcx), static_cast<const T*>(p.dcy), as_desc<T>(p.f_ny),
                     static_cast<cx<T>*>(Gh), cfg.wave);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage 4: temporal interpolation at omega(K) (the window sum of
// eq. NER_NUFFT with the centring phase of eq. PSI) and the inversion
// weight of eq. exact. For lateral mode (j,k) and l = 1..Nz/2-1:
//   s  = c |K| dt n_t / (2 pi)                  (double)
//   S  = exp(-2 pi i s n0/n_t) sum_t phi_t(s - b_t) Gh[j][k][b_t]
//   F  = 2c Kz/|K| * S
// The l = 0, l = Nz/2, j = -Nx/2 and k = -Ny/2 entries are written as 0.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gather(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                                double s_per_k, double kxu, double kyu, double kzu, double two_c,
                                                double n0_over_nt, double scale, int physical, int wt, int deg,
                                                const T* __restrict__ hcoef, cx<T>* __restrict__ Fh) {
  const int Lh = Nz / 2 + 1;
  const long long total = (long long)Nx * Ny * Lh;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int l = int(idx % Lh);
  const long long col = idx / Lh;
  const int kk = int(col % Ny);
  const int jj = int(col / Ny);
  if (l == 0 || l == Nz / 2 || jj == Nx / 2 || kk == Ny / 2) {
    Fh[idx] = cx<T>{T(0), T(0)};
    return;
  }
  const int j = jj < Nx / 2 ? jj : jj - Nx;
  const int k = kk < Ny / 2 ? kk : kk - Ny;
  const double Kx = j * kxu, Ky = k * kyu, Kz = l * kzu;
  const double Kabs = sqrt(Kx * Kx + Ky * Ky + Kz * Kz);
  const double s = Kabs * s_per_k;
  const double fl = floor(s);
  const T y = T(2.0 * (s - fl) - 1.0);
  int base = int(fl) - wt / 2 + 1 - b_lo;
  base = base < 0 ? 0 : (base > nb - wt ? nb - wt : base);
  const cx<T>* src = Gh + col * nb + base;
  cx<T> acc{T(0), T(0)};
  const int np = deg + 1;
  for (int t = 0; t < wt; ++t) {
    const T* c = hcoef + t * np;
    T v = c[deg];
    for (int d = deg - 1; d >= 0; --d) v = v * y + c[d];
    const cx<T> gv = src[t];
    acc.x += v * gv.x;
    acc.y += v * gv.y;
  }
  double q = s * n0_over_nt;
  q -= floor(q);
  double sn, cs;
  sincos(-2.0 * M_PI * q, &sn, &cs);
  double wgt = two_c * Kz / Kabs * scale;
  if (physical && ((jj + kk) & 1)) wgt = -wgt;
  const cx<T> ph{T(wgt * cs), T(wgt * sn)};
  Fh[idx] = cmul(acc, ph);
}

template <typename T>
hipError_t launch_gather(const DevPlan& p, const void* Gh, void* Fh, bool physical, hipStream_t s) {
  const long long total = (long long)p.Nx * p.Ny * (p.Nz / 2 + 1);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  const double scale = physical ? 1.0 : p.inv_vol;
  hipLaunchKernelGGL(k_gather<T>, dim3(blocks), dim3(256), 0, s, static_cast<const cx<T>*>(Gh), p.nb, p.b_lo, p.Nx,
                     p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, scale, physical ? 1 : 0,
                     p.w_t, p.hdeg, static_cast<const T*>(p.hcoef), static_cast<cx<T>*>(Fh));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stage 5: equispaced inverse 3-D FFT (step 3 of the NEDNER list) on the
// half spectrum Fh[jj][kk][l], l = 0..Nz/2: in-place inverse transforms
// along x and along y, then a complex-to-real transform along z.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_ifft_x(cx<T>* __restrict__ F, int Ny, int Lh, int lchunk,
                                                      FftDesc<T> fd, int wm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Nx = fd.n;
  const int bstride = lseq(Nx);
  const int kk = blockIdx.y;
  const int l0 = blockIdx.x * lchunk;
  const int nl = min(lchunk, Lh - l0);
  const FastDiv div_nl(nl);
  staged_copy<kFftMaxV>(
      nl * Nx, tid, nthr,
      [&](int q) {
        const int jj = div_nl(q);
        return F[(size_t(jj) * Ny + kk) * Lh + l0 + (q - jj * nl)];
      },
      [&](int q, cx<T> v) {
        const int jj = div_nl(q);
        buf[(q - jj * nl) * bstride + lpos(jj)] = v;
      });
  __syncthreads();
  fft_group<T, true>(buf, fd, nl, bstride, tid, nthr, wm);
  __syncthreads();
  staged_copy<kFftMaxV>(
      nl * Nx, tid, nthr,
      [&](int q) {
        const int jj = div_nl(q);
        return buf[(q - jj * nl) * bstride + lpos(jj)];
      },
      [&](int q, cx<T> v) {
        const int jj = div_nl(q);
        F[(size_t(jj) * Ny + kk) * Lh + l0 + (q - jj * nl)] = v;
      });
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_ifft_y(cx<T>* __restrict__ F, int Lh, int lchunk, FftDesc<T> fd, int wm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Ny = fd.n;
  const int bstride = lseq(Ny);
  const int jj = blockIdx.y;
  const int l0 = blockIdx.x * lchunk;
  const int nl = min(lchunk, Lh - l0);
  cx<T>* base = F + size_t(jj) * Ny * Lh + l0;
  const FastDiv div_nl(nl);
  staged_copy<kFftMaxV>(
      nl * Ny, tid, nthr,
      [&](int q) {
        const int kk = div_nl(q);
        return base[size_t(kk) * Lh + (q - kk * nl)];
      },
      [&](int q, cx<T> v) {
        const int kk = div_nl(q);
        buf[(q - kk * nl) * bstride + lpos(kk)] = v;
      });
  __syncthreads();
  fft_group<T, true>(buf, fd, nl, bstride, tid, nthr, wm);
  __syncthreads();
  staged_copy<kFftMaxV>(
      nl * Ny, tid, nthr,
      [&](int q) {
        const int kk = div_nl(q);
        return buf[(q - kk * nl) * bstride + lpos(kk)];
      },
      [&](int q, cx<T> v) {
        const int kk = div_nl(q);
        base[size_t(kk) * Lh + (q - kk * nl)] = v;
      });
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_c2r_z(const cx<T>* __restrict__ F, long long nrows, int rows,
                                                     FftDesc<T> fd, T* __restrict__ f, int wm) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Nz = fd.n;
  const int Lh = Nz / 2 + 1;
  const int bstride = lseq(Nz);
  const long long r0 = (long long)blockIdx.x * rows;
  const int nr = (int)min((long long)rows, nrows - r0);
  const FastDiv div_lh(Lh), div_nz(Nz);
  staged_copy<kFftMaxV>(
      nr * Lh, tid, nthr, [&](int q) { return F[r0 * Lh + q]; },
      [&](int q, cx<T> v) {
        const int r = div_lh(q);
        const int l = q - r * Lh;
        buf[r * bstride + lpos(l)] = v;
        if (l > 0 && l < Nz / 2) buf[r * bstride + lpos(Nz - l)] = cx<T>{v.x, -v.y};
      });
  __syncthreads();
  fft_group<T, true>(buf, fd, nr, bstride, tid, nthr, wm);
  __syncthreads();
  staged_copy<kFftMaxV>(
      nr * Nz, tid, nthr,
      [&](int q) {
        const int r = div_nz(q);
        return buf[r * bstride + lpos(q - r * Nz)].x;
      },
      [&](int q, T v) { f[r0 * Nz + q] = v; });
}

template <typename T>
hipError_t launch_inverse(const DevPlan& p, void* Fh, T* f, hipStream_t s) {
  cx<T>* F = static_cast<cx<T>*>(Fh);
  const int Lh = p.Nz / 2 + 1;
  const FftCfg cfg = fft_cfg();
  {
    const int lc = fft_batch<T>(p.Nx, cfg.threads, cfg.cap);
    const size_t lds = size_t(lc) * lseq(p.Nx) * sizeof(cx<T>);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_ifft_x<T>), lds);
    if (e != hipSuccess) return e;
    dim3 grid((Lh + lc - 1) / lc, p.Ny);
    hipLaunchKernelGGL(k_ifft_x<T>, grid, dim3(cfg.threads), lds, s, F, p.Ny, Lh, lc, as_desc<T>(p.f_Nx), cfg.wave);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const int lc = fft_batch<T>(p.Ny, cfg.threads, cfg.cap);
    const size_t lds = size_t(lc) * lseq(p.Ny) * sizeof(cx<T>);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_ifft_y<T>), lds);
    if (e != hipSuccess) return e;
    dim3 grid((Lh + lc - 1) / lc, p.Nx);
    hipLaunchKernelGGL(k_ifft_y<T>, grid, dim3(cfg.threads), lds, s, F, Lh, lc, as_desc<T>(p.f_Ny), cfg.wave);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const int rows = fft_batch<T>(p.Nz, cfg.threads, cfg.cap);
    const size_t lds = size_t(rows) * lseq(p.Nz) * sizeof(cx<T>);
    hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_c2r_z<T>), lds);
    if (e != hipSuccess) return e;
    const long long nrows = (long long)p.Nx * p.Ny;
    hipLaunchKernelGGL(k_c2r_z<T>, dim3((unsigned)((nrows + rows - 1) / rows)), dim3(cfg.threads), lds, s, F, nrows,
                       rows, as_desc<T>(p.f_Nz), f, cfg.wave);
  }
  return hipGetLastError();
}

#define PATK_INSTANTIATE(T)                                                                     \
  template hipError_t launch_temporal<T>(const DevPlan&, const T*, void*, hipStream_t);         \
  template hipError_t launch_spread<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_fft_x<T>(const DevPlan&, const void*, void*, int, int, hipStream_t);  \
  template hipError_t launch_fft_y<T>(const DevPlan&, const void*, void*, hipStream_t);         \
  template hipError_t launch_gather<T>(const DevPlan&, const void*, void*, bool, hipStream_t);  \
  template hipError_t launch_inverse<T>(const DevPlan&, void*, T*, hipStream_t);

PATK_INSTANTIATE(float)
PATK_INSTANTIATE(double)

}  // namespace patk
