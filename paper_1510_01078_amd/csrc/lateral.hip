// Equispaced part of the lateral NUFFT (Section 3.2): FFTs of the
// oversampled grid along x and y, cropping and deconvolution.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
// Stage 2: FFT along x of every grid row, keeping the Nx centred modes.
// U[b][py][px] -> V[b][jj][py], jj = j mod Nx for j in [-Nx/2, Nx/2).
// ---------------------------------------------------------------------------
template <typename T, int NCT = 0>
__device__ __forceinline__ void fft_x_body(const cx<T>* __restrict__ U, int n_y, int Nx, int rows,
                                           int b_begin, FftDesc<T> fd, cx<T>* __restrict__ V, int wm, int bx, int by,
                                           const int* __restrict__ brange = nullptr, int tid = threadIdx.x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nthr = blockDim.x;
  const int n_x = NCT > 0 ? NCT : fd.n;
  const int bstride = lseq(n_x);
  const int b = b_begin + by;
  const int py0 = bx * rows;
  const int nr = min(rows, n_y - py0);
  const cx<T>* src = U + (size_t(b - b_begin) * n_y + py0) * n_x;
  cx<T>* dst = V + size_t(b) * Nx * n_y + py0;
  // output mode jj of the Nx kept, centred, at its slot of the n_x transform
  auto slot = [&](int jj) {
    const int j = jj < Nx / 2 ? jj : jj - Nx;
    return lpos(j < 0 ? j + n_x : j);
  };
  // only the x modes whose band range holds bin b (|j| in [J0, J1]) are
  // written: the y-FFT and the interpolation read no others
  const int J0 = brange ? brange[2 * b] : 0, J1 = brange ? brange[2 * b + 1] : Nx;
  auto kept = [&](int jj) {
    const int aj = jj < Nx / 2 ? jj : Nx - jj;
    return aj >= J0 && aj <= J1;
  };
  cx<T>* twl = buf + rows * bstride;
  if constexpr (NCT > 0) {
    // compile-time geometry (rows = ROWS, 256 threads): no index divisions
    constexpr int ROWS = ct_maxb(NCT, kFftCap), BS = lseq(NCT);
    staged_rows<ROWS, NCT, kFftThreads>(
        nr, tid, [&](int r, int c) { return src[r * NCT + c]; },
        [&](int r, int c, cx<T> v) { buf[r * BS + lpos(c)] = v; });
    for (int t = tid; t < NCT; t += kFftThreads) twl[t] = fd.tw[t];
    __syncthreads();
    fft_ct<T, NCT, kFftThreads, ROWS, false>(buf, nr, twl, tid);
    __syncthreads();
    // V[b][jj][py0 + r]: neighbouring threads write neighbouring rows
    cx<T>* d0 = dst + size_t(tid / ROWS) * n_y + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * n_y;
    staged_cols<ROWS, kFftThreads, (NCT * ROWS + kFftThreads - 1) / kFftThreads>(  // Nx < n_x = NCT
        Nx, nr, tid,
        [&](int jj, int r, int) { return kept(jj) ? buf[r * BS + slot(jj)] : cx<T>{T(0), T(0)}; },
        [&](int jj, int, int u, cx<T> v) {
          if (kept(jj)) d0[u * step] = v;
        });
  } else {
    const FastDiv div_nx(n_x), div_nr(nr);
    staged_copy<kFftMaxV>(
        nr * n_x, tid, nthr, [&](int q) { return src[q]; },
        [&](int q, cx<T> v) {
          const int r = div_nx(q);
          buf[r * bstride + lpos(q - r * n_x)] = v;
        });
    // the twiddles go to LDS behind the rows (every pass reads them)
    for (int t = tid; t < fd.n; t += nthr) twl[t] = fd.tw[t];
    __syncthreads();
    fft_group<T, false>(buf, lds_twiddles(fd, twl), nr, bstride, tid, nthr, wm);
    __syncthreads();
    staged_copy<kFftMaxV>(
        nr * Nx, tid, nthr,
        [&](int q) {
          const int jj = div_nr(q);
          return kept(jj) ? buf[(q - jj * nr) * bstride + slot(jj)] : cx<T>{T(0), T(0)};
        },
        [&](int q, cx<T> v) {
          const int jj = div_nr(q);
          if (kept(jj)) dst[size_t(jj) * n_y + (q - jj * nr)] = v;
        });
  }
}

template <typename T, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_fft_x(const cx<T>* __restrict__ U, int n_y, int Nx, int rows,
                                                     int b_begin, FftDesc<T> fd, cx<T>* __restrict__ V, int wm,
                                                     const int* __restrict__ brange) {
  // neighbouring groups write the two halves of each 128-byte output line:
  // keep them on one XCD so its L2 merges the halves
  const int gl = xcd_linear();
  fft_x_body<T, NCT>(U, n_y, Nx, rows, b_begin, fd, V, wm, gl % gridDim.x, gl / gridDim.x, brange);
}

template <typename T>
hipError_t launch_fft_x(const DevPlan& p, const void* U, void* V, int b_begin, int b_end, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int rows = fft_batch<T>(p.n_x, cfg.threads, cfg.cap);
  const size_t lds = (size_t(rows) * lseq(p.n_x) + p.n_x) * sizeof(cx<T>);
  if (size_t(rows) * p.n_x > size_t(kFftMaxV) * cfg.threads || size_t(rows) * p.Nx > size_t(kFftMaxV) * cfg.threads ||
      b_begin < 0 || b_end > p.nb || b_begin >= b_end)
    return hipErrorInvalidValue;
  auto go = [&](auto kern, int nct) {
    // the compile-time kernels take their geometry from the length
    if (nct > 0 && (rows != ct_maxb(nct, kFftCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds);
    if (e != hipSuccess) return e;
    dim3 grid((p.n_y + rows - 1) / rows, b_end - b_begin);
    hipLaunchKernelGGL(kern, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(U), p.n_y, p.Nx, rows,
                       b_begin, as_desc<T>(p.f_nx), static_cast<cx<T>*>(V), cfg.wave, p.brange);
    return hipGetLastError();
  };
  return ct_pick(CtLateral{}, p.n_x, [&](auto c) { return go(&k_fft_x<T, decltype(c)::value>, decltype(c)::value); });
}

// ---------------------------------------------------------------------------
// Stage 3: FFT along y, keep the Ny centred modes, divide by the window
// transform in x and y (eq. NED_NUFFT's 1/Psi_j), and transpose so the bins
// of each lateral mode are contiguous: V[b][jj][py] -> Gh[jj][kk][b].
// ---------------------------------------------------------------------------
// jrange (may be nullptr): groups of bins outside the x-mode's range are
// skipped (the interpolation never reads them).
template <typename T, int NCT = 0>
__device__ __forceinline__ void fft_y_body(const cx<T>* __restrict__ V, int nb, int Nx, int Ny, int bins,
                                           const T* __restrict__ dcx, const T* __restrict__ dcy,
                                           FftDesc<T> fd, cx<T>* __restrict__ Gh, int wm, int bx, int by,
                                           const int* __restrict__ jrange = nullptr, int tid = threadIdx.x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nthr = blockDim.x;
  const int n_y = NCT > 0 ? NCT : fd.n;
  const int bstride = lseq(n_y);
  const int jj = by;
  const int b0 = bx * bins;
  const int nbc = min(bins, nb - b0);
  if (jrange && (b0 + nbc - 1 < jrange[2 * jj] || b0 > jrange[2 * jj + 1])) return;
  const cx<T>* src = V + (size_t(b0) * Nx + jj) * n_y;  // bin b0 + bi at src + bi * Nx * n_y
  const size_t bin_stride = size_t(Nx) * n_y;
  const T cxj = dcx[jj];
  cx<T>* dst = Gh + size_t(jj) * Ny * nb + b0;
  // output mode kk of the Ny kept, centred, at its slot of the n_y transform
  auto slot = [&](int kk) {
    const int k = kk < Ny / 2 ? kk : kk - Ny;
    return lpos(k < 0 ? k + n_y : k);
  };
  cx<T>* twl = buf + bins * bstride;
  if constexpr (NCT > 0) {
    // compile-time geometry (bins = ROWS, 256 threads): no index divisions
    constexpr int ROWS = ct_maxb(NCT, kFftCap), BS = lseq(NCT);
    // non-temporal loads: each band row is read once, and keeping it out of
    // the caches leaves them to the spectra this kernel writes, which the
    // gather reads next (y-FFT 0.106 -> 0.104 ms, gather 0.077 -> 0.072 ms)
    staged_rows<ROWS, NCT, kFftThreads>(
        nbc, tid, [&](int r, int c) { return nt_load(src + r * bin_stride + c); },
        [&](int r, int c, cx<T> v) { buf[r * BS + lpos(c)] = v; });
    for (int t = tid; t < NCT; t += kFftThreads) twl[t] = fd.tw[t];
    __syncthreads();
    fft_ct<T, NCT, kFftThreads, ROWS, false>(buf, nbc, twl, tid);
    __syncthreads();
    // Gh[jj][kk][b0 + bi]: neighbouring threads write neighbouring bins
    cx<T>* d0 = dst + size_t(tid / ROWS) * nb + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * nb;
    staged_cols<ROWS, kFftThreads, (NCT * ROWS + kFftThreads - 1) / kFftThreads>(  // Ny < n_y = NCT
        Ny, nbc, tid,
        [&](int kk, int bi, int) {
          const T sc = cxj * dcy[kk];
          const cx<T> v = buf[bi * BS + slot(kk)];
          return cx<T>{v.x * sc, v.y * sc};
        },
        [&](int, int, int u, cx<T> v) { d0[u * step] = v; });
  } else {
    const FastDiv div_ny(n_y), div_nbc(nbc);
    staged_copy<kFftMaxV>(
        nbc * n_y, tid, nthr,
        [&](int q) {
          const int bi = div_ny(q);
          return src[bi * bin_stride + (q - bi * n_y)];
        },
        [&](int q, cx<T> v) {
          const int bi = div_ny(q);
          buf[bi * bstride + lpos(q - bi * n_y)] = v;
        });
    for (int t = tid; t < fd.n; t += nthr) twl[t] = fd.tw[t];
    __syncthreads();
    fft_group<T, false>(buf, lds_twiddles(fd, twl), nbc, bstride, tid, nthr, wm);
    __syncthreads();
    staged_copy<kFftMaxV>(
        nbc * Ny, tid, nthr,
        [&](int q) {
          const int kk = div_nbc(q);
          const int bi = q - kk * nbc;
          const T sc = cxj * dcy[kk];
          const cx<T> v = buf[bi * bstride + slot(kk)];
          return cx<T>{v.x * sc, v.y * sc};
        },
        [&](int q, cx<T> v) {
          const int kk = div_nbc(q);
          dst[size_t(kk) * nb + (q - kk * nbc)] = v;
        });
  }
}

template <typename T, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_fft_y(const cx<T>* __restrict__ V, int nb, int Nx, int Ny, int bins,
                                                     const T* __restrict__ dcx, const T* __restrict__ dcy,
                                                     FftDesc<T> fd, cx<T>* __restrict__ Gh, int wm,
                                                     const int* __restrict__ jrange, const int* __restrict__ ylist) {
  // neighbouring groups write the two halves of each 128-byte output line:
  // keep them on one XCD so its L2 merges the halves
  const int gl = xcd_linear();
  int bx = gl % gridDim.x, by = gl / gridDim.x;
  if (ylist) {  // one-dimensional grid over the work items inside the ranges
    const int e = ylist[gl];
    by = e >> 16;
    bx = e & 0xffff;
  }
  fft_y_body<T, NCT>(V, nb, Nx, Ny, bins, dcx, dcy, fd, Gh, wm, bx, by, jrange);
}

template <typename T>
hipError_t launch_fft_y(const DevPlan& p, const void* V, void* Gh, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int bins = fft_batch<T>(p.n_y, cfg.threads, cfg.cap);
  const size_t lds = (size_t(bins) * lseq(p.n_y) + p.n_y) * sizeof(cx<T>);
  if (size_t(bins) * p.n_y > size_t(kFftMaxV) * cfg.threads || size_t(bins) * p.Ny > size_t(kFftMaxV) * cfg.threads)
    return hipErrorInvalidValue;
  auto go = [&](auto kern, int nct) {
    // the compile-time kernels take their geometry from the length
    if (nct > 0 && (bins != ct_maxb(nct, kFftCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds);
    if (e != hipSuccess) return e;
    const bool listed = p.ylist && p.ylist_n > 0 && p.jrange;
    const dim3 grid = listed ? dim3(p.ylist_n) : dim3((p.nb + bins - 1) / bins, p.Nx);
    hipLaunchKernelGGL(kern, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(V), p.nb, p.Nx, p.Ny,
                       bins, static_cast<const T*>(p.dcx), static_cast<const T*>(p.dcy), as_desc<T>(p.f_ny),
                       static_cast<cx<T>*>(Gh), cfg.wave, p.jrange, listed ? p.ylist : nullptr);
    return hipGetLastError();
  };
  return ct_pick(CtLateral{}, p.n_y, [&](auto c) { return go(&k_fft_y<T, decltype(c)::value>, decltype(c)::value); });
}

// ---------------------------------------------------------------------------
// Transposes for the forward model (conjugate transposes of k_fft_y and
// k_fft_x: embed the cropped modes into the oversampled length with zeros,
// inverse FFT).
// Gh'[j][k][b] -> V'[b][j][py] = dcx_j sum_k dcy_k Gh'[j][k][b] e^{+2 pi i k py/n_y}
// ---------------------------------------------------------------------------
template <typename T, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_fft_y_t(const cx<T>* __restrict__ Gh, int nb, int Nx, int Ny,
                                                       int bins, const T* __restrict__ dcx,
                                                       const T* __restrict__ dcy, FftDesc<T> fd,
                                                       cx<T>* __restrict__ V, const int* __restrict__ jrange,
                                                       const int* __restrict__ ylist) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_y = NCT > 0 ? NCT : fd.n;
  const int bstride = lseq(n_y);
  // (an XCD-grouped order measured slower here); with ylist a one-dimensional
  // grid over the work items inside the ranges
  const int jj = ylist ? ylist[blockIdx.x] >> 16 : int(blockIdx.y);
  const int b0 = (ylist ? ylist[blockIdx.x] & 0xffff : int(blockIdx.x)) * bins;
  const int nbc = min(bins, nb - b0);
  // bins outside the x-mode's range hold zeros that nothing reads: skipped
  if (jrange && (b0 + nbc - 1 < jrange[2 * jj] || b0 > jrange[2 * jj + 1])) return;
  const int gap = n_y - Ny;  // zero slots k = Ny/2 .. n_y - Ny/2 - 1
  const T cxj = dcx[jj];
  const cx<T>* src = Gh + size_t(jj) * Ny * nb + b0;
  auto slot = [&](int kk) {
    const int k = kk < Ny / 2 ? kk : kk - Ny;
    return lpos(k < 0 ? k + n_y : k);
  };
  cx<T>* twl = buf + bins * bstride;
  if constexpr (NCT > 0) {
    // compile-time geometry (bins = ROWS, 256 threads): no index divisions
    constexpr int ROWS = ct_maxb(NCT, kFftCap), BS = lseq(NCT);
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
      if (r < nbc)
        for (int c = tid; c < gap; c += kFftThreads) buf[r * BS + lpos(Ny / 2 + c)] = cx<T>{T(0), T(0)};
    const cx<T>* s0 = src + size_t(tid / ROWS) * nb + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * nb;
    staged_cols<ROWS, kFftThreads, (NCT * ROWS + kFftThreads - 1) / kFftThreads>(  // Ny < n_y = NCT
        Ny, nbc, tid,
        [&](int kk, int, int u) {
          const T sc = cxj * dcy[kk];
          const cx<T> v = s0[u * step];
          return cx<T>{v.x * sc, v.y * sc};
        },
        [&](int kk, int bi, int, cx<T> v) { buf[bi * BS + slot(kk)] = v; });
    for (int t = tid; t < NCT; t += kFftThreads) twl[t] = fd.tw[t];
    __syncthreads();
    fft_ct<T, NCT, kFftThreads, ROWS, true>(buf, nbc, twl, tid);
    __syncthreads();
    cx<T>* v0 = V + (size_t(b0) * Nx + jj) * NCT;  // bin b0 + r at v0 + r * Nx * NCT
    const size_t bin_stride = size_t(Nx) * NCT;
    staged_rows<ROWS, NCT, kFftThreads>(
        nbc, tid, [&](int r, int c) { return buf[r * BS + lpos(c)]; },
        // non-temporal: streams out once (measured faster for the fused reader)
        [&](int r, int c, cx<T> v) { nt_store(v0 + r * bin_stride + c, v); });
  } else {
    const FastDiv div_gap(gap), div_nbc(nbc), div_ny(n_y);
    for (int q = tid; q < nbc * gap; q += nthr) {
      const int bi = div_gap(q);
      buf[bi * bstride + lpos(Ny / 2 + (q - bi * gap))] = cx<T>{T(0), T(0)};
    }
    staged_copy<kFftMaxV>(
        nbc * Ny, tid, nthr,
        [&](int q) {
          const int kk = div_nbc(q);
          const T sc = cxj * dcy[kk];
          const cx<T> v = src[size_t(kk) * nb + (q - kk * nbc)];
          return cx<T>{v.x * sc, v.y * sc};
        },
        [&](int q, cx<T> v) {
          const int kk = div_nbc(q);
          buf[(q - kk * nbc) * bstride + slot(kk)] = v;
        });
    for (int t = tid; t < fd.n; t += nthr) twl[t] = fd.tw[t];
    __syncthreads();
    fft_lds<T, kFftMaxV, true, false>(buf, lds_twiddles(fd, twl), nbc, bstride, tid, nthr);
    __syncthreads();
    staged_copy<kFftMaxV>(
        nbc * n_y, tid, nthr,
        [&](int q) {
          const int bi = div_ny(q);
          return buf[bi * bstride + lpos(q - bi * n_y)];
        },
        [&](int q, cx<T> v) {  // non-temporal: streams out once (measured faster for the fused reader)
          const int bi = div_ny(q);
          nt_store(V + (size_t(b0 + bi) * Nx + jj) * n_y + (q - bi * n_y), v);
        });
  }
}

template <typename T>
hipError_t launch_fft_y_t(const DevPlan& p, const void* Gh, void* V, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int bins = fft_batch<T>(p.n_y, cfg.threads, cfg.cap);
  const size_t lds = (size_t(bins) * lseq(p.n_y) + p.n_y) * sizeof(cx<T>);
  if (size_t(bins) * p.n_y > size_t(kFftMaxV) * cfg.threads || size_t(bins) * p.Ny > size_t(kFftMaxV) * cfg.threads)
    return hipErrorInvalidValue;
  auto go = [&](auto kern, int nct) {
    // the compile-time kernels take their geometry from the length
    if (nct > 0 && (bins != ct_maxb(nct, kFftCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
    hipError_t e = allow_lds(reinterpret_cast<const void*>(kern), lds);
    if (e != hipSuccess) return e;
    const bool listed = p.ylist && p.ylist_n > 0 && p.jrange;
    const dim3 grid = listed ? dim3(p.ylist_n) : dim3((p.nb + bins - 1) / bins, p.Nx);
    hipLaunchKernelGGL(kern, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(Gh), p.nb, p.Nx, p.Ny,
                       bins, static_cast<const T*>(p.dcx), static_cast<const T*>(p.dcy), as_desc<T>(p.f_ny),
                       static_cast<cx<T>*>(V), p.jrange, listed ? p.ylist : nullptr);
    return hipGetLastError();
  };
  return ct_pick(CtLateral{}, p.n_y, [&](auto c) { return go(&k_fft_y_t<T, decltype(c)::value>, decltype(c)::value); });
}

// V'[b][j][py] -> U'[b - b_begin][py][px] = sum_j V'[b][j][py] e^{+2 pi i j px/n_x}
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_t(const cx<T>* __restrict__ V, int n_y, int Nx, int rows,
                                                       int b_begin, FftDesc<T> fd, cx<T>* __restrict__ U) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n_x = fd.n;
  const int bstride = lseq(n_x);
  const int b = b_begin + blockIdx.y;
  const int py0 = blockIdx.x * rows;
  const int nr = min(rows, n_y - py0);
  const int gap = n_x - Nx;
  const FastDiv div_gap(gap), div_nr(nr), div_nx(n_x);
  for (int q = tid; q < nr * gap; q += nthr) {
    const int r = div_gap(q);
    buf[r * bstride + lpos(Nx / 2 + (q - r * gap))] = cx<T>{T(0), T(0)};
  }
  const cx<T>* src = V + size_t(b) * Nx * n_y + py0;
  staged_copy<kFftMaxV>(
      nr * Nx, tid, nthr,
      [&](int q) {
        const int jj = div_nr(q);
        return src[size_t(jj) * n_y + (q - jj * nr)];
      },
      [&](int q, cx<T> v) {
        const int jj = div_nr(q);
        const int j = jj < Nx / 2 ? jj : jj - Nx;
        buf[(q - jj * nr) * bstride + lpos(j < 0 ? j + n_x : j)] = v;
      });
  __syncthreads();
  fft_lds<T, kFftMaxV, true, false>(buf, fd, nr, bstride, tid, nthr);
  __syncthreads();
  cx<T>* dst = U + (size_t(b - b_begin) * n_y + py0) * n_x;
  staged_copy<kFftMaxV>(
      nr * n_x, tid, nthr,
      [&](int q) {
        const int r = div_nx(q);
        return buf[r * bstride + lpos(q - r * n_x)];
      },
      [&](int q, cx<T> v) { dst[q] = v; });
}

template <typename T>
hipError_t launch_fft_x_t(const DevPlan& p, const void* V, void* U, int b_begin, int b_end, hipStream_t s) {
  const FftCfg cfg = fft_cfg();
  const int rows = fft_batch<T>(p.n_x, cfg.threads, cfg.cap);
  const size_t lds = size_t(rows) * lseq(p.n_x) * sizeof(cx<T>);
  if (size_t(rows) * p.n_x > size_t(kFftMaxV) * cfg.threads || size_t(rows) * p.Nx > size_t(kFftMaxV) * cfg.threads ||
      b_begin < 0 || b_end > p.nb || b_begin >= b_end)
    return hipErrorInvalidValue;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_x_t<T>), lds);
  if (e != hipSuccess) return e;
  dim3 grid((p.n_y + rows - 1) / rows, b_end - b_begin);
  hipLaunchKernelGGL(k_fft_x_t<T>, grid, dim3(cfg.threads), lds, s, static_cast<const cx<T>*>(V), p.n_y, p.Nx, rows,
                     b_begin, as_desc<T>(p.f_nx), static_cast<cx<T>*>(U));
  return hipGetLastError();
}

// Batched forms of the x and y passes.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_x_batch(const FftXBA* __restrict__ args,
                                                             const int* __restrict__ prefix, int nprob, int total,
                                                             BatchIO io) {
  __shared__ BatchMeta<FftXBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const FftXBA a = batch_args(meta, p);
    const int local = w - meta.prefix[p];
    const int by = local / a.gx;
    fft_x_body<T>(static_cast<const cx<T>*>(a.U), a.n_y, a.Nx, a.rows, 0, view_desc<T>(a.fd),
                  static_cast<cx<T>*>(a.V), 0, local - by * a.gx, by, a.brange, loop_lane());
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_fft_y_batch(const FftYBA* __restrict__ args,
                                                             const int* __restrict__ prefix, int nprob, int total,
                                                             BatchIO io) {
  __shared__ BatchMeta<FftYBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const FftYBA a = batch_args(meta, p);
    const int local = w - meta.prefix[p];
    int by = local / a.gx, bx = local - by * a.gx;
    if (a.ylist) {  // the problem's work items inside its ranges
      const int e = a.ylist[local];
      by = e >> 16;
      bx = e & 0xffff;
    }
    fft_y_body<T>(static_cast<const cx<T>*>(a.V), a.nb, a.Nx, a.Ny, a.bins, static_cast<const T*>(a.dcx),
                  static_cast<const T*>(a.dcy), view_desc<T>(a.fd), static_cast<cx<T>*>(a.Gh), 0, bx, by, a.jrange,
                  loop_lane());
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_fft_x_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_x_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_x_batch<T>), dim3(batch_grid(st)), dim3(kFftThreads), st.lds, s,
                     static_cast<const FftXBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_y_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_fft_y_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fft_y_batch<T>), dim3(batch_grid(st)), dim3(kFftThreads), st.lds, s,
                     static_cast<const FftYBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T)                                                                    \
  template hipError_t launch_fft_x<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_fft_y<T>(const DevPlan&, const void*, void*, hipStream_t);          \
  template hipError_t launch_fft_y_t<T>(const DevPlan&, const void*, void*, hipStream_t);        \
  template hipError_t launch_fft_x_t<T>(const DevPlan&, const void*, void*, int, int, hipStream_t); \
  template hipError_t launch_fft_x_batch<T>(const BatchStage&, const BatchIO&, hipStream_t); \
  template hipError_t launch_fft_y_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
