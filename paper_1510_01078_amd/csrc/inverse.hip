// Equispaced inverse 3-D FFT of the weighted spectrum (the last step of the
// NEDNER list in Section 3), and its transpose for the forward model.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
// Stage 5: equispaced inverse 3-D FFT (step 3 of the NEDNER list) on the
// half spectrum Fh[jj][kk][l], l = 0..Nz/2: in-place inverse transforms
// along x and along y, then a complex-to-real transform along z.
// ---------------------------------------------------------------------------
template <typename T, bool INV, int NCT = 0>
__device__ __forceinline__ void cfft_x_body(cx<T>* __restrict__ F, int Ny, int Lh, int lchunk,
                                            FftDesc<T> fd, int wm, int bx, int by) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Nx = NCT > 0 ? NCT : fd.n;
  const int bstride = lseq(Nx);
  const int kk = by;
  const int l0 = bx * lchunk;
  const int nl = min(lchunk, Lh - l0);
  cx<T>* base = F + size_t(kk) * Lh + l0;  // x mode jj, z mode l0 + li at base[jj * Ny * Lh + li]
  const size_t col = size_t(Ny) * Lh;
  cx<T>* twl = buf + lchunk * bstride;  // the twiddles go to LDS behind the rows
  if constexpr (NCT > 0) {
    // compile-time geometry (lchunk = ROWS z modes, 256 threads): no index divisions
    constexpr int ROWS = ct_maxb(NCT, kInvCap), BS = lseq(NCT), U = NCT * ROWS / kFftThreads;
    cx<T>* b0 = base + size_t(tid / ROWS) * col + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * col;
    staged_cols<ROWS, kFftThreads, U>(
        NCT, nl, tid, [&](int, int, int u) { return b0[u * step]; },
        [&](int jj, int li, int, cx<T> v) { buf[li * BS + lpos(jj)] = v; });
    for (int t = tid; t < NCT; t += kFftThreads) twl[t] = fd.tw[t];
    __syncthreads();
    fft_ct<T, NCT, kFftThreads, ROWS, INV>(buf, nl, twl, tid);
    __syncthreads();
    staged_cols<ROWS, kFftThreads, U>(
        NCT, nl, tid, [&](int jj, int li, int) { return buf[li * BS + lpos(jj)]; },
        [&](int, int, int u, cx<T> v) { b0[u * step] = v; });
  } else {
    const FastDiv div_nl(nl);
    staged_copy<kFftMaxV>(
        nl * Nx, tid, nthr,
        [&](int q) {
          const int jj = div_nl(q);
          return base[jj * col + (q - jj * nl)];
        },
        [&](int q, cx<T> v) {
          const int jj = div_nl(q);
          buf[(q - jj * nl) * bstride + lpos(jj)] = v;
        });
    for (int t = tid; t < fd.n; t += nthr) twl[t] = fd.tw[t];
    __syncthreads();
    fft_group<T, INV>(buf, lds_twiddles(fd, twl), nl, bstride, tid, nthr, wm);
    __syncthreads();
    staged_copy<kFftMaxV>(
        nl * Nx, tid, nthr,
        [&](int q) {
          const int jj = div_nl(q);
          return buf[(q - jj * nl) * bstride + lpos(jj)];
        },
        [&](int q, cx<T> v) {
          const int jj = div_nl(q);
          base[jj * col + (q - jj * nl)] = v;
        });
  }
}

template <typename T, bool INV, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_cfft_x(cx<T>* __restrict__ F, int Ny, int Lh, int lchunk,
                                                      FftDesc<T> fd, int wm) {
  // neighbouring groups share the 128-byte lines of the z runs: keep them on one XCD
  const int gl = xcd_linear();
  cfft_x_body<T, INV, NCT>(F, Ny, Lh, lchunk, fd, wm, gl % gridDim.x, gl / gridDim.x);
}

template <typename T, bool INV, int NCT = 0>
__device__ __forceinline__ void cfft_y_body(cx<T>* __restrict__ F, int Lh, int lchunk, FftDesc<T> fd, int wm, int bx,
                                            int by, int tid = threadIdx.x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nthr = blockDim.x;
  const int Ny = NCT > 0 ? NCT : fd.n;
  const int bstride = lseq(Ny);
  const int jj = by;
  const int l0 = bx * lchunk;
  const int nl = min(lchunk, Lh - l0);
  cx<T>* base = F + size_t(jj) * Ny * Lh + l0;
  cx<T>* twl = buf + lchunk * bstride;  // the twiddles go to LDS behind the rows
  if constexpr (NCT > 0) {
    // compile-time geometry (lchunk = ROWS z modes, 256 threads): no index divisions
    constexpr int ROWS = ct_maxb(NCT, kInvCap), BS = lseq(NCT), U = NCT * ROWS / kFftThreads;
    cx<T>* b0 = base + size_t(tid / ROWS) * Lh + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * Lh;
    staged_cols<ROWS, kFftThreads, U>(
        NCT, nl, tid, [&](int, int, int u) { return b0[u * step]; },
        [&](int kk, int li, int, cx<T> v) { buf[li * BS + lpos(kk)] = v; });
    for (int t = tid; t < NCT; t += kFftThreads) twl[t] = fd.tw[t];
    __syncthreads();
    fft_ct<T, NCT, kFftThreads, ROWS, INV>(buf, nl, twl, tid);
    __syncthreads();
    staged_cols<ROWS, kFftThreads, U>(
        NCT, nl, tid, [&](int kk, int li, int) { return buf[li * BS + lpos(kk)]; },
        [&](int, int, int u, cx<T> v) { b0[u * step] = v; });
  } else {
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
    for (int t = tid; t < fd.n; t += nthr) twl[t] = fd.tw[t];
    __syncthreads();
    fft_group<T, INV>(buf, lds_twiddles(fd, twl), nl, bstride, tid, nthr, wm);
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
}

template <typename T, bool INV, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_cfft_y(cx<T>* __restrict__ F, int Lh, int lchunk, FftDesc<T> fd,
                                                      int wm) {
  // neighbouring groups share the 128-byte lines of the z runs: keep them on one XCD
  const int gl = xcd_linear();
  cfft_y_body<T, INV, NCT>(F, Lh, lchunk, fd, wm, gl % gridDim.x, gl / gridDim.x);
}

template <typename T, int NCT = 0>
__device__ __forceinline__ void c2r_z_body(const cx<T>* __restrict__ F, long long nrows, int rows,
                                           FftDesc<T> fd, T* __restrict__ f, int wm, int bx, int tid = threadIdx.x) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int nthr = blockDim.x;
  const int Nz = NCT > 0 ? NCT : fd.n;
  const int Lh = Nz / 2 + 1;
  const int bstride = lseq(Nz);
  const long long r0 = (long long)bx * rows;
  const int nr = (int)min((long long)rows, nrows - r0);
  // two real rows per complex transform: Z = X0 + i X1 (each Hermitian-
  // extended) transforms to x0 + i x1. The DC and Nyquist bins keep their
  // real parts only, as the real part of a single row's transform would.
  const int np = (nr + 1) / 2;
  const FastDiv fdiv_lh(Lh), fdiv_nz(Nz);
  // compile-time lengths divide by constants (a shift for Nz)
  auto div_lh = [&](int q) { return NCT > 0 ? int(unsigned(q) / unsigned(NCT / 2 + 1)) : fdiv_lh(q); };
  auto div_nz = [&](int q) { return NCT > 0 ? int(unsigned(q) / unsigned(NCT > 0 ? NCT : 1)) : fdiv_nz(q); };
  struct Two {
    cx<T> a, c;
  };
  // values staged per thread: what the pairs of a compile-time length need
  // (5 at 256 points), else kC2rStage; kFftMaxV held 64 registers for the
  // pairs (launches check np * Lh <= kC2rStage * threads)
  constexpr int UL = NCT > 0 ? ((ct_maxb(NCT, kInvCap) + 1) / 2 * (NCT / 2 + 1) + kFftThreads - 1) / kFftThreads
                             : kC2rStage;
  staged_copy<UL>(
      np * Lh, tid, nthr,
      [&](int q) {
        const int s = div_lh(q);
        const long long at = (r0 + 2 * s) * Lh + (q - s * Lh);
        return Two{F[at], 2 * s + 1 < nr ? F[at + Lh] : cx<T>{T(0), T(0)}};
      },
      [&](int q, Two v) {
        const int s = div_lh(q);
        const int l = q - s * Lh;
        cx<T>* row = buf + s * bstride;
        if (l == 0 || l == Nz / 2) {
          row[lpos(l)] = cx<T>{v.a.x, v.c.x};
        } else {
          row[lpos(l)] = cx<T>{v.a.x - v.c.y, v.a.y + v.c.x};
          row[lpos(Nz - l)] = cx<T>{v.a.x + v.c.y, v.c.x - v.a.y};
        }
      });
  // the sequences hold (rows + 1) / 2 pairs: the twiddles go behind them,
  // and the transform is compiled for that many (with LDS and registers for
  // `rows` sequences, half unused, the kernel held 100 registers and 37 KiB
  // of LDS per work-group at 256 points: 4 per CU)
  cx<T>* twl = buf + (rows + 1) / 2 * bstride;
  for (int t = tid; t < (NCT > 0 ? NCT : fd.n); t += nthr) twl[t] = fd.tw[t];
  __syncthreads();
  if constexpr (NCT > 0)
    fft_ct<T, NCT, kFftThreads, (ct_maxb(NCT, kInvCap) + 1) / 2, true>(buf, np, twl, tid);
  else
    fft_group<T, true>(buf, lds_twiddles(fd, twl), np, bstride, tid, nthr, wm);
  __syncthreads();
  staged_copy<kFftMaxV>(
      nr * Nz, tid, nthr,
      [&](int q) {
        const int r = div_nz(q);
        const cx<T> v = buf[(r >> 1) * bstride + lpos(q - r * Nz)];
        return (r & 1) ? v.y : v.x;
      },
      [&](int q, T v) { f[r0 * Nz + q] = v; });
}

template <typename T, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_c2r_z(const cx<T>* __restrict__ F, long long nrows, int rows,
                                                     FftDesc<T> fd, T* __restrict__ f, int wm) {
  c2r_z_body<T, NCT>(F, nrows, rows, fd, f, wm, blockIdx.x);
}

// Transpose of k_c2r_z for the forward model: real rows f[r][e] ->
// Dh[r][l] = sum_e f[r][e] exp(-2 pi i l e/Nz), l = 0..Nz/2. Two real rows
// share one complex transform, Z = FFT(x0 + i x1): X0[l] = (Z[l] + conj
// Z[-l])/2 and X1[l] = (Z[l] - conj Z[-l])/(2i), so a work-group of `rows`
// rows transforms (rows + 1) / 2 sequences (half the transforms, LDS and
// registers of one sequence per row).
template <typename T, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_r2c_z(const T* __restrict__ f, long long nrows, int rows,
                                                     FftDesc<T> fd, cx<T>* __restrict__ D) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Nz = NCT > 0 ? NCT : fd.n;
  const int Lh = Nz / 2 + 1;
  const int bstride = lseq(Nz);
  const long long r0 = (long long)blockIdx.x * rows;
  const int nr = (int)min((long long)rows, nrows - r0);
  const int np = (nr + 1) / 2;
  const FastDiv fdiv_lh(Lh), fdiv_nz(Nz);
  // compile-time lengths divide by constants (a shift for Nz)
  auto div_lh = [&](int q) { return NCT > 0 ? int(unsigned(q) / unsigned(NCT / 2 + 1)) : fdiv_lh(q); };
  auto div_nz = [&](int q) { return NCT > 0 ? int(unsigned(q) / unsigned(NCT > 0 ? NCT : 1)) : fdiv_nz(q); };
  struct Two {
    T a, b;
  };
  // values staged per thread: what a compile-time length needs, else
  // kFftMaxV (np * Nz <= rows * Nz / 2 + Nz / 2 <= 3 * 1024 by fft_batch)
  constexpr int ROWS = NCT > 0 ? ct_maxb(NCT, kInvCap) : 1;
  constexpr int UL = NCT > 0 ? ((ROWS + 1) / 2 * NCT + kFftThreads - 1) / kFftThreads : kFftMaxV;
  constexpr int UO = NCT > 0 ? (ROWS * (NCT / 2 + 1) + kFftThreads - 1) / kFftThreads : kFftMaxV;
  staged_copy<UL>(
      np * Nz, tid, nthr,
      [&](int q) {
        const int s = div_nz(q);
        const long long at = (r0 + 2 * s) * Nz + (q - s * Nz);
        return Two{f[at], 2 * s + 1 < nr ? f[at + Nz] : T(0)};
      },
      [&](int q, Two v) {
        const int s = div_nz(q);
        buf[s * bstride + lpos(q - s * Nz)] = cx<T>{v.a, v.b};
      });
  cx<T>* twl = buf + (rows + 1) / 2 * bstride;
  for (int t = tid; t < (NCT > 0 ? NCT : fd.n); t += nthr) twl[t] = fd.tw[t];
  __syncthreads();
  if constexpr (NCT > 0)
    fft_ct<T, NCT, kFftThreads, (ROWS + 1) / 2, false>(buf, np, twl, tid);
  else
    fft_lds<T, kFftMaxV, false, false>(buf, lds_twiddles(fd, twl), np, bstride, tid, nthr);
  __syncthreads();
  staged_copy<UO>(
      nr * Lh, tid, nthr,
      [&](int q) {
        const int r = div_lh(q);
        const int l = q - r * Lh;
        const cx<T>* row = buf + (r >> 1) * bstride;
        const cx<T> z = row[lpos(l)];
        const cx<T> zm = row[lpos(l == 0 ? 0 : Nz - l)];
        return (r & 1) ? cx<T>{T(0.5) * (z.y + zm.y), T(-0.5) * (z.x - zm.x)}
                       : cx<T>{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
      },
      [&](int q, cx<T> v) { D[r0 * Lh + q] = v; });
}

// In-place transforms of the half spectrum along x and y (INV: e^{+i}).
template <typename T, bool INV>
static hipError_t launch_xy(const DevPlan& p, cx<T>* F, bool x_first, hipStream_t s, int first_pass = 0) {
  const int Lh = p.Nz / 2 + 1;
  const FftCfg cfg = inv_cfg();
  for (int pass = first_pass; pass < 2; ++pass) {
    const bool along_x = (pass == 0) == x_first;
    hipError_t e;
    if (along_x) {
      const int lc = fft_batch<T>(p.Nx, cfg.threads, cfg.cap);
      const size_t lds = (size_t(lc) * lseq(p.Nx) + p.Nx) * sizeof(cx<T>);
      e = ct_pick(CtInverse{}, p.Nx, [&](auto c) {
        constexpr int NCT = decltype(c)::value;
        // the compile-time kernels take their geometry from the length
        if (NCT > 0 && (lc != ct_maxb(NCT, kInvCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
        const void* kern = reinterpret_cast<const void*>(&k_cfft_x<T, INV, NCT>);
        hipError_t e2 = allow_lds(kern, lds);
        if (e2 != hipSuccess) return e2;
        dim3 grid((Lh + lc - 1) / lc, p.Ny);
        hipLaunchKernelGGL((k_cfft_x<T, INV, decltype(c)::value>), grid, dim3(cfg.threads), lds, s, F, p.Ny, Lh, lc,
                           as_desc<T>(p.f_Nx), cfg.wave);
        return hipGetLastError();
      });
    } else {
      const int lc = fft_batch<T>(p.Ny, cfg.threads, cfg.cap);
      const size_t lds = (size_t(lc) * lseq(p.Ny) + p.Ny) * sizeof(cx<T>);
      e = ct_pick(CtInverse{}, p.Ny, [&](auto c) {
        constexpr int NCT = decltype(c)::value;
        if (NCT > 0 && (lc != ct_maxb(NCT, kInvCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
        const void* kern = reinterpret_cast<const void*>(&k_cfft_y<T, INV, NCT>);
        hipError_t e2 = allow_lds(kern, lds);
        if (e2 != hipSuccess) return e2;
        dim3 grid((Lh + lc - 1) / lc, p.Nx);
        hipLaunchKernelGGL((k_cfft_y<T, INV, decltype(c)::value>), grid, dim3(cfg.threads), lds, s, F, Lh, lc,
                           as_desc<T>(p.f_Ny), cfg.wave);
        return hipGetLastError();
      });
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_inverse(const DevPlan& p, void* Fh, T* f, hipStream_t s, bool x_done) {
  cx<T>* F = static_cast<cx<T>*>(Fh);
  hipError_t e = launch_xy<T, true>(p, F, true, s, x_done ? 1 : 0);
  if (e != hipSuccess) return e;
  const FftCfg cfg = inv_cfg();
  const int rows = fft_batch<T>(p.Nz, cfg.threads, cfg.cap);
  const size_t lds = size_t(c2r_lds_slots(rows, p.Nz)) * sizeof(cx<T>);
  const long long nrows = (long long)p.Nx * p.Ny;
  if ((rows + 1) / 2 * (p.Nz / 2 + 1) > kC2rStage * cfg.threads) return hipErrorInvalidValue;
  return ct_pick(CtInverse{}, p.Nz, [&](auto c) {
    hipError_t e2 = allow_lds(reinterpret_cast<const void*>(&k_c2r_z<T, decltype(c)::value>), lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL((k_c2r_z<T, decltype(c)::value>), dim3((unsigned)((nrows + rows - 1) / rows)),
                       dim3(cfg.threads), lds, s, F, nrows, rows, as_desc<T>(p.f_Nz), f, cfg.wave);
    return hipGetLastError();
  });
}

template <typename T>
hipError_t launch_forward3d(const DevPlan& p, const T* f, void* Dh, hipStream_t s) {
  cx<T>* D = static_cast<cx<T>*>(Dh);
  const FftCfg cfg = inv_cfg();
  const int rows = fft_batch<T>(p.Nz, cfg.threads, cfg.cap);
  const size_t lds = size_t(c2r_lds_slots(rows, p.Nz)) * sizeof(cx<T>);  // (rows + 1) / 2 sequences
  const long long nrows = (long long)p.Nx * p.Ny;
  if ((rows + 1) / 2 * p.Nz > kFftMaxV * cfg.threads || rows * (p.Nz / 2 + 1) > kFftMaxV * cfg.threads)
    return hipErrorInvalidValue;
  hipError_t e = ct_pick(CtInverse{}, p.Nz, [&](auto c) {
    hipError_t e2 = allow_lds(reinterpret_cast<const void*>(&k_r2c_z<T, decltype(c)::value>), lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL((k_r2c_z<T, decltype(c)::value>), dim3((unsigned)((nrows + rows - 1) / rows)),
                       dim3(cfg.threads), lds, s, f, nrows, rows, as_desc<T>(p.f_Nz), D);
    return hipGetLastError();
  });
  if (e != hipSuccess) return e;
  return launch_xy<T, false>(p, D, false, s);
}


// Batched forms of the inverse passes.
template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_cfft_y_inv_batch(const CfftBA* __restrict__ args,
                                                                  const int* __restrict__ prefix, int nprob, int total,
                                                                  BatchIO io) {
  __shared__ BatchMeta<CfftBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const CfftBA a = batch_args(meta, p);
    const int local = w - meta.prefix[p];
    const int by = local / a.gx;
    cfft_y_body<T, true>(static_cast<cx<T>*>(a.F), a.Lh, a.lchunk, view_desc<T>(a.fd), 0, local - by * a.gx, by,
                         loop_lane());
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_c2r_z_batch(const C2rBA* __restrict__ args,
                                                             const int* __restrict__ prefix, int nprob, int total,
                                                             BatchIO io) {
  __shared__ BatchMeta<C2rBA> meta;
  batch_meta_load(meta, args, prefix, nprob);
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const C2rBA a = batch_args(meta, p);
    c2r_z_body<T>(static_cast<const cx<T>*>(a.F), a.nrows, a.rows, view_desc<T>(a.fd), static_cast<T*>(io.out[p]), 0,
                  w - meta.prefix[p]);  // (a re-read lane index raised its registers here)
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_cfft_y_inv_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_cfft_y_inv_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_cfft_y_inv_batch<T>), dim3(batch_grid(st)), dim3(kFftThreads), st.lds, s,
                     static_cast<const CfftBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_c2r_z_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_c2r_z_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_c2r_z_batch<T>), dim3(batch_grid(st)), dim3(kFftThreads), st.lds, s,
                     static_cast<const C2rBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T)                                                                \
  template hipError_t launch_inverse<T>(const DevPlan&, void*, T*, hipStream_t, bool); \
  template hipError_t launch_forward3d<T>(const DevPlan&, const T*, void*, hipStream_t); \
  template hipError_t launch_cfft_y_inv_batch<T>(const BatchStage&, const BatchIO&, hipStream_t); \
  template hipError_t launch_c2r_z_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
