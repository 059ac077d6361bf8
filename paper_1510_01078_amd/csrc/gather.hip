// Temporal interpolation at omega(K) with the inversion weight
// (Section 3.1, eq. NER_NUFFT; Section 2, eq. exact), the adjoint's
// cos(c|K|t) form of it, and the exact transpose used by the forward model.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "kernels_common.hpp"

namespace patk {

// Interpolation point of lattice mode (j, k, l >= 0): s = c|K| dt n_t/(2 pi)
// in oversampled bins (double), the first band bin of its w_t taps (clamped
// to the band), the tap argument y = 2 frac(s) - 1 and the centring phase
// exp(-2 pi i s n0/n_t) of eq. PSI (samples sit at n - n0 in the FFT).
struct TapPoint {
  int base;
  double y;
  double cs, sn;
};

template <typename T>
__device__ __forceinline__ TapPoint tap_point(double Kabs, double s_per_k, double n0_over_nt, int wt, int b_lo,
                                              int nb) {
  TapPoint tp;
  const double s = Kabs * s_per_k;
  const double fl = floor(s);
  tp.y = 2.0 * (s - fl) - 1.0;
  int base = int(fl) - wt / 2 + 1 - b_lo;
  tp.base = base < 0 ? 0 : (base > nb - wt ? nb - wt : base);
  double q = s * n0_over_nt;
  if constexpr (sizeof(T) == 4) {
    // FP32 plans round the phase to FP32 anyway: reduce q to [-1/2, 1/2] in
    // FP64 (its FP32 rounding then errs by at most 3e-8) and take the FP32
    // sincospi, a fraction of the FP64 one's instructions
    q -= rint(q);
    float sn, cs;
    sincospif(float(-2.0 * q), &sn, &cs);  // e^{-2 pi i q}
    tp.sn = sn;
    tp.cs = cs;
  } else {
    q -= floor(q);
    sincospi(-2.0 * q, &tp.sn, &tp.cs);  // e^{-2 pi i q}; no range reduction needed
  }
  return tp;
}

// |K| and 1/|K| of a lattice point from one reciprocal square root (no FP64
// division for the weight W); K = 0 keeps |K| = 0. The interpolation and its
// transpose both take |K| from here, so they choose the same first tap bin
// and weights for every lattice point, bit for bit: where s = |K| c dt n_t /
// (2 pi) is an integer, two roundings of |K| could otherwise pick bases one
// bin apart (both valid interpolations, but no longer exact transposes).
__device__ __forceinline__ double lattice_kabs(double Kx, double Ky, double Kz, double& rK) {
  const double K2 = Kx * Kx + Ky * Ky + Kz * Kz;
  rK = K2 > 0.0 ? rsqrt(K2) : 0.0;
  return K2 * rK;
}

// Tap weight t of the temporal window at argument y (Horner on the per-tap
// polynomial fitted at plan time).
template <typename T>
__device__ __forceinline__ T tap_weight(const T* __restrict__ hcoef, int t, int deg, T y) {
  const T* c = hcoef + t * (deg + 1);
  T v = c[deg];
  for (int d = deg - 1; d >= 0; --d) v = v * y + c[d];
  return v;
}

// Compile-time tap count WT: the coefficients sit in LDS by degree
// (c[d*WT + t] is the y^d coefficient of tap t), and all taps' Horner chains
// advance together, so the multiply-adds of different taps are independent
// and the coefficient reads are LDS broadcasts. Same operations per tap as
// tap_weight (the batched gather's form); the batch tests check that both
// give the same bits.

template <typename T, int WT>
__device__ __forceinline__ void stage_tap_coefs(T* c, const T* __restrict__ hcoef, int deg) {
  for (int q = threadIdx.x; q < WT * (deg + 1); q += blockDim.x) {
    const int t = q / (deg + 1);
    c[(q - t * (deg + 1)) * WT + t] = hcoef[q];
  }
}

template <typename T, int WT>
__device__ __forceinline__ void tap_weights(const T* c, int deg, T y, T (&v)[WT]) {
#pragma unroll
  for (int t = 0; t < WT; ++t) v[t] = c[deg * WT + t];
  for (int d = deg - 1; d >= 0; --d) {
#pragma unroll
    for (int t = 0; t < WT; ++t) v[t] = v[t] * y + c[d * WT + t];
  }
}

// ---------------------------------------------------------------------------
// Stage 4: temporal interpolation, one thread per (j, k, l), l = 0..Nz/2.
//   S+(K) = exp(-2 pi i s n0/n_t) sum_t phi_t(s - b_t) Gh[j][k][b_t]
// MODE_IMAGE / MODE_PHYSICAL (reconstruction, eq. exact):
//   F = 2c Kz/|K| * S+ on l = 1..Nz/2-1; 0 on l = 0, l = Nz/2 and the
//   j = -Nx/2, k = -Ny/2 planes. MODE_IMAGE scales by 1/(XYZ) for the
//   inverse transform; MODE_PHYSICAL restores the (-1)^(j+k) sign of the
//   centred lateral coordinates instead.
// MODE_ADJOINT (adjoint of the forward model): the time kernel is
//   cos(c|K|t) = (e^{-i c|K| t} + e^{+i c|K| t})/2, and the second term is
//   the conjugate of S+ at (-Kx, -Ky) because the data are real, so
//   F = scale * (S+(j,k,l) + conj S+(-j,-k,l)) on l = 0..Nz/2-1 (l = 0
//   included), 0 on l = Nz/2 and the two lateral Nyquist planes.
// ---------------------------------------------------------------------------
enum { MODE_IMAGE = 0, MODE_PHYSICAL = 1, MODE_ADJOINT = 2 };

// WT > 0: compile-time tap count with the coefficients staged in LDS at
// `coefs` (stage_tap_coefs, before the call); WT = 0: runtime wt, coefficients
// read from hcoef.
// One spectrum value F(jj, kk, l) of the given mode.
template <typename T, int MODE, int WT = 0>
__device__ __forceinline__ cx<T> gather_point(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                              double s_per_k, double kxu, double kyu, double kzu, double two_c,
                                              double n0_over_nt, double scale, int wt, int deg,
                                              const T* __restrict__ hcoef, int jj, int kk, int l,
                                              const T* coefs) {
  const bool zero_l = MODE == MODE_ADJOINT ? (l == Nz / 2) : (l == 0 || l == Nz / 2);
  if (zero_l || jj == Nx / 2 || kk == Ny / 2) return cx<T>{T(0), T(0)};
  const long long col = (long long)jj * Ny + kk;
  const int j = jj < Nx / 2 ? jj : jj - Nx;
  const int k = kk < Ny / 2 ? kk : kk - Ny;
  const double Kx = j * kxu, Ky = k * kyu, Kz = l * kzu;
  double rK;
  const double Kabs = lattice_kabs(Kx, Ky, Kz, rK);
  const TapPoint tp = tap_point<T>(Kabs, s_per_k, n0_over_nt, wt, b_lo, nb);
  const T y = T(tp.y);
  const cx<T>* src = Gh + col * nb + tp.base;
  const cx<T>* src2 = Gh + ((long long)((Nx - jj) % Nx) * Ny + (Ny - kk) % Ny) * nb + tp.base;
  cx<T> acc{T(0), T(0)}, acc2{T(0), T(0)};
  if constexpr (WT > 0) {
    cx<T> gv[WT], gv2[MODE == MODE_ADJOINT ? WT : 1];
#pragma unroll
    for (int t = 0; t < WT; ++t) {
      gv[t] = src[t];
      if (MODE == MODE_ADJOINT) gv2[t] = src2[t];
    }
    T v[WT];
    tap_weights<T, WT>(coefs, deg, y, v);
#pragma unroll
    for (int t = 0; t < WT; ++t) {
      acc.x += v[t] * gv[t].x;
      acc.y += v[t] * gv[t].y;
      if (MODE == MODE_ADJOINT) {
        acc2.x += v[t] * gv2[t].x;
        acc2.y += v[t] * gv2[t].y;
      }
    }
  } else {
    for (int t = 0; t < wt; ++t) {
      const T v = tap_weight(hcoef, t, deg, y);
      const cx<T> gv = src[t];
      acc.x += v * gv.x;
      acc.y += v * gv.y;
      if (MODE == MODE_ADJOINT) {
        const cx<T> gv2 = src2[t];
        acc2.x += v * gv2.x;
        acc2.y += v * gv2.y;
      }
    }
  }
  if (MODE == MODE_ADJOINT) {
    const cx<T> ph{T(tp.cs * scale), T(tp.sn * scale)};
    const cx<T> a = cmul(acc, ph), b = cmul(acc2, ph);
    return cx<T>{a.x + b.x, a.y - b.y};
  }
  double wgt = two_c * Kz * rK * scale;
  if (MODE == MODE_PHYSICAL && ((jj + kk) & 1)) wgt = -wgt;
  const cx<T> ph{T(wgt * tp.cs), T(wgt * tp.sn)};
  return cmul(acc, ph);
}

template <typename T, int MODE, int WT = 0>
__device__ __forceinline__ void gather_body(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                            double s_per_k, double kxu, double kyu, double kzu, double two_c,
                                            double n0_over_nt, double scale, int wt, int deg,
                                            const T* __restrict__ hcoef, cx<T>* __restrict__ Fh, int bx,
                                            const T* coefs = nullptr) {
  const int Lh = Nz / 2 + 1;
  const long long total = (long long)Nx * Ny * Lh;
  const long long idx = (long long)bx * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int l = int(idx % Lh);
  const long long col = idx / Lh;
  const int kk = int(col % Ny);
  const int jj = int(col / Ny);
  Fh[idx] = gather_point<T, MODE, WT>(Gh, nb, b_lo, Nx, Ny, Nz, s_per_k, kxu, kyu, kzu, two_c, n0_over_nt, scale, wt,
                                      deg, hcoef, jj, kk, l, coefs);
}

template <typename T, int MODE, int WT>
__global__ __launch_bounds__(256) void k_gather(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                                double s_per_k, double kxu, double kyu, double kzu, double two_c,
                                                double n0_over_nt, double scale, int wt, int deg,
                                                const T* __restrict__ hcoef, cx<T>* __restrict__ Fh) {
  __shared__ T coefs[kMaxTapCoefs];
  stage_tap_coefs<T, WT>(coefs, hcoef, deg);
  __syncthreads();
  gather_body<T, MODE, WT>(Gh, nb, b_lo, Nx, Ny, Nz, s_per_k, kxu, kyu, kzu, two_c, n0_over_nt, scale, wt, deg, hcoef,
                           Fh, blockIdx.x, coefs);
}

// Gather fused with the first pass of the inverse 3-D FFT (image and
// adjoint modes): a work-group owns one y mode kk and a run of lchunk z
// modes, computes the spectrum for every x mode into LDS, transforms along x
// there (the same transform and layout as the inverse x pass) and writes the
// x-transformed values once. The spectrum itself never goes through HBM.
template <typename T, int MODE, int WT, int NCT>
__device__ __forceinline__ void gather_x_body(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                              double s_per_k, double kxu, double kyu, double kzu, double two_c,
                                              double n0_over_nt, double scale, int wt, int deg,
                                              const T* __restrict__ hcoef, int lchunk, FftDesc<T> fd, int wm,
                                              cx<T>* __restrict__ F, int bx, int kk, const T* coefs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Lh = Nz / 2 + 1;
  const int bstride = lseq(Nx);
  const int l0 = bx * lchunk;
  const int nl = min(lchunk, Lh - l0);
  cx<T>* twl = buf + lchunk * bstride;  // the twiddles go to LDS behind the rows
  for (int t = tid; t < (NCT > 0 ? NCT : fd.n); t += nthr) twl[t] = fd.tw[t];
  __syncthreads();
  const FastDiv div_nl(nl);
  // (one loop form for every length: the batched reconstruction runs this
  // loop too, and the same code keeps the two paths' values bit for bit equal)
  constexpr int ROWS = NCT > 0 ? ct_maxb(NCT, kGatherCap) : 1;
  for (int q = tid; q < nl * Nx; q += nthr) {
    const int jj = div_nl(q);
    const int li = q - jj * nl;
    buf[li * bstride + lpos(jj)] =
        gather_point<T, MODE, WT>(Gh, nb, b_lo, Nx, Ny, Nz, s_per_k, kxu, kyu, kzu, two_c, n0_over_nt, scale, wt,
                                  deg, hcoef, jj, kk, l0 + li, coefs);
  }
  __syncthreads();
  if constexpr (NCT > 0)
    fft_ct<T, NCT, kFftThreads, ROWS, true>(buf, nl, twl, tid);
  else
    fft_group<T, true>(buf, lds_twiddles(fd, twl), nl, bstride, tid, nthr, wm);
  __syncthreads();
  cx<T>* base = F + size_t(kk) * Lh + l0;  // x mode jj, z mode l0 + li at base[jj * Ny * Lh + li]
  const size_t col = size_t(Ny) * Lh;
  if constexpr (NCT > 0) {
    cx<T>* b0 = base + size_t(tid / ROWS) * col + tid % ROWS;
    const size_t step = size_t(kFftThreads / ROWS) * col;
    staged_cols<ROWS, kFftThreads, NCT * ROWS / kFftThreads>(  // Nx = NCT
        NCT, nl, tid, [&](int jj, int li, int) { return buf[li * bstride + lpos(jj)]; },
        [&](int, int, int u, cx<T> v) { b0[u * step] = v; });
  } else {
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

template <typename T, int MODE, int WT, int NCT>
__global__ __launch_bounds__(kFftThreads) void k_gather_x(const cx<T>* __restrict__ Gh, int nb, int b_lo, int Nx,
                                                        int Ny, int Nz, double s_per_k, double kxu, double kyu,
                                                        double kzu, double two_c, double n0_over_nt, double scale,
                                                        int wt, int deg, const T* __restrict__ hcoef, int lchunk,
                                                        FftDesc<T> fd, int wm, cx<T>* __restrict__ F) {
  __shared__ T coefs[kMaxTapCoefs];
  stage_tap_coefs<T, WT>(coefs, hcoef, deg);  // visible after the body's first barrier
  // neighbouring groups share the 128-byte lines of the z runs: keep them on one XCD
  const int gl = xcd_linear();
  const int kk = gl / int(gridDim.x);
  gather_x_body<T, MODE, WT, NCT>(Gh, nb, b_lo, Nx, Ny, Nz, s_per_k, kxu, kyu, kzu, two_c, n0_over_nt, scale, wt, deg,
                                  hcoef, lchunk, fd, wm, F, gl - kk * int(gridDim.x), kk, coefs);
}

// Compile-time tap counts: every even w_t in 2..16 (the plan's range).
template <class F>
static hipError_t wt_pick(int wt, F&& f) {
  switch (wt) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 10: return f(std::integral_constant<int, 10>{});
    case 12: return f(std::integral_constant<int, 12>{});
    case 14: return f(std::integral_constant<int, 14>{});
    case 16: return f(std::integral_constant<int, 16>{});
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_gather_x(const DevPlan& p, const void* Gh, void* F, int mode, hipStream_t s) {
  if (mode != GATHER_IMAGE && mode != GATHER_ADJOINT) return hipErrorInvalidValue;
  if (p.w_t * (p.hdeg + 1) > kMaxTapCoefs) return hipErrorInvalidValue;
  const int Lh = p.Nz / 2 + 1;
  const FftCfg cfg = inv_cfg();
  const int lc = fft_batch<T>(p.Nx, cfg.threads, kGatherCap);
  const size_t lds = (size_t(lc) * lseq(p.Nx) + p.Nx) * sizeof(cx<T>);
  const dim3 grid((Lh + lc - 1) / lc, p.Ny);
  const cx<T>* in = static_cast<const cx<T>*>(Gh);
  cx<T>* out = static_cast<cx<T>*>(F);
  const T* hc = static_cast<const T*>(p.hcoef);
  const bool adj = mode == GATHER_ADJOINT;
  const double scale = adj ? p.adj_scale : p.inv_vol;
  return wt_pick(p.w_t, [&](auto w) {
    constexpr int WT = decltype(w)::value;
    return ct_pick(CtInverse{}, p.Nx, [&](auto c) {
      constexpr int NCT = decltype(c)::value;
      // the compile-time kernels take their geometry from the length
      if (NCT > 0 && (lc != ct_maxb(NCT, kGatherCap) || cfg.threads != kFftThreads)) return hipErrorInvalidValue;
      const void* kern = adj ? reinterpret_cast<const void*>(&k_gather_x<T, MODE_ADJOINT, WT, NCT>)
                             : reinterpret_cast<const void*>(&k_gather_x<T, MODE_IMAGE, WT, NCT>);
      hipError_t e = allow_lds(kern, lds);
      if (e != hipSuccess) return e;
      if (adj)
        hipLaunchKernelGGL((k_gather_x<T, MODE_ADJOINT, WT, NCT>), grid, dim3(cfg.threads), lds, s, in, p.nb, p.b_lo,
                           p.Nx, p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, scale, p.w_t,
                           p.hdeg, hc, lc, as_desc<T>(p.f_Nx), cfg.wave, out);
      else
        hipLaunchKernelGGL((k_gather_x<T, MODE_IMAGE, WT, NCT>), grid, dim3(cfg.threads), lds, s, in, p.nb, p.b_lo,
                           p.Nx, p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, scale, p.w_t,
                           p.hdeg, hc, lc, as_desc<T>(p.f_Nx), cfg.wave, out);
      return hipGetLastError();
    });
  });
}

template <typename T>
hipError_t launch_gather(const DevPlan& p, const void* Gh, void* Fh, int mode, hipStream_t s) {
  const long long total = (long long)p.Nx * p.Ny * (p.Nz / 2 + 1);
  const unsigned blocks = (unsigned)((total + 255) / 256);
  const cx<T>* in = static_cast<const cx<T>*>(Gh);
  cx<T>* out = static_cast<cx<T>*>(Fh);
  const T* hc = static_cast<const T*>(p.hcoef);
  if (p.w_t * (p.hdeg + 1) > kMaxTapCoefs) return hipErrorInvalidValue;
  return wt_pick(p.w_t, [&](auto c) {
    constexpr int WT = decltype(c)::value;
    switch (mode) {
      case GATHER_IMAGE:
        hipLaunchKernelGGL((k_gather<T, MODE_IMAGE, WT>), dim3(blocks), dim3(256), 0, s, in, p.nb, p.b_lo, p.Nx,
                           p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, p.inv_vol, p.w_t, p.hdeg,
                           hc, out);
        break;
      case GATHER_PHYSICAL:
        hipLaunchKernelGGL((k_gather<T, MODE_PHYSICAL, WT>), dim3(blocks), dim3(256), 0, s, in, p.nb, p.b_lo, p.Nx,
                           p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, 1.0, p.w_t, p.hdeg, hc,
                           out);
        break;
      case GATHER_ADJOINT:
        hipLaunchKernelGGL((k_gather<T, MODE_ADJOINT, WT>), dim3(blocks), dim3(256), 0, s, in, p.nb, p.b_lo, p.Nx,
                           p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu, p.two_c, p.n0_over_nt, p.adj_scale, p.w_t,
                           p.hdeg, hc, out);
        break;
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  });
}

// ---------------------------------------------------------------------------
// Transpose of MODE_ADJOINT (the forward model's temporal step). Input: the
// forward-transformed image Dh[j][k][l], l = 0..Nz/2 (real-input transform
// along z, so Dh(-j,-k,l) pairs with Dh(j,k,-l)). One work-group owns the
// lateral column (j, k) and writes its band Gh'[j][k][0..nb):
//   Gh'[b] = sum_l phi_{b - base_l}(y_l) Z_l,
//   Z_l = scale c_l conj(phase_l) m(j,k) (Dh(j,k,l) + conj Dh(-j,-k,l)),
// over l = 0..Nz/2-1, with c_l = 1 at l = 0 and 2 otherwise (the two
// z-halves of the real-to-complex transform) and m = 1, i Kx or i Ky (the
// derivative of the traces in the sensor's x or y); Z = 0 on the Nyquist
// columns. Interpolation points and tap weights are computed exactly as in
// k_gather. Every bin sums its contributions in increasing l (the taps'
// first bins are non-decreasing in l), so the result is deterministic and
// atomic-free. A work-group handles a few consecutive columns so that the
// per-l phase keeps its threads busy.
// ---------------------------------------------------------------------------
template <typename T, int WT>
__global__ __launch_bounds__(256) void k_scatter(const cx<T>* __restrict__ Dh, int nb, int b_lo, int Nx, int Ny, int Nz,
                                                 double s_per_k, double kxu, double kyu, double kzu, double n0_over_nt,
                                                 double scale, int deriv, int wt, int deg, const T* __restrict__ hcoef,
                                                 int cols_per_group, int first_table, const int* __restrict__ jrange,
                                                 cx<T>* __restrict__ Gh) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* coefs = reinterpret_cast<T*>(smem_raw);  // [kMaxTapCoefs] tap coefficients by degree
  stage_tap_coefs<T, WT>(coefs, hcoef, deg);
  __syncthreads();
  const int Lz = Nz / 2;
  const int Lh = Lz + 1;
  const int ncol_total = Nx * Ny;
  const int col0 = blockIdx.x * cols_per_group;
  const int ncol = min(cols_per_group, ncol_total - col0);
  cx<T>* s_z = reinterpret_cast<cx<T>*>(coefs + kMaxTapCoefs);      // [ncol][Lz]
  T* s_w = reinterpret_cast<T*>(s_z + cols_per_group * Lz);          // [ncol][Lz][wt]
  int* s_base = reinterpret_cast<int*>(s_w + cols_per_group * Lz * wt);  // [ncol][Lz]
  int* s_first = s_base + cols_per_group * Lz;  // [ncol][nb] first contributing l per bin (when first_table)
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int q = tid; q < ncol * Lz; q += nthr) {
    const int ci = q / Lz;
    const int l = q - ci * Lz;
    const int col = col0 + ci;
    const int jj = col / Ny, kk = col - (col / Ny) * Ny;
    const int j = jj < Nx / 2 ? jj : jj - Nx;
    const int k = kk < Ny / 2 ? kk : kk - Ny;
    const double Kx = j * kxu, Ky = k * kyu, Kz = l * kzu;
    double rK;
    const double Kabs = lattice_kabs(Kx, Ky, Kz, rK);
    const TapPoint tp = tap_point<T>(Kabs, s_per_k, n0_over_nt, wt, b_lo, nb);
    const T y = T(tp.y);
    {
      T v[WT];
      tap_weights<T, WT>(coefs, deg, y, v);
#pragma unroll
      for (int t = 0; t < WT; ++t) s_w[q * WT + t] = v[t];
    }
    s_base[q] = tp.base;
    cx<T> z{T(0), T(0)};
    if (jj != Nx / 2 && kk != Ny / 2) {
      const cx<T> a = Dh[(size_t)col * Lh + l];
      const cx<T> b = Dh[((size_t)((Nx - jj) % Nx) * Ny + (Ny - kk) % Ny) * Lh + l];
      cx<T> u{a.x + b.x, a.y - b.y};
      if (deriv == 1) u = cx<T>{T(-Kx) * u.y, T(Kx) * u.x};
      if (deriv == 2) u = cx<T>{T(-Ky) * u.y, T(Ky) * u.x};
      const double sc = (l == 0 ? 1.0 : 2.0) * scale;
      z = cmul(u, cx<T>{T(tp.cs * sc), T(-tp.sn * sc)});
    }
    s_z[q] = z;
  }
  __syncthreads();
  if (first_table) {
    // the bases are non-decreasing in l, so the first l whose taps reach bin
    // b (base_l + wt - 1 >= b) is l for the bins in
    // (base_{l-1} + wt - 1, base_l + wt - 1]; bins below base_0 or past
    // base_{Lz-1} + wt - 1 get no contribution and are not tabulated
    for (int q = tid; q < ncol * Lz; q += nthr) {
      const int ci = q / Lz;
      const int l = q - ci * Lz;
      const int* base = s_base + ci * Lz;
      const int b0 = l == 0 ? base[0] : base[l - 1] + wt;
      const int b1 = min(nb - 1, base[l] + wt - 1);
      for (int b = b0; b <= b1; ++b) s_first[ci * nb + b] = l;
    }
    __syncthreads();
  }
  // bins written per column: the x-mode's range (the transposed y-FFT skips
  // the rest, which get no contribution), else the whole band
  __shared__ int s_run[2 * 8];
  if (tid < ncol) {
    int lo = 0, hi = nb - 1;
    if (jrange) {
      const int jj = (col0 + tid) / Ny;
      lo = jrange[2 * jj];
      hi = jrange[2 * jj + 1];
    }
    s_run[2 * tid] = lo;
    s_run[2 * tid + 1] = hi >= lo ? hi - lo + 1 : 0;
  }
  __syncthreads();
  int total = 0;
  for (int ci = 0; ci < ncol; ++ci) total += s_run[2 * ci + 1];
  for (int q = tid; q < total; q += nthr) {
    int ci = 0, rq = q;
    while (rq >= s_run[2 * ci + 1]) {
      rq -= s_run[2 * ci + 1];
      ++ci;
    }
    const int b = s_run[2 * ci] + rq;
    const int* base = s_base + ci * Lz;
    // contributions come from the l with base_l in [b - wt + 1, b]
    int lo = 0, hi = Lz;
    if (first_table) {
      lo = b < base[0] || b > base[Lz - 1] + wt - 1 ? Lz : s_first[ci * nb + b];
    } else {
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (base[mid] < b - wt + 1) lo = mid + 1; else hi = mid;
      }
    }
    cx<T> acc{T(0), T(0)};
    for (int l = lo; l < Lz && base[l] <= b; ++l) {
      const T v = s_w[(ci * Lz + l) * wt + (b - base[l])];
      const cx<T> z = s_z[ci * Lz + l];
      acc.x += v * z.x;
      acc.y += v * z.y;
    }
    Gh[(size_t)(col0 + ci) * nb + b] = acc;
  }
}

// lateral columns per work-group: enough (l) rows to occupy 256 threads
template <typename T>
static int scatter_cols(const DevPlan& p) {
  const int Lz = p.Nz / 2;
  int c = 256 / Lz;
  return c < 1 ? 1 : (c > 8 ? 8 : c);
}

// per-bin table of first contributions in LDS when it takes at most 16 KiB
// (else a binary search over the bases per bin)
template <typename T>
static bool scatter_first_table(const DevPlan& p) {
  return size_t(scatter_cols<T>(p)) * p.nb * sizeof(int) <= 16384;
}

template <typename T>
size_t scatter_lds_bytes(const DevPlan& p) {
  const size_t Lz = size_t(p.Nz / 2) * scatter_cols<T>(p);
  const size_t first = scatter_first_table<T>(p) ? size_t(scatter_cols<T>(p)) * p.nb * sizeof(int) : 0;
  return kMaxTapCoefs * sizeof(T) + Lz * sizeof(cx<T>) + Lz * p.w_t * sizeof(T) + Lz * sizeof(int) + first;
}

template <typename T>
hipError_t launch_scatter(const DevPlan& p, const void* Dh, void* Gh, int deriv, hipStream_t s) {
  if (deriv < 0 || deriv > 2) return hipErrorInvalidValue;
  const size_t lds = scatter_lds_bytes<T>(p);
  if (p.w_t * (p.hdeg + 1) > kMaxTapCoefs) return hipErrorInvalidValue;
  return wt_pick(p.w_t, [&](auto c) {
  constexpr int WT = decltype(c)::value;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_scatter<T, WT>), lds);
  if (e != hipSuccess) return e;
  const int cpg = scatter_cols<T>(p);
  const int ncol = p.Nx * p.Ny;
  hipLaunchKernelGGL((k_scatter<T, WT>), dim3((unsigned)((ncol + cpg - 1) / cpg)), dim3(256), lds, s,
                     static_cast<const cx<T>*>(Dh), p.nb, p.b_lo, p.Nx, p.Ny, p.Nz, p.s_per_k, p.kxu, p.kyu, p.kzu,
                     p.n0_over_nt, p.adj_scale, deriv, p.w_t, p.hdeg, static_cast<const T*>(p.hcoef), cpg,
                     scatter_first_table<T>(p) ? 1 : 0, p.jrange, static_cast<cx<T>*>(Gh));
  return hipGetLastError();
  });
}

// Batched form of the reconstruction's interpolation (image-ready spectrum)
// fused with the inverse transform along x, each work item as in the
// single-problem launch (same arithmetic; the runtime-planned transform, as
// the problems' lengths differ). Each problem runs with its own tap count at
// compile time when it is one of kBatchTaps (else the runtime-tap form); a
// work-group restages the tap coefficients in LDS when its next work item
// belongs to another problem.
template <typename T, int WT>
__device__ __forceinline__ void gather_batch_item(const GatherBA& a, T* coefs, int& staged, int p, int local) {
  if constexpr (WT > 0) {
    if (p != staged) {  // visible after the body's first barrier
      stage_tap_coefs<T, WT>(coefs, static_cast<const T*>(a.hcoef), a.deg);
      staged = p;
    }
  }
  const int kk = local / a.gx;
  gather_x_body<T, MODE_IMAGE, WT, 0>(static_cast<const cx<T>*>(a.Gh), a.nb, a.b_lo, a.Nx, a.Ny, a.Nz, a.s_per_k,
                                      a.kxu, a.kyu, a.kzu, a.two_c, a.n0_over_nt, a.scale, a.wt, a.deg,
                                      static_cast<const T*>(a.hcoef), a.lchunk, view_desc<T>(a.fd), 0,
                                      static_cast<cx<T>*>(a.Fh), local - kk * a.gx, kk, coefs);
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_gather_batch(const GatherBA* __restrict__ args,
                                                            const int* __restrict__ prefix, int nprob, int total,
                                                            BatchIO io) {
  __shared__ BatchMeta<GatherBA> meta;
  __shared__ T coefs[kMaxTapCoefs];
  batch_meta_load(meta, args, prefix, nprob);
  int staged = -1;
  for (int slot = blockIdx.x; slot < total; slot += gridDim.x) {
    const int w = batch_item(slot, total);
    const int p = __builtin_amdgcn_readfirstlane(batch_locate(meta.prefix, nprob, w));
    const GatherBA a = batch_args(meta, p);
    const int local = w - meta.prefix[p];
    static_assert(kBatchTaps[0] == 6 && kBatchTaps[1] == 8 && kBatchTaps[2] == 10 && kBatchTaps[3] == 12,
                  "tap instantiations");
    switch (a.wt_ct) {
      case 6: gather_batch_item<T, 6>(a, coefs, staged, p, local); break;
      case 8: gather_batch_item<T, 8>(a, coefs, staged, p, local); break;
      case 10: gather_batch_item<T, 10>(a, coefs, staged, p, local); break;
      case 12: gather_batch_item<T, 12>(a, coefs, staged, p, local); break;
      default: gather_batch_item<T, 0>(a, coefs, staged, p, local); break;
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_gather_batch(const BatchStage& st, const BatchIO& io, hipStream_t s) {
  if (st.total <= 0) return hipSuccess;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_gather_batch<T>), st.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gather_batch<T>), dim3(batch_grid(st)), dim3(256), st.lds, s,
                     static_cast<const GatherBA*>(st.args), st.prefix, st.nprob, st.total, io);
  return hipGetLastError();
}

#define PATK_INST(T)                                                                     \
  template hipError_t launch_gather<T>(const DevPlan&, const void*, void*, int, hipStream_t); \
  template hipError_t launch_gather_x<T>(const DevPlan&, const void*, void*, int, hipStream_t); \
  template size_t scatter_lds_bytes<T>(const DevPlan&);                                  \
  template hipError_t launch_scatter<T>(const DevPlan&, const void*, void*, int, hipStream_t); \
  template hipError_t launch_gather_batch<T>(const BatchStage&, const BatchIO&, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
