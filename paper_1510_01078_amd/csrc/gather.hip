// Temporal interpolation at omega(K) with the inversion weight
// (Section 3.1, eq. NER_NUFFT; Section 2, eq. exact).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

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

#define PATK_INST(T) template hipError_t launch_gather<T>(const DevPlan&, const void*, void*, bool, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
