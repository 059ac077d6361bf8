// Host side of the C ABI: descriptor validation, the plan's precomputed
// tables (Section 5.2: window values precomputed for a fixed discretisation),
// workspace layout and the enqueueing of the stage kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "kernels.hpp"
#include "kernels_common.hpp"
#include "pat_nufft.h"
#include "plan_internal.hpp"
#include "plan_sizes.hpp"
#include "window.hpp"

using namespace patint;

namespace {


using patsz::next_smooth_even;

// exact-division multiplier for x < 2^16, d < 2^16 (0 encodes d == 1)
inline uint32_t div_magic(int d) { return d == 1 ? 0u : uint32_t((uint64_t(1) << 32) / uint64_t(d) + 1); }

bool radix_plan(int n, patk::FftRaw& f) {
  f.n = n;
  f.npass = 0;
  int radix[24], np = 0, r = n;
  for (int R : {8, 6, 4, 2, 5, 3})  // radix 6 after the 8s: 384 = 8 8 6, 288 = 8 6 6 (one pass fewer)
    while (r % R == 0 && np < 24) {
      radix[np++] = R;
      r /= R;
    }
  if (r != 1 || np > 12 || n >= 65536) return false;
  int p = 1;
  for (int i = 0; i < np; ++i) {
    patk::FftPassRaw& ps = f.pass[i];
    ps.R = radix[i];
    ps.p = p;
    ps.nbf = n / radix[i];
    ps.twstep = n / (p * radix[i]);
    ps.m_nbf = div_magic(ps.nbf);
    ps.m_p = div_magic(p);
    p *= radix[i];
  }
  f.npass = np;
  return true;
}

struct HostBlob {
  std::vector<unsigned char> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = align_up(bytes.size());
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
};

template <typename T>
size_t add_real(HostBlob& b, const std::vector<double>& v) {
  std::vector<T> t(v.begin(), v.end());
  return b.add(t.data(), t.size() * sizeof(T));
}

template <typename T>
size_t add_twiddles(HostBlob& b, int n) {
  std::vector<T> t(2 * size_t(n));
  for (int i = 0; i < n; ++i) {
    const double a = -2.0 * M_PI * double(i) / double(n);
    t[2 * i] = T(std::cos(a));
    t[2 * i + 1] = T(std::sin(a));
  }
  return b.add(t.data(), t.size() * sizeof(T));
}

}  // namespace


namespace {

pat_status validate(const pat_plan_desc* d) {
  if (!d) return PAT_ERR_INVALID_ARGUMENT;
  if (d->n_sensors < 1 || d->n_t < 2) return PAT_ERR_INVALID_ARGUMENT;
  if (!(d->dt > 0.0) || !std::isfinite(d->dt) || !(d->c > 0.0) || !std::isfinite(d->c)) return PAT_ERR_INVALID_ARGUMENT;
  if (!d->sensor_xy) return PAT_ERR_INVALID_ARGUMENT;
  for (int32_t n : {d->nx, d->ny, d->nz})
    if (n < 4 || (n % 2) != 0) return PAT_ERR_INVALID_ARGUMENT;
  for (double L : {d->lx, d->ly, d->lz})
    if (!(L > 0.0) || !std::isfinite(L)) return PAT_ERR_INVALID_ARGUMENT;
  if (d->temporal_interp != PAT_INTERP_WINDOW && d->temporal_interp != PAT_INTERP_LINEAR)
    return PAT_ERR_INVALID_ARGUMENT;
  const double sigma_t_min = d->temporal_interp == PAT_INTERP_LINEAR ? 1.0 : 1.1;
  if (!(d->sigma_xy >= 1.1 && d->sigma_xy <= 4.0) || !(d->sigma_t >= sigma_t_min && d->sigma_t <= 4.0))
    return PAT_ERR_INVALID_ARGUMENT;
  if (d->width_xy < 2 || d->width_xy > 16 || (d->width_xy % 2) || d->width_t < 2 || d->width_t > 16 ||
      (d->width_t % 2))
    return d->width_xy > 16 || d->width_t > 16 ? PAT_ERR_UNSUPPORTED : PAT_ERR_INVALID_ARGUMENT;
  if (d->kernel != PAT_KERNEL_GAUSSIAN && d->kernel != PAT_KERNEL_KAISER_BESSEL) return PAT_ERR_INVALID_ARGUMENT;
  if (d->precision != PAT_FP64 && d->precision != PAT_FP32 && d->precision != PAT_FP32_KAHAN)
    return PAT_ERR_INVALID_ARGUMENT;
  if ((d->alloc == nullptr) != (d->free == nullptr)) return PAT_ERR_INVALID_ARGUMENT;
  const double hx = 0.5 * d->lx, hy = 0.5 * d->ly;
  for (int32_t m = 0; m < d->n_sensors; ++m) {
    const double x = d->sensor_xy[2 * m], y = d->sensor_xy[2 * m + 1];
    if (!(x >= -hx && x < hx && y >= -hy && y < hy)) return PAT_ERR_INVALID_ARGUMENT;
    if (d->sensor_h && !(d->sensor_h[m] > 0.0 && std::isfinite(d->sensor_h[m]))) return PAT_ERR_INVALID_ARGUMENT;
  }
  return PAT_OK;
}



template <typename T>
pat_status build_tables(pat_plan* P, hipStream_t stream) {
  const pat_plan_desc& d = P->d;
  patk::DevPlan& dp = P->dp;
  const int M = d.n_sensors, Nt = d.n_t;
  dp.M = M;
  dp.Nt = Nt;
  dp.Nx = d.nx;
  dp.Ny = d.ny;
  dp.Nz = d.nz;
  // an oversampled lateral axis holds at least one window footprint, so a
  // footprint meets every grid point at most once (short axes get a larger
  // effective oversampling; the deconvolution uses the actual length)
  dp.n_x = next_smooth_even(std::max(d.sigma_xy * d.nx, double(d.width_xy)));
  dp.n_y = next_smooth_even(std::max(d.sigma_xy * d.ny, double(d.width_xy)));
  const bool linear_t = d.temporal_interp == PAT_INTERP_LINEAR;
  // band of oversampled temporal bins the interpolation reads: |K| from 0 (the
  // l = 0 plane, read by the forward model and the adjoint) to the largest
  // non-Nyquist lattice point, w_t/2 bins of margin below and w_t/2 + 1
  // above, rounded up to an even count (plan_sizes.hpp)
  {
    const int wt_taps = linear_t ? 2 : d.width_t;
    const double Kx = (d.nx / 2 - 1) * 2.0 * M_PI / d.lx, Ky = (d.ny / 2 - 1) * 2.0 * M_PI / d.ly;
    const double Kz = (d.nz / 2 - 1) * 2.0 * M_PI / d.lz;
    const double kmax = std::sqrt(Kx * Kx + Ky * Ky + Kz * Kz);
    const patsz::Band band = patsz::temporal_band(d.sigma_t, Nt, wt_taps, kmax, d.c, d.dt);
    if (!band.ok) return PAT_ERR_UNSUPPORTED;  // |omega| dt near or past pi
    dp.n_t = band.n_t;
    dp.b_lo = band.b_lo;
    dp.nb = band.nb;
  }
  // the spread stages each sensor's band row with 16-byte loads: rows must
  // start on 16-byte boundaries (the workspace regions are 256-byte aligned)
  if ((size_t(dp.nb) * 2 * sizeof(T)) % 16 != 0) return PAT_ERR_UNSUPPORTED;
  // window form: samples centred on n0 = Nt/2; linear baseline: zeros appended
  // after the trace (time origin 0) and two taps
  dp.n0 = linear_t ? 0 : Nt / 2;
  dp.w_xy = d.width_xy;
  dp.w_t = linear_t ? 2 : d.width_t;
  dp.kahan = d.precision == PAT_FP32_KAHAN;
  const size_t cxb = 2 * sizeof(T);
  // FFT lengths the LDS kernels handle: one padded sequence per work-group must fit the device's LDS
  int lds_limit = 65536;
  if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) != hipSuccess) {
    (void)hipGetLastError();
    return PAT_ERR_HIP;
  }
  auto seq_bytes = [&](int n) { return size_t(patk::lseq(n)) * cxb; };
  if (seq_bytes(dp.n_t) > (size_t)lds_limit || seq_bytes(dp.n_x) > (size_t)lds_limit ||
      seq_bytes(dp.n_y) > (size_t)lds_limit || seq_bytes(d.nx) > (size_t)lds_limit ||
      seq_bytes(d.ny) > (size_t)lds_limit || seq_bytes(d.nz) > (size_t)lds_limit)
    return PAT_ERR_UNSUPPORTED;
  if (dp.n_t > 8192) return PAT_ERR_UNSUPPORTED;  // temporal kernel: 512 threads x 16 values
  if (dp.n_x > 4096 || dp.n_y > 4096 || d.nx > 2048 || d.ny > 2048 || d.nz > 2048) return PAT_ERR_UNSUPPORTED;
  if (!radix_plan(dp.n_t, dp.f_nt) || !radix_plan(dp.n_x, dp.f_nx) || !radix_plan(dp.n_y, dp.f_ny) ||
      !radix_plan(d.nx, dp.f_Nx) || !radix_plan(d.ny, dp.f_Ny) || !radix_plan(d.nz, dp.f_Nz))
    return PAT_ERR_UNSUPPORTED;

  dp.kxu = 2.0 * M_PI / d.lx;
  dp.kyu = 2.0 * M_PI / d.ly;
  dp.kzu = 2.0 * M_PI / d.lz;
  dp.two_c = 2.0 * d.c;
  dp.s_per_k = d.c * d.dt * dp.n_t / (2.0 * M_PI);
  dp.n0_over_nt = double(dp.n0) / double(dp.n_t);
  dp.inv_vol = 1.0 / (d.lx * d.ly * d.lz);
  dp.adj_scale = 0.5 / (double(d.nx) * d.ny * d.nz);

  const pathost::Window wxy(d.kernel == PAT_KERNEL_KAISER_BESSEL ? 1 : 0, d.width_xy, d.sigma_xy);
  const pathost::Window wt(d.kernel == PAT_KERNEL_KAISER_BESSEL ? 1 : 0, d.width_t, double(dp.n_t) / Nt);

  HostBlob blob;
  // per-sensor scalar weight h_m * dt
  std::vector<double> hw(M);
  for (int m = 0; m < M; ++m) hw[m] = (d.sensor_h ? d.sensor_h[m] : d.lx * d.ly / M) * d.dt;
  const size_t o_hw = add_real<T>(blob, hw);
  // temporal deapodisation 1/phihat_t((n - n0)/n_t) (none for the linear baseline)
  std::vector<double> deap(Nt);
  for (int n = 0; n < Nt; ++n) deap[n] = linear_t ? 1.0 : 1.0 / wt.phihat(double(n - dp.n0) / dp.n_t);
  const size_t o_deap = add_real<T>(blob, deap);
  // sensor footprints and weights on the oversampled lateral grid
  const int w = dp.w_xy;
  std::vector<int> sbx(M), sby(M);
  std::vector<double> swx(size_t(M) * w), swy(size_t(M) * w);
  for (int m = 0; m < M; ++m) {
    const double ux = (d.sensor_xy[2 * m] + 0.5 * d.lx) * dp.n_x / d.lx;
    const double uy = (d.sensor_xy[2 * m + 1] + 0.5 * d.ly) * dp.n_y / d.ly;
    const long fx = (long)std::floor(ux), fy = (long)std::floor(uy);
    const long bx = fx - w / 2 + 1, by = fy - w / 2 + 1;
    for (int t = 0; t < w; ++t) {
      swx[size_t(m) * w + t] = wxy.phi(ux - double(bx + t));
      swy[size_t(m) * w + t] = wxy.phi(uy - double(by + t));
    }
    sbx[m] = (int)(((bx % dp.n_x) + dp.n_x) % dp.n_x);
    sby[m] = (int)(((by % dp.n_y) + dp.n_y) % dp.n_y);
  }
  const size_t o_sbx = blob.add(sbx.data(), sbx.size() * sizeof(int));
  const size_t o_sby = blob.add(sby.data(), sby.size() * sizeof(int));
  const size_t o_swx = add_real<T>(blob, swx);
  const size_t o_swy = add_real<T>(blob, swy);
  // 16 x 16 tiles of the oversampled grid (the forward model's home lists)
  const int TS = patk::kSpreadTile;
  dp.tiles_x = (dp.n_x + TS - 1) / TS;
  dp.tiles_y = (dp.n_y + TS - 1) / TS;
  const int ntiles = dp.tiles_x * dp.tiles_y;
  // wave-patch lists: sensors whose footprint meets each 16 x kPatchRows patch
  // (a tile column and a group of rows), ascending per patch
  const int PR = patk::kPatchRows;
  dp.patches_y = (dp.n_y + PR - 1) / PR;
  const int npatch = dp.tiles_x * dp.patches_y;
  std::vector<int> pcnt(npatch + 1, 0);
  std::vector<std::pair<int, int>> pinc;
  pinc.reserve(size_t(M) * 6);
  for (int m = 0; m < M; ++m) {
    int txs[4], rgs[8], ntx = 0, nrg = 0;
    for (int t = 0; t < w; ++t) {
      const int tx = ((sbx[m] + t) % dp.n_x) / TS;
      if (ntx < 4 && std::find(txs, txs + ntx, tx) == txs + ntx) txs[ntx++] = tx;
      const int rg = ((sby[m] + t) % dp.n_y) / PR;
      if (nrg < 8 && std::find(rgs, rgs + nrg, rg) == rgs + nrg) rgs[nrg++] = rg;
    }
    for (int a = 0; a < ntx; ++a)
      for (int b = 0; b < nrg; ++b) pinc.emplace_back(rgs[b] * dp.tiles_x + txs[a], m);
  }
  P->spread_pairs = (int64_t)pinc.size();
  for (auto& e : pinc) pcnt[e.first + 1]++;
  for (int i = 0; i < npatch; ++i) pcnt[i + 1] += pcnt[i];
  std::vector<int> psens(pinc.size());
  {
    std::vector<int> pos(pcnt.begin(), pcnt.end() - 1);
    for (auto& e : pinc) psens[pos[e.first]++] = e.second;  // stable: sensors ascending per patch
  }
  // packed slots of each patch: the patch's sensors (in list order) placed
  // first-fit into slots of up to kSlotK sensors whose footprints share no
  // grid point of the patch, with every lane's weight wx*wy and the index of
  // the slot's sensor that covers it (weight 0 and index 0 where none does)
  constexpr int SK = patk::kSlotK;
  std::vector<int> soff(npatch + 1, 0), ssens;
  std::vector<double> sw;
  std::vector<unsigned char> sk;
  for (int pt = 0; pt < npatch; ++pt) {
    const int px0 = (pt % dp.tiles_x) * TS, py0 = (pt / dp.tiles_x) * PR;
    const size_t first = ssens.size() / SK;
    std::vector<uint64_t> used;
    std::vector<int> fill;
    for (int q = pcnt[pt]; q < pcnt[pt + 1]; ++q) {
      const int m = psens[q];
      uint64_t mask = 0;
      for (int lane = 0; lane < 64; ++lane) {
        const int px = px0 + (lane & 15), py = py0 + (lane >> 4);
        if (px >= dp.n_x || py >= dp.n_y) continue;
        const int tx = ((px - sbx[m]) % dp.n_x + dp.n_x) % dp.n_x;
        const int ty = ((py - sby[m]) % dp.n_y + dp.n_y) % dp.n_y;
        if (tx < w && ty < w) mask |= uint64_t(1) << lane;
      }
      if (!mask) continue;
      size_t sl = 0;
      while (sl < used.size() && (fill[sl] == SK || (used[sl] & mask))) ++sl;
      if (sl == used.size()) {
        used.push_back(0);
        fill.push_back(0);
        ssens.insert(ssens.end(), SK, -1);
        sw.insert(sw.end(), 64, 0.0);
        sk.insert(sk.end(), 64, 0);
      }
      const size_t gs = first + sl;
      const int k = fill[sl]++;
      used[sl] |= mask;
      ssens[gs * SK + k] = m;
      for (int lane = 0; lane < 64; ++lane) {
        if (!((mask >> lane) & 1)) continue;
        const int tx = ((px0 + (lane & 15) - sbx[m]) % dp.n_x + dp.n_x) % dp.n_x;
        const int ty = ((py0 + (lane >> 4) - sby[m]) % dp.n_y + dp.n_y) % dp.n_y;
        sw[gs * 64 + lane] = swx[size_t(m) * w + tx] * swy[size_t(m) * w + ty];
        sk[gs * 64 + lane] = (unsigned char)k;
      }
    }
    soff[pt + 1] = int(ssens.size() / SK);
  }
  // per slot and lane, the places of the kSlotBatch slots from it on within
  // its patch, two bits each: a round reads one word per lane
  std::vector<unsigned> sk16(sk.size(), 0);
  for (int pt = 0; pt < npatch; ++pt)
    for (int q = soff[pt]; q < soff[pt + 1]; ++q)
      for (int lane = 0; lane < 64; ++lane) {
        unsigned v = 0;
        for (int i = 0; i < patk::kSlotBatch && q + i < soff[pt + 1]; ++i)
          v |= unsigned(sk[size_t(q + i) * 64 + lane]) << (2 * i);
        sk16[size_t(q) * 64 + lane] = v;
      }
  P->spread_slots = (int64_t)(ssens.size() / SK);
  const size_t o_soff = blob.add(soff.data(), soff.size() * sizeof(int));
  const size_t o_ssens = blob.add(ssens.data(), std::max<size_t>(1, ssens.size()) * sizeof(int));
  const size_t o_sw = add_real<T>(blob, sw.empty() ? std::vector<double>(1, 0.0) : sw);
  const size_t o_sk = blob.add(sk16.data(), std::max<size_t>(1, sk16.size()) * sizeof(unsigned));
  // home lists for the interpolation to the sensors: each sensor once, in
  // the tile holding its footprint origin, sensors ascending per tile
  std::vector<int> hcnt(ntiles + 1, 0), home(M);
  for (int m = 0; m < M; ++m) hcnt[(sby[m] / TS) * dp.tiles_x + sbx[m] / TS + 1]++;
  for (int i = 0; i < ntiles; ++i) hcnt[i + 1] += hcnt[i];
  {
    std::vector<int> pos(hcnt.begin(), hcnt.end() - 1);
    for (int m = 0; m < M; ++m) home[pos[(sby[m] / TS) * dp.tiles_x + sbx[m] / TS]++] = m;
  }
  const size_t o_hoff = blob.add(hcnt.data(), hcnt.size() * sizeof(int));
  const size_t o_hsens = blob.add(home.data(), home.size() * sizeof(int));
  // lateral deconvolution 1/phihat(j/n), zero on the Nyquist mode j = -N/2
  std::vector<double> dcx(d.nx), dcy(d.ny);
  for (int jj = 0; jj < d.nx; ++jj) {
    const int j = jj < d.nx / 2 ? jj : jj - d.nx;
    dcx[jj] = (jj == d.nx / 2) ? 0.0 : 1.0 / wxy.phihat(double(j) / dp.n_x);
  }
  for (int kk = 0; kk < d.ny; ++kk) {
    const int k = kk < d.ny / 2 ? kk : kk - d.ny;
    dcy[kk] = (kk == d.ny / 2) ? 0.0 : 1.0 / wxy.phihat(double(k) / dp.n_y);
  }
  const size_t o_dcx = add_real<T>(blob, dcx);
  const size_t o_dcy = add_real<T>(blob, dcy);
  // dynamic range of the deconvolutions (largest over smallest 1/phihat over
  // the kept modes): FP32 rounding in the grid and the band is amplified by
  // it, so FP32 plans beyond 1e4 (sigma near 1 with wide windows) are refused
  {
    auto range = [](const std::vector<double>& v) {
      double lo = 0.0, hi = 0.0;
      for (double a : v) {
        a = std::fabs(a);
        if (a == 0.0) continue;
        lo = lo == 0.0 ? a : std::min(lo, a);
        hi = std::max(hi, a);
      }
      return lo > 0.0 ? hi / lo : 1.0;
    };
    P->range_xy = range(dcx) * range(dcy);
    P->range_t = range(deap);
    if (sizeof(T) == 4 && (P->range_xy > 1e4 || P->range_t > 1e4)) return PAT_ERR_UNSUPPORTED;
  }
  // temporal tap polynomials: FP64 plans fit them to 1e-13 of the window's
  // peak, FP32 plans to 2e-8 (a third of FP32's unit roundoff; each degree
  // fewer is one multiply-add per tap and interpolation point)
  std::vector<double> coef;
  const double tol = sizeof(T) == 8 ? 1e-13 : 2e-8;
  int deg = 6;
  for (; deg <= 24; ++deg)
    if (pathost::fit_tap_polynomials(wt, deg, coef) <= tol) break;
  if (deg > 24) deg = 24;
  if (linear_t) {
    // linear interpolation between bins floor(s) and floor(s)+1 with
    // weights 1 - frac and frac; in y = 2 frac - 1 these are (1 -+ y)/2
    deg = 1;
    coef = {0.5, -0.5, 0.5, 0.5};
  }
  dp.hdeg = deg;
  const size_t o_hc = add_real<T>(blob, coef);
  // per x-mode range of band bins the interpolation reads (reconstruction,
  // adjoint, spectrum): modes (j, k, l) with |k| <= Ny/2, l <= Nz/2 read bins
  // base(s) .. base(s) + w_t - 1 with s = |K| s_per_k non-decreasing in |k| and
  // l, so x-mode j needs base(s(j,0,0)) .. base(s(j,Ny/2,Nz/2)) + w_t - 1; one
  // bin of margin on each side (host and device may round |K| apart), widened
  // to whole groups of the y-FFT's bins. The compile-time x-FFT writes and
  // the y-FFT transforms only these (x mode, bin) pairs.
  std::vector<int> jr(2 * size_t(d.nx));
  {
    const int ybins = patk::fft_batch<T>(dp.n_y, patk::kFftThreads, patk::kFftCap);
    const int wt = dp.w_t;
    auto base = [&](double sv) {
      long b = (long)std::floor(sv) - wt / 2 + 1 - dp.b_lo;
      return (int)std::min<long>(std::max<long>(b, 0), dp.nb - wt);
    };
    const double Ky = (d.ny / 2) * dp.kyu, Kz = (d.nz / 2) * dp.kzu;
    for (int jj = 0; jj < d.nx; ++jj) {
      const int j = jj < d.nx / 2 ? jj : jj - d.nx;
      const double Kx = j * dp.kxu;
      int lo = std::max(0, base(std::fabs(Kx) * dp.s_per_k) - 1);
      int hi = std::min(dp.nb - 1, base(std::sqrt(Kx * Kx + Ky * Ky + Kz * Kz) * dp.s_per_k) + wt);
      lo = lo / ybins * ybins;
      hi = std::min(dp.nb - 1, hi / ybins * ybins + ybins - 1);
      jr[2 * jj] = lo;
      jr[2 * jj + 1] = hi;
    }
  }
  P->band_pairs = 0;
  for (int jj = 0; jj < d.nx; ++jj) P->band_pairs += jr[2 * jj + 1] - jr[2 * jj] + 1;
  const size_t o_jr = blob.add(jr.data(), jr.size() * sizeof(int));
  // the y-FFT's (x mode, bin group) work items inside the ranges, x-mode
  // major: its grid holds these only (no work-groups that would return at once)
  std::vector<int> yl;
  {
    const int ybins = patk::fft_batch<T>(dp.n_y, patk::kFftThreads, patk::kFftCap);
    for (int jj = 0; jj < d.nx; ++jj)
      for (int b = jr[2 * jj]; b <= jr[2 * jj + 1]; b += ybins) yl.push_back(jj << 16 | (b / ybins));
  }
  const size_t o_yl = blob.add(yl.data(), std::max<size_t>(1, yl.size()) * sizeof(int));
  // the same ranges per bin: both ends are non-decreasing in |j|, so the
  // x-modes that hold bin b are J0(b) <= |j| <= J1(b) (J0 > J1: none)
  std::vector<int> br(2 * size_t(dp.nb));
  {
    const int half = d.nx / 2;
    for (int b = 0; b < dp.nb; ++b) {
      int j0 = half + 1, j1 = -1;
      for (int aj = 0; aj <= half; ++aj) {
        const int jj = aj < half ? aj : half;  // |j| = Nx/2 is the mode jj = Nx/2
        if (jr[2 * jj] <= b && b <= jr[2 * jj + 1]) {
          j0 = std::min(j0, aj);
          j1 = std::max(j1, aj);
        }
      }
      br[2 * b] = j0;
      br[2 * b + 1] = j1;
    }
  }
  const size_t o_br = blob.add(br.data(), br.size() * sizeof(int));
  // twiddles
  const size_t o_tw_nt = add_twiddles<T>(blob, dp.n_t);
  const size_t o_tw_nx = add_twiddles<T>(blob, dp.n_x);
  const size_t o_tw_ny = add_twiddles<T>(blob, dp.n_y);
  const size_t o_tw_Nx = add_twiddles<T>(blob, d.nx);
  const size_t o_tw_Ny = add_twiddles<T>(blob, d.ny);
  const size_t o_tw_Nz = add_twiddles<T>(blob, d.nz);
  patk::FftRaw* ffts[6] = {&dp.f_nt, &dp.f_nx, &dp.f_ny, &dp.f_Nx, &dp.f_Ny, &dp.f_Nz};
  size_t o_pass[6];
  for (int i = 0; i < 6; ++i) o_pass[i] = blob.add(ffts[i]->pass, sizeof(patk::FftPassRaw) * ffts[i]->npass);

  P->dev_bytes = align_up(blob.bytes.size());
  P->dev = dev_alloc(d, P->dev_bytes);
  if (!P->dev) return PAT_ERR_ALLOC;
  if (hipMemcpyAsync(P->dev, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    (void)hipGetLastError();
    return PAT_ERR_HIP;
  }
  auto at = [&](size_t off) { return static_cast<const void*>(static_cast<unsigned char*>(P->dev) + off); };
  dp.hw = at(o_hw);
  dp.deap = at(o_deap);
  dp.sbx = static_cast<const int*>(at(o_sbx));
  dp.sby = static_cast<const int*>(at(o_sby));
  dp.swx = at(o_swx);
  dp.swy = at(o_swy);
  dp.slot_off = static_cast<const int*>(at(o_soff));
  dp.slot_sens = static_cast<const int*>(at(o_ssens));
  dp.slot_w = at(o_sw);
  dp.slot_k = static_cast<const unsigned*>(at(o_sk));
  dp.home_off = static_cast<const int*>(at(o_hoff));
  dp.home_sens = static_cast<const int*>(at(o_hsens));
  dp.dcx = at(o_dcx);
  dp.dcy = at(o_dcy);
  dp.hcoef = at(o_hc);
  dp.jrange = static_cast<const int*>(at(o_jr));
  dp.ylist = static_cast<const int*>(at(o_yl));
  dp.ylist_n = int(yl.size());
  dp.brange = static_cast<const int*>(at(o_br));
  dp.f_nt.tw = at(o_tw_nt);
  dp.f_nx.tw = at(o_tw_nx);
  dp.f_ny.tw = at(o_tw_ny);
  dp.f_Nx.tw = at(o_tw_Nx);
  dp.f_Ny.tw = at(o_tw_Ny);
  dp.f_Nz.tw = at(o_tw_Nz);
  for (int i = 0; i < 6; ++i) ffts[i]->dpass = at(o_pass[i]);

  // Spread and x-FFT can run in rounds of chunk_bins bins through one smaller
  // grid buffer (a multiple of the spread's 16-bin groups). One round is the
  // default: on MI355X, rounds sized for the last-level cache measured slower
  // (each round adds the spread's load-imbalance tail). PATNUFFT_CHUNK_BINS
  // sets a round size (0 or >= nb: one round) to trade speed for workspace.
  {
    long cb = 0;
    if (const char* env = std::getenv("PATNUFFT_CHUNK_BINS")) cb = std::atol(env);
    if (cb <= 0 || cb >= dp.nb) cb = dp.nb;
    cb = std::max<long>(16, (cb + 15) / 16 * 16);
    dp.chunk_bins = int(std::min<long>(cb, dp.nb));
  }
  // workspace: region A = grid chunk U, later the lateral spectra Gh;
  // region B = x-transformed rows V, later the spectrum F; region C = Gt.
  const size_t c = cxb;
  const size_t sz_Gt = size_t(M) * dp.nb * c;
  const size_t sz_U = size_t(dp.chunk_bins) * dp.n_y * dp.n_x * c;
  const size_t sz_V = size_t(dp.nb) * d.nx * dp.n_y * c;
  const size_t sz_Gh = size_t(d.nx) * d.ny * dp.nb * c;
  const size_t sz_F = size_t(d.nx) * d.ny * (d.nz / 2 + 1) * c;
  P->forward_ok = patk::scatter_lds_bytes<T>(dp) + patk::kStaticLdsMargin <= (size_t)lds_limit;
  P->forward_fused = patk::fused_interp_ok<T>(dp, (size_t)lds_limit - patk::kStaticLdsMargin);
  // two home-tile rows per fused strip (32 + w - 1 grid rows for 32: less
  // halo recomputation, measured faster) where the work-group LDS holds them
  dp.fused_strip =
      dp.tiles_y >= 2 && patk::fused_interp_lds<T>(dp, 2) + patk::kStaticLdsMargin <= (size_t)lds_limit ? 2 : 1;
  const size_t szA = align_up(std::max(sz_U, sz_Gh));
  const size_t szB = align_up(std::max(sz_V, sz_F));
  P->off_B = szA;
  P->off_C = szA + szB;
  P->ws_bytes = szA + szB + align_up(sz_Gt);
  return PAT_OK;
}



struct Marker {
  pat_plan* P;
  int call;
  int next = 0;
  hipStream_t s;
  // boundary between stage `done` (the work since the previous boundary; -1
  // at the call's start) and stage `after` (-1 at its end): an event is
  // recorded where either is timed, so a timed stage always lies between two
  // consecutive events of the call
  void operator()(int done, int after) {
    if (call < 0 || next >= P->marks_per_call || !(timed(done) || timed(after))) return;
    const size_t i = size_t(call) * P->marks_per_call + next;
    P->ev_stage[i] = done;
    (void)hipEventRecord(P->ev[i], s);
    ++next;
  }
  bool timed(int stage) const { return stage >= 0 && ((P->ev_mask >> stage) & 1u); }
};

inline int rounds(const patk::DevPlan& dp) { return (dp.nb + dp.chunk_bins - 1) / dp.chunk_bins; }

enum Op { OP_RECONSTRUCT, OP_SPECTRUM, OP_ADJOINT, OP_FORWARD, OP_FORWARD_DX, OP_FORWARD_DY };

// Reconstruction, physical spectrum and adjoint: traces in, image (or
// spectrum) out. The adjoint uses unit trace weights and the adjoint gather.
template <typename T>
pat_status run_traces_in(pat_plan* P, const void* g, void* out, void* ws, hipStream_t s, Op op) {
  const patk::DevPlan& dp = P->dp;
  unsigned char* A = static_cast<unsigned char*>(ws);
  unsigned char* B = A + P->off_B;
  unsigned char* C = A + P->off_C;
  Marker mark{P, P->ev_used < P->ev_max ? P->ev_used++ : -1, 0, s};
  hipError_t e;
  mark(-1, 0);
  if ((e = patk::launch_temporal<T>(dp, static_cast<const T*>(g), C, op != OP_ADJOINT, s)) != hipSuccess)
    return to_status(e);
  mark(0, 1);
  for (int b0 = 0; b0 < dp.nb; b0 += dp.chunk_bins) {
    const int b1 = std::min(dp.nb, b0 + dp.chunk_bins);
    if ((e = patk::launch_spread<T>(dp, C, A, b0, b1, s)) != hipSuccess) return to_status(e);
    mark(1, 2);
    if ((e = patk::launch_fft_x<T>(dp, A, B, b0, b1, s)) != hipSuccess) return to_status(e);
    mark(2, b1 < dp.nb ? 1 : 3);
  }
  if ((e = patk::launch_fft_y<T>(dp, B, A, s)) != hipSuccess) return to_status(e);
  mark(3, 4);
  if (op == OP_SPECTRUM) {
    if ((e = patk::launch_gather<T>(dp, A, out, patk::GATHER_PHYSICAL, s)) != hipSuccess) return to_status(e);
    mark(4, -1);
    return PAT_OK;
  }
  // the gather and the inverse transform along x run as one kernel
  const int mode = op == OP_ADJOINT ? patk::GATHER_ADJOINT : patk::GATHER_IMAGE;
  if ((e = patk::launch_gather_x<T>(dp, A, B, mode, s)) != hipSuccess) return to_status(e);
  mark(4, 5);
  if ((e = patk::launch_inverse<T>(dp, B, static_cast<T*>(out), s, true)) != hipSuccess) return to_status(e);
  mark(5, -1);
  return PAT_OK;
}

// Forward model (and its position derivatives): image in, traces out; the
// transposes of the adjoint's stages in reverse order. Timing marks use the
// stage index of the stage each kernel transposes.
template <typename T>
pat_status run_image_in(pat_plan* P, const void* f, void* g, void* ws, hipStream_t s, Op op) {
  // the band ranges prune the forward path only with the fused kernel (the
  // two-kernel form reads every x-mode of every bin)
  patk::DevPlan dp = P->dp;
  if (!P->forward_fused) {
    dp.jrange = nullptr;
    dp.brange = nullptr;
    dp.ylist = nullptr;
    dp.ylist_n = 0;
  }
  unsigned char* A = static_cast<unsigned char*>(ws);
  unsigned char* B = A + P->off_B;
  unsigned char* C = A + P->off_C;
  Marker mark{P, P->ev_used < P->ev_max ? P->ev_used++ : -1, 0, s};
  hipError_t e;
  const int deriv = op == OP_FORWARD_DX ? 1 : (op == OP_FORWARD_DY ? 2 : 0);
  mark(-1, 5);
  if ((e = patk::launch_forward3d<T>(dp, static_cast<const T*>(f), B, s)) != hipSuccess) return to_status(e);
  mark(5, 4);
  if ((e = patk::launch_scatter<T>(dp, B, A, deriv, s)) != hipSuccess) return to_status(e);
  mark(4, 3);
  if ((e = patk::launch_fft_y_t<T>(dp, A, B, s)) != hipSuccess) return to_status(e);
  mark(3, P->forward_fused ? 1 : 2);
  if (P->forward_fused) {
    if ((e = patk::launch_fft_x_interp<T>(dp, B, C, s)) != hipSuccess) return to_status(e);
    mark(1, 0);
  } else {
    for (int b0 = 0; b0 < dp.nb; b0 += dp.chunk_bins) {
      const int b1 = std::min(dp.nb, b0 + dp.chunk_bins);
      if ((e = patk::launch_fft_x_t<T>(dp, B, A, b0, b1, s)) != hipSuccess) return to_status(e);
      mark(2, 1);
      if ((e = patk::launch_interp<T>(dp, A, C, b0, b1, s)) != hipSuccess) return to_status(e);
      mark(1, b1 < dp.nb ? 2 : 0);
    }
  }
  if ((e = patk::launch_temporal_t<T>(dp, C, static_cast<T*>(g), s)) != hipSuccess) return to_status(e);
  mark(0, -1);
  return PAT_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const unsigned char* pa = static_cast<const unsigned char*>(a);
  const unsigned char* pb = static_cast<const unsigned char*>(b);
  return pa < pb + nb && pb < pa + na;
}

pat_status compute(pat_plan* P, const void* in, void* out, void* ws, void* stream, Op op) {
  if (!P || !in || !out || !ws) return PAT_ERR_INVALID_ARGUMENT;
  if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return PAT_ERR_INVALID_ARGUMENT;
  const size_t eb = P->fp64 ? 8 : 4;
  const size_t traces = size_t(P->d.n_sensors) * P->d.n_t * eb;
  const size_t image = size_t(P->d.nx) * P->d.ny * P->d.nz * eb;
  const size_t half = size_t(P->d.nx) * P->d.ny * (P->d.nz / 2 + 1) * 2 * eb;
  const bool image_in = op == OP_FORWARD || op == OP_FORWARD_DX || op == OP_FORWARD_DY;
  const size_t i_bytes = image_in ? image : traces;
  const size_t o_bytes = image_in ? traces : (op == OP_SPECTRUM ? half : image);
  if (overlaps(in, i_bytes, out, o_bytes) || overlaps(in, i_bytes, ws, P->ws_bytes) ||
      overlaps(out, o_bytes, ws, P->ws_bytes))
    return PAT_ERR_INVALID_ARGUMENT;
  if (image_in && !P->forward_ok) return PAT_ERR_UNSUPPORTED;
  DeviceGuard guard(P->device);
  if (!guard.ok) return PAT_ERR_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (image_in)
    return P->fp64 ? run_image_in<double>(P, in, out, ws, s, op) : run_image_in<float>(P, in, out, ws, s, op);
  return P->fp64 ? run_traces_in<double>(P, in, out, ws, s, op) : run_traces_in<float>(P, in, out, ws, s, op);
}

void destroy_events(pat_plan* P) {
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  P->ev.clear();
  P->ev_stage.clear();
  P->ev_max = 0;
  P->ev_used = 0;
}

}  // namespace

extern "C" {

pat_status pat_plan_desc_init(pat_plan_desc* d) {
  if (!d) return PAT_ERR_INVALID_ARGUMENT;
  std::memset(d, 0, sizeof(*d));
  d->sigma_xy = 2.0;
  d->width_xy = 8;
  d->sigma_t = 2.0;
  d->width_t = 8;
  d->kernel = PAT_KERNEL_KAISER_BESSEL;
  d->precision = PAT_FP32;
  return PAT_OK;
}

pat_status nufft_plan(const pat_plan_desc* desc, void* stream, pat_plan** out) {
  if (!out) return PAT_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  pat_status st = validate(desc);
  if (st != PAT_OK) return st;
  pat_plan* P = new (std::nothrow) pat_plan();
  if (!P) return PAT_ERR_ALLOC;
  P->d = *desc;
  P->fp64 = desc->precision == PAT_FP64;
  if (hipGetDevice(&P->device) != hipSuccess) {
    (void)hipGetLastError();
    delete P;
    return PAT_ERR_HIP;
  }
  st = P->fp64 ? build_tables<double>(P, static_cast<hipStream_t>(stream))
               : build_tables<float>(P, static_cast<hipStream_t>(stream));
  P->d.sensor_xy = nullptr;  // host arrays were copied into the tables
  P->d.sensor_h = nullptr;
  if (st != PAT_OK) {
    dev_free(P->d, P->dev);
    delete P;
    return st;
  }
  *out = P;
  return PAT_OK;
}

pat_status nufft_plan_workspace_size(const pat_plan* P, size_t* bytes) {
  if (!P || !bytes) return PAT_ERR_INVALID_ARGUMENT;
  *bytes = P->ws_bytes;
  return PAT_OK;
}

pat_status pat_plan_get_info(const pat_plan* P, pat_plan_info* info) {
  if (!P || !info) return PAT_ERR_INVALID_ARGUMENT;
  std::memset(info, 0, sizeof(*info));
  info->nx_over = P->dp.n_x;
  info->ny_over = P->dp.n_y;
  info->nt_over = P->dp.n_t;
  info->band_lo = P->dp.b_lo;
  info->band_bins = P->dp.nb;
  info->time_origin = P->dp.n0;
  info->element_bytes = P->fp64 ? 8 : 4;
  info->spread_tiles = P->dp.tiles_x * P->dp.tiles_y;
  info->spread_pairs = P->spread_pairs;
  info->workspace_bytes = P->ws_bytes;
  info->table_bytes = P->dev_bytes;
  info->chunk_bins = P->dp.chunk_bins;
  info->rounds = rounds(P->dp);
  info->deconv_range_xy = P->range_xy;
  info->deconv_range_t = P->range_t;
  info->forward_fused = P->forward_fused ? 1 : 0;
  info->pad0 = 0;
  info->spread_slots = P->spread_slots;
  info->band_pairs = P->band_pairs;
  return PAT_OK;
}

pat_status nufft_plan_destroy(pat_plan* P) {
  if (!P) return PAT_OK;
  DeviceGuard guard(P->device);
  (void)hipDeviceSynchronize();
  destroy_events(P);
  dev_free(P->d, P->dev);
  delete P;
  return PAT_OK;
}

pat_status pat_reconstruct(pat_plan* P, const void* g, void* f, void* ws, void* stream) {
  return compute(P, g, f, ws, stream, OP_RECONSTRUCT);
}

pat_status pat_spectrum(pat_plan* P, const void* g, void* fhat, void* ws, void* stream) {
  return compute(P, g, fhat, ws, stream, OP_SPECTRUM);
}

pat_status pat_forward(pat_plan* P, const void* f, void* g, void* ws, void* stream) {
  return compute(P, f, g, ws, stream, OP_FORWARD);
}

pat_status pat_adjoint(pat_plan* P, const void* g, void* f, void* ws, void* stream) {
  return compute(P, g, f, ws, stream, OP_ADJOINT);
}

pat_status pat_forward_dxy(pat_plan* P, const void* f, int32_t axis, void* g, void* ws, void* stream) {
  if (axis != 0 && axis != 1) return PAT_ERR_INVALID_ARGUMENT;
  return compute(P, f, g, ws, stream, axis == 0 ? OP_FORWARD_DX : OP_FORWARD_DY);
}

pat_status pat_timing_begin(pat_plan* P, int32_t max_calls) {
  return pat_timing_begin_stages(P, max_calls, (1u << PAT_TIMING_STAGES) - 1u);
}

pat_status pat_timing_begin_stages(pat_plan* P, int32_t max_calls, uint32_t stage_mask) {
  if (!P || max_calls < 1 || max_calls > 100000 || stage_mask == 0 || stage_mask >= (1u << PAT_TIMING_STAGES))
    return PAT_ERR_INVALID_ARGUMENT;
  DeviceGuard guard(P->device);
  destroy_events(P);
  P->ev_mask = stage_mask;
  P->marks_per_call = 5 + 2 * rounds(P->dp);
  const size_t n = size_t(max_calls) * P->marks_per_call;
  P->ev.resize(n);
  P->ev_stage.assign(n, -1);
  for (size_t i = 0; i < n; ++i) {
    if (hipEventCreate(&P->ev[i]) != hipSuccess) {
      P->ev.resize(i);
      destroy_events(P);
      return PAT_ERR_HIP;
    }
  }
  P->ev_max = max_calls;
  P->ev_used = 0;
  return PAT_OK;
}

pat_status pat_timing_end(pat_plan* P, double* ms, int32_t nstage, int32_t* calls) {
  if (!P || (!ms && nstage > 0) || nstage < 0 || nstage > PAT_TIMING_STAGES) return PAT_ERR_INVALID_ARGUMENT;
  DeviceGuard guard(P->device);
  for (int i = 0; i < nstage; ++i) ms[i] = 0.0;
  pat_status st = PAT_OK;
  if (P->ev_used > 0 && hipDeviceSynchronize() != hipSuccess) st = PAT_ERR_HIP;
  for (int c = 0; c < P->ev_used && st == PAT_OK; ++c) {
    const size_t base = size_t(c) * P->marks_per_call;
    for (int k = 1; k < P->marks_per_call; ++k) {
      const int stage = P->ev_stage[base + k];
      if (stage < 0) break;
      if (!((P->ev_mask >> stage) & 1u)) continue;  // an untimed stage: its ends need not be events
      float t = 0.f;
      if (hipEventElapsedTime(&t, P->ev[base + k - 1], P->ev[base + k]) != hipSuccess) {
        st = PAT_ERR_HIP;
        break;
      }
      if (stage < nstage) ms[stage] += t;
    }
  }
  if (calls) *calls = P->ev_used;
  destroy_events(P);
  return st;
}

const char* pat_status_str(pat_status s) {
  switch (s) {
    case PAT_OK: return "PAT_OK";
    case PAT_ERR_INVALID_ARGUMENT: return "PAT_ERR_INVALID_ARGUMENT: invalid argument";
    case PAT_ERR_UNSUPPORTED: return "PAT_ERR_UNSUPPORTED: size or parameter not supported";
    case PAT_ERR_ALLOC: return "PAT_ERR_ALLOC: device allocation failed";
    case PAT_ERR_HIP: return "PAT_ERR_HIP: HIP runtime error";
    case PAT_ERR_NOT_IMPLEMENTED: return "PAT_ERR_NOT_IMPLEMENTED: not implemented";
    case PAT_ERR_WORKSPACE_TOO_LARGE:
      return "PAT_ERR_WORKSPACE_TOO_LARGE: the plan's workspace exceeds the library's fixed scratch "
             "(PAT_NOALLOC_SCRATCH_BYTES); use pat_reconstruct with a caller workspace";
  }
  return "unknown pat_status";
}

const char* pat_version(void) { return "patnufft 0.1 (gfx950)"; }

}  // extern "C"
