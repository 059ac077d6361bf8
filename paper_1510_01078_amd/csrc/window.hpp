// Host-side (double precision) window functions for the NUFFT steps.
//
// The window Psi of Section 3.1 (eq. NUFFT1) must be supported on a finite
// interval, positive on the band, and have a Fourier transform concentrated
// near the origin (Section 3.1 names the Kaiser-Bessel function). Here the
// window is written on the oversampled grid's index scale: phi(x), support
// |x| <= w/2 for a footprint of w grid points, with continuous transform
// phihat(xi) = integral phi(x) exp(-2 pi i xi x) dx (xi in cycles per grid
// step). Spreading uses phi at the w grid points nearest a sample; the
// deconvolution divides by phihat at the kept modes (the division by Psi_j
// of eq. NED_NUFFT and by Psi_n of eq. NER_NUFFT).
#pragma once
#include <cmath>
#include <vector>

namespace pathost {

// Modified Bessel function I0 by its power series (all terms positive).
inline double bessel_i0(double z) {
  const double q = 0.25 * z * z;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / (double(k) * double(k));
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// Gauss-Legendre nodes/weights on [-1, 1] (Newton on Legendre polynomials).
inline void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct Window {
  int kind = 1;       // 0 Gaussian, 1 Kaiser-Bessel
  int w = 8;          // footprint in grid points
  double sigma = 2.0; // oversampling factor the shape is tuned for
  double beta = 0.0;  // Kaiser-Bessel shape
  double a = 0.0;     // Gaussian exp(-a x^2)
  std::vector<double> qx, qw;  // quadrature for the truncated Gaussian transform

  Window() = default;
  Window(int kind_, int w_, double sigma_) : kind(kind_), w(w_), sigma(sigma_) {
    if (kind == 1) {
      // Beatty, Nishimura, Pauly (2005) shape for oversampling sigma
      double r = (double(w) / sigma) * (sigma - 0.5);
      double v = r * r - 0.8;
      beta = M_PI * std::sqrt(v > 0.1 ? v : 0.1);
    } else {
      // Greengard-Lee (2004) Gaussian width for half-width w/2 and ratio sigma
      a = M_PI * (sigma - 0.5) / (sigma * 0.5 * w);
      gauss_legendre(96, qx, qw);
      for (size_t i = 0; i < qx.size(); ++i) {
        qx[i] *= 0.5 * w;
        qw[i] *= 0.5 * w;
      }
    }
  }

  double phi(double x) const {
    const double hw = 0.5 * w;
    if (std::fabs(x) > hw) return 0.0;
    if (kind == 1) {
      double t = x / hw;
      double r = 1.0 - t * t;
      return bessel_i0(beta * std::sqrt(r > 0.0 ? r : 0.0));
    }
    return std::exp(-a * x * x);
  }

  double phihat(double xi) const {
    if (kind == 1) {
      // integral over |x| <= w/2 of I0(beta sqrt(1 - (2x/w)^2)) e^{-2 pi i xi x} dx
      //   = w sinh(sqrt(beta^2 - (pi w xi)^2)) / sqrt(beta^2 - (pi w xi)^2)
      double u = M_PI * w * xi;
      double z = beta * beta - u * u;
      if (z > 1e-12) {
        double s = std::sqrt(z);
        return w * std::sinh(s) / s;
      } else if (z < -1e-12) {
        double s = std::sqrt(-z);
        return w * std::sin(s) / s;
      }
      return double(w);
    }
    // Gaussian: the truncated window's transform by Gauss-Legendre quadrature
    double s = 0.0;
    for (size_t i = 0; i < qx.size(); ++i) s += qw[i] * std::exp(-a * qx[i] * qx[i]) * std::cos(2.0 * M_PI * xi * qx[i]);
    return s;
  }
};

// Per-tap polynomial fits of the temporal interpolation weights. With
// s = fl + f (fl = floor(s), f in [0,1)), tap t (0 <= t < w) sits at bin
// fl - w/2 + 1 + t and carries phi(f + w/2 - 1 - t). Each tap's weight is a
// smooth function of y = 2f - 1 on [-1, 1]; it is interpolated at Chebyshev
// points and stored as monomial coefficients in y (coef[t*(deg+1) + d]).
// Returns the max abs error (relative to phi(0)) seen on a dense check grid.
inline double fit_tap_polynomials(const Window& win, int deg, std::vector<double>& coef) {
  const int w = win.w;
  const int np = deg + 1;
  coef.assign(size_t(w) * np, 0.0);
  std::vector<double> nodes(np), vals(np), cheb(np);
  for (int i = 0; i < np; ++i) nodes[i] = std::cos(M_PI * (i + 0.5) / np);
  // monomial expansion of Chebyshev polynomials T_0..T_deg
  std::vector<std::vector<double>> Tm(np, std::vector<double>(np, 0.0));
  Tm[0][0] = 1.0;
  if (np > 1) Tm[1][1] = 1.0;
  for (int k = 2; k < np; ++k)
    for (int d = 0; d < np; ++d) Tm[k][d] = (d > 0 ? 2.0 * Tm[k - 1][d - 1] : 0.0) - Tm[k - 2][d];
  for (int t = 0; t < w; ++t) {
    for (int i = 0; i < np; ++i) {
      double f = 0.5 * (nodes[i] + 1.0);
      vals[i] = win.phi(f + 0.5 * w - 1.0 - t);
    }
    for (int k = 0; k < np; ++k) {
      double s = 0.0;
      for (int i = 0; i < np; ++i) s += vals[i] * std::cos(M_PI * k * (i + 0.5) / np);
      cheb[k] = (k == 0 ? 1.0 : 2.0) * s / np;
    }
    for (int k = 0; k < np; ++k)
      for (int d = 0; d < np; ++d) coef[size_t(t) * np + d] += cheb[k] * Tm[k][d];
  }
  const double peak = win.phi(0.0);
  double err = 0.0;
  for (int i = 0; i <= 400; ++i) {
    double f = (i < 400) ? i / 400.0 : 0.999999;
    double y = 2.0 * f - 1.0;
    for (int t = 0; t < w; ++t) {
      double v = 0.0;
      for (int d = deg; d >= 0; --d) v = v * y + coef[size_t(t) * np + d];
      double e = std::fabs(v - win.phi(f + 0.5 * w - 1.0 - t)) / peak;
      if (e > err) err = e;
    }
  }
  return err;
}

}  // namespace pathost
