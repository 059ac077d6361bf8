// Host arithmetic of a plan's lengths, free of HIP so that it can be built
// and checked by a plain C++ compiler: the oversampled FFT lengths and the
// band of oversampled temporal bins that the interpolation at omega(K)
// reads (Section 3.1: the window sum of eq. NER_NUFFT touches the w_t bins
// nearest each non-equispaced frequency).
#pragma once
#include <cmath>
#include <initializer_list>

namespace patsz {

inline bool smooth235(long n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// smallest even 2,3,5-smooth integer >= v (and >= 2)
inline int next_smooth_even(double v) {
  long n = (long)std::ceil(v - 1e-9);
  if (n < 2) n = 2;
  while (!(smooth235(n) && n % 2 == 0)) ++n;
  return (int)n;
}

// Longest temporal FFT the kernels take (512 threads x 16 values).
constexpr int kMaxTemporalFft = 8192;

struct Band {
  int n_t = 0;   // oversampled temporal FFT length
  int b_lo = 0;  // first kept bin (may be negative: the bins wrap)
  int nb = 0;    // kept bins, always even
  bool ok = false;
};

// Band of oversampled bins for interpolation points s = |K| c dt n_t/(2 pi)
// with |K| from 0 to kmax and wt taps: bins -wt/2 .. floor(s_max) + wt/2 + 1.
// The count is rounded up to an even number, so in single precision every
// sensor's row of band values (nb complex floats) spans a whole number of
// 16-byte units and each row starts on a 16-byte boundary. Short traces can
// need more bins than smooth(sigma_t Nt) holds: the FFT is then lengthened
// until the band fits (more oversampling). ok = false when no FFT up to
// kMaxTemporalFft points holds it (|omega| dt close to or beyond pi).
inline Band temporal_band(double sigma_t, int Nt, int wt, double kmax, double c, double dt) {
  Band b;
  b.n_t = next_smooth_even(sigma_t * Nt);
  for (;;) {
    const double smax = kmax * c * dt * b.n_t / (2.0 * M_PI);
    const long blo = -wt / 2;
    long bhi = (long)std::floor(smax) + wt / 2 + 1;
    if ((bhi - blo + 1) % 2) ++bhi;
    if (bhi - blo + 1 <= b.n_t && bhi < b.n_t) {
      b.b_lo = (int)blo;
      b.nb = (int)(bhi - blo + 1);
      b.ok = true;
      return b;
    }
    if (b.n_t >= kMaxTemporalFft) return b;
    b.n_t = next_smooth_even(b.n_t + 1);
  }
}

}  // namespace patsz
