// Device-side complex helpers and an LDS-resident, self-sorting (Stockham)
// mixed-radix FFT for gfx950 work-groups.
//
// A work-group transforms `batch` sequences of length n that live in LDS
// (sequence f starts at buf + f*bstride). Each radix-R pass reads the R
// inputs of every butterfly into registers, applies the twiddles and the
// length-R DFT, waits at a barrier, then writes the outputs in Stockham
// order, so the transform runs in place in one LDS buffer and leaves the
// result in natural order. With p the product of the radices already done,
// butterfly i (0 <= i < n/R, k = i mod p) reads x[i + r*n/R], multiplies
// input r by w^(r*k*n/(p*R)) with w = exp(-2*pi*i/n) (conjugated for the
// inverse) and writes output r to position (i-k)*R + k + r*p.
#pragma once
#include <hip/hip_runtime.h>

namespace patk {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return cx<T>{a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return cx<T>{a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return cx<T>{a.x * s, a.y * s}; }
// a * (i*s) for s = +-1
template <typename T>
__device__ __forceinline__ cx<T> mul_is(cx<T> a, T s) { return cx<T>{-s * a.y, s * a.x}; }

// Descriptor of one FFT length: the radix sequence and its twiddle table
// tw[t] = exp(-2*pi*i*t/n), t = 0..n-1 (computed in double on the host).
template <typename T>
struct FftDesc {
  int n;
  int npass;
  int radix[16];
  const cx<T>* tw;
};

// Length-R DFT in place; INV selects exp(+2 pi i rk/R).
template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s = INV ? T(1) : T(-1);  // factor i*s multiplies the odd difference
    cx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    cx<T> t2 = a[1] + a[3], t3 = mul_is(a[1] - a[3], s);
    a[0] = t0 + t2;
    a[2] = t0 - t2;
    a[1] = t1 + t3;
    a[3] = t1 - t3;
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s = INV ? T(1) : T(-1);
    const T r2 = T(0.70710678118654752440084436210485);
    cx<T> e[4] = {a[0], a[2], a[4], a[6]};
    cx<T> o[4] = {a[1], a[3], a[5], a[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
    // w8^k = exp(s*i*pi*k/4)
    cx<T> o1 = cx<T>{r2 * (o[1].x - s * o[1].y), r2 * (o[1].y + s * o[1].x)};
    cx<T> o2 = mul_is(o[2], s);
    cx<T> o3 = cx<T>{r2 * (-o[3].x - s * o[3].y), r2 * (-o[3].y + s * o[3].x)};
    a[0] = e[0] + o[0];
    a[4] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[5] = e[1] - o1;
    a[2] = e[2] + o2;
    a[6] = e[2] - o2;
    a[3] = e[3] + o3;
    a[7] = e[3] - o3;
  }
};

template <typename T, bool INV>
struct Dft<T, 3, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s = INV ? T(1) : T(-1);
    const T h = T(0.86602540378443864676372317075294);  // sin(2 pi/3)
    cx<T> t = a[1] + a[2];
    cx<T> d = mul_is(a[1] - a[2], s * h);
    cx<T> m = cx<T>{a[0].x - T(0.5) * t.x, a[0].y - T(0.5) * t.y};
    a[0] = a[0] + t;
    a[1] = m + d;
    a[2] = m - d;
  }
};

template <typename T, bool INV>
struct Dft<T, 5, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s = INV ? T(1) : T(-1);
    const T c1 = T(0.30901699437494742410229341718282);   // cos(2 pi/5)
    const T c2 = T(-0.80901699437494742410229341718282);  // cos(4 pi/5)
    const T s1 = T(0.95105651629515357211643933337938);   // sin(2 pi/5)
    const T s2 = T(0.58778525229247312916870595463907);   // sin(4 pi/5)
    cx<T> t1 = a[1] + a[4], t2 = a[2] + a[3];
    cx<T> d1 = a[1] - a[4], d2 = a[2] - a[3];
    cx<T> m1 = cx<T>{a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y};
    cx<T> m2 = cx<T>{a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y};
    cx<T> n1 = mul_is(cx<T>{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y}, s);
    cx<T> n2 = mul_is(cx<T>{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y}, s);
    a[0] = a[0] + t1 + t2;
    a[1] = m1 + n1;
    a[4] = m1 - n1;
    a[2] = m2 + n2;
    a[3] = m2 - n2;
  }
};

// One radix-R Stockham pass over `batch` sequences; every thread holds at
// most MAXV values, so batch*n <= MAXV*nthr is required.
template <typename T, int R, int MAXV, bool INV>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int n, int p, int batch, int bstride,
                                              const cx<T>* __restrict__ tw, int tid, int nthr) {
  constexpr int K = (MAXV + R - 1) / R;
  const int nbf = n / R;
  const int total = nbf * batch;
  const int twstep = n / (p * R);
  cx<T> v[K][R];
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * nthr;
    if (idx < total) {
      const int f = idx / nbf;
      const int i = idx - f * nbf;
      const cx<T>* src = buf + f * bstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = src[i + r * nbf];
      const int k = i % p;
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw[r * k * twstep];
          if (INV) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      Dft<T, R, INV>::run(v[it]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * nthr;
    if (idx < total) {
      const int f = idx / nbf;
      const int i = idx - f * nbf;
      const int k = i % p;
      cx<T>* dst = buf + f * bstride;
      const int j = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[j + r * p] = v[it][r];
    }
  }
  __syncthreads();
}

// Full transform (all passes). Callers must __syncthreads() after filling buf.
template <typename T, int MAXV, bool INV>
__device__ void fft_lds(cx<T>* buf, const FftDesc<T>& fd, int batch, int bstride, int tid, int nthr) {
  int p = 1;
  for (int s = 0; s < fd.npass; ++s) {
    const int R = fd.radix[s];
    switch (R) {
      case 8: stockham_pass<T, 8, MAXV, INV>(buf, fd.n, p, batch, bstride, fd.tw, tid, nthr); break;
      case 4: stockham_pass<T, 4, MAXV, INV>(buf, fd.n, p, batch, bstride, fd.tw, tid, nthr); break;
      case 2: stockham_pass<T, 2, MAXV, INV>(buf, fd.n, p, batch, bstride, fd.tw, tid, nthr); break;
      case 3: stockham_pass<T, 3, MAXV, INV>(buf, fd.n, p, batch, bstride, fd.tw, tid, nthr); break;
      default: stockham_pass<T, 5, MAXV, INV>(buf, fd.n, p, batch, bstride, fd.tw, tid, nthr); break;
    }
    p *= R;
  }
}

}  // namespace patk
