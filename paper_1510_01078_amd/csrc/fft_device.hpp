// Device-side complex helpers and an LDS-resident, self-sorting (Stockham)
// mixed-radix FFT for gfx950 work-groups.
//
// A work-group transforms `batch` sequences of length n that live in LDS
// (sequence f starts at buf + f*bstride, element a at slot lpos(a)). Each
// radix-R pass reads the R inputs of every butterfly into registers,
// applies the twiddles and the length-R DFT, waits at a barrier, then
// writes the outputs in Stockham order, so the transform runs in place in
// one LDS buffer and leaves the result in natural order. With p the product
// of the radices already done, butterfly i (0 <= i < n/R, k = i mod p)
// reads x[i + r*n/R], multiplies input r by w^(r*k*n/(p*R)) with
// w = exp(-2*pi*i/n) (conjugated for the inverse) and writes output r to
// position (i-k)*R + k + r*p.
#pragma once
#include <hip/hip_runtime.h>

namespace patk {

template <typename T>
struct cx {
  T x, y;
};

// Store that streams past the caches (the value is read once, later, by the
// next kernel), as two non-temporal 32- or 64-bit stores.
template <typename T>
__device__ __forceinline__ void nt_store(cx<T>* p, cx<T> v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
template <typename T>
__device__ __forceinline__ cx<T> nt_load(const cx<T>* p) {
  return cx<T>{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
}

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

// One radix pass: radix R, p = product of the radices before it, nbf = n/R
// butterflies per sequence, twstep = n/(p*R), and multipliers for exact
// division by nbf and by p (q = umulhi(x, m) for x < 2^16; m = 0 marks a
// divisor of 1).
struct FftPass {
  int R, p, nbf, twstep;
  uint32_t m_nbf, m_p;
};

// Descriptor of one FFT length: the pass sequence and its twiddle table
// tw[t] = exp(-2*pi*i*t/n), t = 0..n-1 (computed in double on the host).
template <typename T>
struct FftDesc {
  int n;
  int npass;
  const FftPass* pass;  // device array of npass entries
  const cx<T>* tw;
};

// Twiddle sources w(t) = exp(-2*pi*i*t/n), 0 <= t < n, for the passes below.
// TwTable reads a full table (global memory or a copy in LDS). TwSplit
// multiplies two short LDS tables, w(t) = w(64*(t >> 6)) * w(t & 63): n/64 +
// 64 entries instead of n (832 bytes instead of 20 KiB at 2560 points), for
// one complex multiply more per twiddle and about one more rounding.
template <typename T>
struct TwTable {
  const cx<T>* tw;
  __device__ __forceinline__ cx<T> operator()(int t) const { return tw[t]; }
};

template <typename T>
struct TwSplit {
  const cx<T>* hi;  // hi[u] = w(64 u), u < ceil(n / 64)
  const cx<T>* lo;  // lo[v] = w(v), v < min(n, 64)
  __device__ __forceinline__ cx<T> operator()(int t) const { return cmul(hi[t >> 6], lo[t & 63]); }
};

// Entries of the split tables of an n-point transform.
__host__ __device__ constexpr int tw_split_slots(int n) { return (n + 63) / 64 + 64; }

// Fill the split tables at `slots` (tw_split_slots(n) entries) from the full
// table; the caller's next barrier publishes them.
template <typename T>
__device__ __forceinline__ TwSplit<T> tw_split_fill(cx<T>* slots, const cx<T>* __restrict__ tw, int n, int tid,
                                                    int nthr) {
  const int nh = (n + 63) / 64;
  for (int i = tid; i < nh + 64; i += nthr) {
    if (i < nh) slots[i] = tw[64 * i];
    else if (i - nh < n) slots[i] = tw[i - nh];
  }
  return TwSplit<T>{slots, slots + nh};
}

__device__ __forceinline__ int fdiv(int x, uint32_t m) { return m ? int(__umulhi(uint32_t(x), m)) : x; }

// Exact x / d for 0 <= x, d < 2^16 by a multiply-high (the multiplier is
// computed once, so loops over flattened indices avoid integer division).
struct FastDiv {
  uint32_t m;
  __device__ __forceinline__ explicit FastDiv(int d) : m(d == 1 ? 0u : 0xFFFFFFFFu / uint32_t(d) + 1u) {}
  __device__ __forceinline__ int operator()(int x) const { return m ? int(__umulhi(uint32_t(x), m)) : x; }
};

// Move `count` elements through registers: every thread first issues all of
// its (at most U) loads, then all of its stores, so many global accesses are
// in flight at once. Requires count <= U * nthr.
template <int U, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int count, int tid, int nthr, Load ld, Store st) {
  using V = decltype(ld(0));
  V tmp[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * nthr;
    if (q < count) tmp[u] = ld(q);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int q = tid + u * nthr;
    if (q < count) st(q, tmp[u]);
  }
}

// The same for the compile-time FFT kernels, whose geometry is known: a block
// of nrows <= ROWS rows of N elements, thread t taking elements t, t + NT, ...
// of every row, so no index needs a division (ld(r, c), st(r, c, v)).
template <int ROWS, int N, int NT, typename Load, typename Store>
__device__ __forceinline__ void staged_rows(int nrows, int tid, Load ld, Store st) {
  constexpr int CPR = (N + NT - 1) / NT;
  static_assert(ROWS * CPR <= 16, "at most 16 staged values per thread");
  using V = decltype(ld(0, 0));
  V tmp[ROWS][CPR];
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int k = 0; k < CPR; ++k) {
      const int c = tid + k * NT;
      if (r < nrows && (N % NT == 0 || c < N)) tmp[r][k] = ld(r, c);
    }
#pragma unroll
  for (int r = 0; r < ROWS; ++r)
#pragma unroll
    for (int k = 0; k < CPR; ++k) {
      const int c = tid + k * NT;
      if (r < nrows && (N % NT == 0 || c < N)) st(r, c, tmp[r][k]);
    }
}

// Columns of a ROWS-row block written out column by column (element (j, r)
// of column j < ncols, row r < nrows): thread t takes row t % ROWS of columns
// t / ROWS + u * (NT / ROWS), u = 0, 1, ... (at most U of them), so
// neighbouring threads write neighbouring rows of one column and the column
// index steps by a constant (ld(j, r, u), st(j, r, u, v)).
template <int ROWS, int NT, int U, typename Load, typename Store>
__device__ __forceinline__ void staged_cols(int ncols, int nrows, int tid, Load ld, Store st) {
  static_assert(NT % ROWS == 0, "rows must divide the thread count");
  constexpr int CPI = NT / ROWS;
  using V = decltype(ld(0, 0, 0));
  const int r = tid % ROWS, j0 = tid / ROWS;
  V tmp[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = j0 + u * CPI;
    if (j < ncols && r < nrows) tmp[u] = ld(j, r, u);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int j = j0 + u * CPI;
    if (j < ncols && r < nrows) st(j, r, u, tmp[u]);
  }
}

// LDS slot of element a of a sequence: one pad slot after every
// 2^kLdsPadShift elements, so the stride-R stores of the first radix-8
// passes hit distinct banks. Runs of 16 measured fastest on MI355X: a pad
// every 8 elements puts a wave's contiguous 8-byte accesses across a pad
// (bank conflicts on every contiguous pass), runs of 32 slowed the lateral
// x and y transforms.
constexpr int kLdsPadShift = 4;
constexpr int kLdsPadRun = 1 << kLdsPadShift;
__host__ __device__ __forceinline__ constexpr int lpos(int a) { return a + (a >> kLdsPadShift); }
// Slots one sequence of length n occupies (odd, so sequences start on different banks).
__host__ __device__ __forceinline__ constexpr int lseq(int n) { return n + (n >> kLdsPadShift) + 1; }

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

// Radix 6 as two length-3 DFTs of the even and odd inputs, combined with the
// sixth roots of unity: X_k = E_(k mod 3) + w6^k O_(k mod 3), w6^(k+3) = -w6^k.
template <typename T, bool INV>
struct Dft<T, 6, INV> {
  __device__ __forceinline__ static void run(cx<T>* a) {
    const T s = INV ? T(1) : T(-1);
    const T h = T(0.86602540378443864676372317075294);  // sin(pi/3)
    cx<T> e[3] = {a[0], a[2], a[4]};
    cx<T> o[3] = {a[1], a[3], a[5]};
    Dft<T, 3, INV>::run(e);
    Dft<T, 3, INV>::run(o);
    // w6 = 1/2 + s i h, w6^2 = -1/2 + s i h
    const cx<T> o1 = cx<T>{T(0.5) * o[1].x - s * h * o[1].y, T(0.5) * o[1].y + s * h * o[1].x};
    const cx<T> o2 = cx<T>{T(-0.5) * o[2].x - s * h * o[2].y, T(-0.5) * o[2].y + s * h * o[2].x};
    a[0] = e[0] + o[0];
    a[3] = e[0] - o[0];
    a[1] = e[1] + o1;
    a[4] = e[1] - o1;
    a[2] = e[2] + o2;
    a[5] = e[2] - o2;
  }
};

// Ordering between the read and write phases of a pass: a work-group barrier,
// or (when one wave owns the sequences) wave-local ordering of its LDS traffic.
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One radix-R Stockham pass over `batch` sequences; every thread holds at
// most MAXV values, so batch*n <= MAXV*nthr is required (and batch*n < 2^16).
template <typename T, int R, int MAXV, bool INV, bool WAVE, typename TW>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, const FftPass& ps, int batch, int bstride, TW tw, int tid,
                                              int nthr) {
  constexpr int K = (MAXV + R - 1) / R;
  const int nbf = ps.nbf;
  const int p = ps.p;
  const int total = nbf * batch;
  cx<T> v[K][R];
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * nthr;
    if (idx < total) {
      const int f = fdiv(idx, ps.m_nbf);
      const int i = idx - f * nbf;
      const cx<T>* src = buf + f * bstride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[it][r] = src[lpos(i + r * nbf)];
      const int k = i - fdiv(i, ps.m_p) * p;
      if (k != 0) {
        const int ts = k * ps.twstep;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cx<T> w = tw(r * ts);
          if (INV) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      Dft<T, R, INV>::run(v[it]);
    }
  }
  fft_sync<WAVE>();
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * nthr;
    if (idx < total) {
      const int f = fdiv(idx, ps.m_nbf);
      const int i = idx - f * nbf;
      const int k = i - fdiv(i, ps.m_p) * p;
      cx<T>* dst = buf + f * bstride;
      const int j0 = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[lpos(j0 + r * p)] = v[it][r];
    }
  }
  fft_sync<WAVE>();
}

// Full transform (all passes). With WAVE = false the work-group's threads
// cooperate on `batch` sequences and callers must __syncthreads() after
// filling buf; with WAVE = true the 64 lanes of one wave (tid = lane,
// nthr = 64) own the sequences and only wave-local ordering is used.
template <typename T, int MAXV, bool INV, bool WAVE, typename TW>
__device__ __forceinline__ void fft_lds_tw(cx<T>* buf, const FftDesc<T> fd, TW tw, int batch, int bstride, int tid,
                                           int nthr) {
  for (int s = 0; s < fd.npass; ++s) {
    const FftPass ps = fd.pass[s];
    switch (ps.R) {
      case 8: stockham_pass<T, 8, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
      case 4: stockham_pass<T, 4, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
      case 2: stockham_pass<T, 2, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
      case 3: stockham_pass<T, 3, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
      case 6: stockham_pass<T, 6, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
      default: stockham_pass<T, 5, MAXV, INV, WAVE>(buf, ps, batch, bstride, tw, tid, nthr); break;
    }
  }
}

template <typename T, int MAXV, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_lds(cx<T>* buf, const FftDesc<T> fd, int batch, int bstride, int tid, int nthr) {
  fft_lds_tw<T, MAXV, INV, WAVE>(buf, fd, TwTable<T>{fd.tw}, batch, bstride, tid, nthr);
}

// ---------------------------------------------------------------------------
// Compile-time form for one length N: the same passes (radices taken greedily
// in the order 8, 6, 4, 2, 5, 3, as the host planner does), twiddle reads and
// butterflies as fft_lds with the host plan for N (the compiler may fuse
// multiplies and adds differently in the two forms, so results agree to
// rounding, and bit for bit where it does not); with N, the radix, p and the
// butterfly count known to the compiler,
// the index arithmetic folds to constants and the LDS offsets of a
// butterfly's R inputs and outputs become instruction immediates where the
// pad pattern allows (strides that are multiples of 8 slots). Sequences sit
// lseq(N) slots apart. NT threads cooperate on at most MAXB sequences
// (WAVE = true: one wave, nthr = 64, wave-local ordering only).
// ---------------------------------------------------------------------------
struct CtPlan {
  int np;
  int r[16];
};

__host__ __device__ constexpr CtPlan ct_plan(int n) {
  CtPlan c{0, {}};
  const int rs[6] = {8, 6, 4, 2, 5, 3};
  int m = n;
  for (int q = 0; q < 6; ++q)
    while (m % rs[q] == 0 && c.np < 16) {
      c.r[c.np++] = rs[q];
      m /= rs[q];
    }
  return c;
}

__host__ __device__ constexpr int ct_prefix(int n, int s) {
  const CtPlan c = ct_plan(n);
  int p = 1;
  for (int i = 0; i < s; ++i) p *= c.r[i];
  return p;
}

template <typename T, int N, int S, int NT, int MAXB, bool INV, bool WAVE, typename TW>
__device__ __forceinline__ void ct_pass(cx<T>* buf, int batch, TW tw, int tid) {
  constexpr CtPlan pl = ct_plan(N);
  constexpr int R = pl.r[S];
  constexpr int P = ct_prefix(N, S);
  constexpr int NBF = N / R;
  constexpr int TWS = N / (P * R);
  constexpr int BS = lseq(N);
  constexpr int K = (NBF * MAXB + NT - 1) / NT;
  const int total = NBF * batch;
  // butterfly (sequence f, index i) of iteration it: idx = tid + it*NT, with
  // f and i stepped from the previous iteration's (no divisions after the first)
  int fq[K], iq[K];
  fq[0] = tid / NBF;
  iq[0] = tid - fq[0] * NBF;
#pragma unroll
  for (int it = 1; it < K; ++it) {
    constexpr int DF = NT / NBF, DI = NT % NBF;
    const bool wrap = iq[it - 1] + DI >= NBF;
    iq[it] = iq[it - 1] + DI - (wrap ? NBF : 0);
    fq[it] = fq[it - 1] + DF + (wrap ? 1 : 0);
  }
  cx<T> v[K][R];
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * NT;
    if (idx < total) {
      const int f = fq[it];
      const int i = iq[it];
      const cx<T>* src = buf + f * BS;
      if constexpr (NBF % kLdsPadRun == 0) {
        const cx<T>* s0 = src + lpos(i);
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = s0[r * lpos(NBF)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = src[lpos(i + r * NBF)];
      }
      if constexpr (P > 1) {
        const int k = i % P;
        if (k != 0) {
          const int ts = k * TWS;
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = tw(r * ts);
            if (INV) w.y = -w.y;
            v[it][r] = cmul(v[it][r], w);
          }
        }
      }
      Dft<T, R, INV>::run(v[it]);
    }
  }
  fft_sync<WAVE>();
#pragma unroll
  for (int it = 0; it < K; ++it) {
    const int idx = tid + it * NT;
    if (idx < total) {
      const int f = fq[it];
      const int i = iq[it];
      cx<T>* dst = buf + f * BS;
      if constexpr (P == 1) {
        // j0 = i*R; for R = 8 the outputs r share one padded run: lpos(8i) + r
        if constexpr (R == 8 && kLdsPadRun % 8 == 0) {
          cx<T>* d0 = dst + lpos(8 * i);
#pragma unroll
          for (int r = 0; r < R; ++r) d0[r] = v[it][r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) dst[lpos(i * R + r)] = v[it][r];
        }
      } else {
        const int k = i % P;
        const int j0 = (i - k) * R + k;
        if constexpr (P % kLdsPadRun == 0) {
          cx<T>* d0 = dst + lpos(j0);
#pragma unroll
          for (int r = 0; r < R; ++r) d0[r * lpos(P)] = v[it][r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) dst[lpos(j0 + r * P)] = v[it][r];
        }
      }
    }
  }
  fft_sync<WAVE>();
}

template <typename T, int N, int S, int NT, int MAXB, bool INV, bool WAVE, typename TW>
__device__ __forceinline__ void ct_passes(cx<T>* buf, int batch, TW tw, int tid) {
  if constexpr (S < ct_plan(N).np) {
    ct_pass<T, N, S, NT, MAXB, INV, WAVE>(buf, batch, tw, tid);
    ct_passes<T, N, S + 1, NT, MAXB, INV, WAVE>(buf, batch, tw, tid);
  }
}

// Transform `batch` (<= MAXB) sequences of length N at buf + f*lseq(N),
// twiddles from the source tw (fft_ct: a full table).
template <typename T, int N, int NT, int MAXB, bool INV, bool WAVE = false, typename TW>
__device__ __forceinline__ void fft_ct_tw(cx<T>* buf, int batch, TW tw, int tid) {
  static_assert(ct_prefix(N, ct_plan(N).np) == N, "length must factor into 2, 3, 5");
  ct_passes<T, N, 0, NT, MAXB, INV, WAVE>(buf, batch, tw, tid);
}

template <typename T, int N, int NT, int MAXB, bool INV, bool WAVE = false>
__device__ __forceinline__ void fft_ct(cx<T>* buf, int batch, const cx<T>* __restrict__ tw, int tid) {
  fft_ct_tw<T, N, NT, MAXB, INV, WAVE>(buf, batch, TwTable<T>{tw}, tid);
}

}  // namespace patk
