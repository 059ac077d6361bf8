// Interpolation from the oversampled lateral grid to the sensors: the
// transpose of the lateral gridding (the type-2 counterpart of
// eq. NED_NUFFT), used by the forward model.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_common.hpp"

namespace patk {

// ---------------------------------------------------------------------------
//   Gt'[m][b] = sum_{ty,tx < w} wy_m[ty] wx_m[tx] U'[b][(by_m + ty) mod n_y][(bx_m + tx) mod n_x]
// with the spread's footprint origin and weights. A work-group owns one
// 16x16 home tile (the tile holding the footprint origins of its sensors)
// and `bc` bins: it stages the tile plus a (w-1) halo of those bins in LDS
// (periodic wrap), then one thread per (sensor, bin) pair sums the footprint
// from LDS. Each output is written once; no atomics.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_interp(const cx<T>* __restrict__ U, int nb, const int* __restrict__ home_off,
                                                const int* __restrict__ home_sens, const int* __restrict__ sbx,
                                                const int* __restrict__ sby, const T* __restrict__ swx,
                                                const T* __restrict__ swy, int w, int n_x, int n_y, int tiles_x,
                                                int nchunks, int bc, int b_begin, int b_end, cx<T>* __restrict__ Gt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cx<T>* patch = reinterpret_cast<cx<T>*>(smem_raw);
  const int chunk = blockIdx.x % nchunks;
  const int tile = blockIdx.x / nchunks;
  const int q0 = home_off[tile], q1 = home_off[tile + 1];
  if (q0 == q1) return;
  const int tyi = tile / tiles_x;
  const int txi = tile - tyi * tiles_x;
  const int tx0 = txi * kSpreadTile, ty0 = tyi * kSpreadTile;
  const int P = kSpreadTile + w - 1;  // patch edge
  const int PR = P | 1;               // odd row pitch
  const int plane = P * PR;
  const int b0 = b_begin + chunk * bc;
  const int nbc = min(bc, b_end - b0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const size_t slice = size_t(n_y) * n_x;
  const FastDiv div_p(P), div_pp(P * P);
  // stage the patch: each thread issues up to kStage loads before its LDS stores
  constexpr int kStage = 8;
  const int total = nbc * P * P;
  for (int q0s = 0; q0s < total; q0s += kStage * nthr) {
    cx<T> v[kStage];
    int dst[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int q = q0s + tid + u * nthr;
      dst[u] = -1;
      if (q < total) {
        const int bi = div_pp(q);
        const int rem = q - bi * P * P;
        const int r = div_p(rem);
        const int cc = rem - r * P;
        int py = ty0 + r;
        while (py >= n_y) py -= n_y;
        int px = tx0 + cc;
        while (px >= n_x) px -= n_x;
        v[u] = U[size_t(b0 - b_begin + bi) * slice + size_t(py) * n_x + px];
        dst[u] = bi * plane + r * PR + cc;
      }
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u)
      if (dst[u] >= 0) patch[dst[u]] = v[u];
  }
  __syncthreads();
  const int npairs = (q1 - q0) * nbc;  // may exceed 2^16: plain division below
  for (int pq = tid; pq < npairs; pq += nthr) {
    const int qi = pq / nbc;
    const int bi = pq - qi * nbc;
    const int m = home_sens[q0 + qi];
    const int ox = sbx[m] - tx0, oy = sby[m] - ty0;
    const T* wx = swx + size_t(m) * w;
    const T* wy = swy + size_t(m) * w;
    const cx<T>* pp = patch + bi * plane + oy * PR + ox;
    cx<T> acc{T(0), T(0)};
    for (int ty = 0; ty < w; ++ty) {
      cx<T> row{T(0), T(0)};
      for (int tx = 0; tx < w; ++tx) {
        const cx<T> v = pp[ty * PR + tx];
        row.x += wx[tx] * v.x;
        row.y += wx[tx] * v.y;
      }
      acc.x += wy[ty] * row.x;
      acc.y += wy[ty] * row.y;
    }
    Gt[size_t(m) * nb + b0 + bi] = acc;
  }
}

// bins per work-group: the largest of 8, 4, 2, 1 whose patch fits 40 KiB
// (four work-groups per CU)
template <typename T>
static int interp_bins(int w) {
  const int P = kSpreadTile + w - 1;
  const size_t plane = size_t(P) * (P | 1) * sizeof(cx<T>);
  int bc = 8;
  while (bc > 1 && plane * bc > 40960) bc >>= 1;
  return bc;
}

template <typename T>
hipError_t launch_interp(const DevPlan& p, const void* U, void* Gt, int b_begin, int b_end, hipStream_t s) {
  if (p.w_xy > 16 || b_begin < 0 || b_end > p.nb || b_begin >= b_end) return hipErrorInvalidValue;
  const int bc = interp_bins<T>(p.w_xy);
  const int P = kSpreadTile + p.w_xy - 1;
  const size_t lds = size_t(P) * (P | 1) * sizeof(cx<T>) * bc;
  hipError_t e = allow_lds(reinterpret_cast<const void*>(&k_interp<T>), lds);
  if (e != hipSuccess) return e;
  const int nchunks = (b_end - b_begin + bc - 1) / bc;
  const long long blocks = (long long)p.tiles_x * p.tiles_y * nchunks;
  hipLaunchKernelGGL(k_interp<T>, dim3((unsigned)blocks), dim3(256), lds, s, static_cast<const cx<T>*>(U), p.nb,
                     p.home_off, p.home_sens, p.sbx, p.sby, static_cast<const T*>(p.swx), static_cast<const T*>(p.swy),
                     p.w_xy, p.n_x, p.n_y, p.tiles_x, nchunks, bc, b_begin, b_end, static_cast<cx<T>*>(Gt));
  return hipGetLastError();
}

#define PATK_INST(T) template hipError_t launch_interp<T>(const DevPlan&, const void*, void*, int, int, hipStream_t);
PATK_INST(float)
PATK_INST(double)
#undef PATK_INST

}  // namespace patk
