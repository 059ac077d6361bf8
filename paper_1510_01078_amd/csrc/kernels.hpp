// Interface between the host plan code and the gfx950 stage kernels of the
// NEDNER-NUFFT reconstruction (Section 3: a non-equispaced-range NUFFT in
// time, a non-equispaced-data NUFFT over the sensor plane, then an
// equispaced inverse FFT).
//
// Order of the steps on the device. The temporal transform's equispaced part
// (deapodise, zero-pad, FFT) runs first, per sensor; the lateral NUFFT then
// runs once per kept temporal bin; the temporal interpolation at
// omega(K) = c|K| runs last, per lateral mode. This is the paper's
// composition with the two linear maps on different indices applied in the
// other order, which lets the lateral grid be built only for the band of
// temporal bins that the interpolation reads.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace patk {

struct FftPassRaw {
  int R = 0, p = 0, nbf = 0, twstep = 0;
  uint32_t m_nbf = 0, m_p = 0;
};

struct FftRaw {
  int n = 0;
  int npass = 0;
  FftPassRaw pass[12];           // host copy
  const void* dpass = nullptr;   // device copy of pass[0..npass)
  const void* tw = nullptr;      // device, n complex entries exp(-2 pi i t/n)
};

// Everything a launch needs, as plain values and device pointers.
struct DevPlan {
  int M = 0, Nt = 0, Nx = 0, Ny = 0, Nz = 0;
  int n_x = 0, n_y = 0, n_t = 0, n0 = 0, b_lo = 0, nb = 0;
  int w_xy = 0, w_t = 0, hdeg = 0;
  int tiles_x = 0, tiles_y = 0;
  int chunk_bins = 0;          // bins per spread / x-FFT round (the grid buffer holds this many)
  bool kahan = false;
  double s_per_k = 0.0;        // c*dt*n_t/(2 pi): oversampled bin per unit |K|
  double kxu = 0, kyu = 0, kzu = 0;  // 2 pi/X, 2 pi/Y, 2 pi/Z
  double two_c = 0.0;          // 2c of W(K) = 2c|Kz|/|K|
  double n0_over_nt = 0.0;     // centring phase factor n0/n_t
  double inv_vol = 0.0;        // 1/(XYZ)
  double adj_scale = 0.0;      // dV/(2V) = 1/(2 Nx Ny Nz): the adjoint's constant weight with the 1/V of the inverse
  // device tables (element type T unless int)
  const void* hw = nullptr;       // [M]   h_m*dt
  const void* deap = nullptr;     // [Nt]  1/phihat_t((n - n0)/n_t)
  const int* sbx = nullptr;       // [M]   first x grid point of the footprint (mod n_x)
  const int* sby = nullptr;       // [M]
  const void* swx = nullptr;      // [M][w] x weights
  const void* swy = nullptr;      // [M][w]
  const int* slot_off = nullptr;  // [tiles_x*patches_y+1] packed slots of each 16 x kPatchRows patch (CSR)
  const int* slot_sens = nullptr; // [slots][kSlotK] sensor ids of each slot, -1 for an empty place
  const void* slot_w = nullptr;   // [slots][64] each lane's weight wx*wy (0 where no sensor covers it)
  const unsigned* slot_k = nullptr;       // [slots][64] places in their slots of the lane's sensors for the
                                          // kSlotBatch slots from this one on (2 bits each, 0 past the patch)
  int patches_y = 0;
  const int* home_off = nullptr;  // [tiles+1] sensors whose footprint starts in each tile (CSR)
  const int* home_sens = nullptr; // [M]
  int fused_strip = 1;            // home-tile rows per strip of the fused forward kernel (1 or 2)
  const int* jrange = nullptr;    // [Nx][2] first and last band bin the interpolation reads per x-mode,
                                  // in whole groups of the y-FFT's bins; the y-FFT skips the others
  const int* brange = nullptr;    // [nb][2] per band bin the smallest and largest |j| whose range holds it
  const int* ylist = nullptr;     // the y-FFT's work items inside the ranges: jj << 16 | bin group
  int ylist_n = 0;
  const void* dcx = nullptr;      // [Nx] 1/phihat(j/n_x), 0 at j = -Nx/2
  const void* dcy = nullptr;      // [Ny]
  const void* hcoef = nullptr;    // [w_t][hdeg+1] temporal tap polynomials
  FftRaw f_nt, f_nx, f_ny, f_Nx, f_Ny, f_Nz;
};

constexpr int kSpreadTile = 16;  // spread tile edge (grid points)
constexpr int kPatchRows = 4;    // rows of the spread's one-wave patch (16 x 4 grid points)
constexpr int kSlotK = 4;        // sensors per packed spread slot
constexpr int kSpreadGroups = 2; // spread bin groups (16 bins each) per work-group
constexpr int kSlotBatch = 8;    // spread slots staged per round (their places fit one 32-bit word)

// Stage launchers; T = float or double. Buffers are device pointers.
//
// Reconstruction and adjoint: temporal -> spread -> fft_x -> fft_y -> gather
// -> inverse. Forward model (the exact transpose of the adjoint's stages, in
// reverse order): forward3d -> scatter -> fft_y_t -> fft_x_t -> interp ->
// temporal_t.

// weighted = true: traces scaled by h_m dt (reconstruction); false: unit
// weights (adjoint of the forward model).
template <typename T>
hipError_t launch_temporal(const DevPlan& p, const T* g, void* Gt, bool weighted, hipStream_t s);
// Bins [b_begin, b_end) of the band: U holds only those bins (U[b - b_begin]),
// V all bins.
template <typename T>
hipError_t launch_spread(const DevPlan& p, const void* Gt, void* U, int b_begin, int b_end, hipStream_t s);
template <typename T>
hipError_t launch_fft_x(const DevPlan& p, const void* U, void* V, int b_begin, int b_end, hipStream_t s);
template <typename T>
hipError_t launch_fft_y(const DevPlan& p, const void* V, void* Gh, hipStream_t s);
// GATHER_PHYSICAL: F(K) as defined (sign (-1)^(j+k), no 1/V); GATHER_IMAGE:
// the image-ready spectrum (-1)^(j+k) F(K) / (XYZ) consumed by
// launch_inverse; GATHER_ADJOINT: the adjoint's image-ready spectrum.
enum { GATHER_IMAGE = 0, GATHER_PHYSICAL = 1, GATHER_ADJOINT = 2 };
template <typename T>
hipError_t launch_gather(const DevPlan& p, const void* Gh, void* Fh, int mode, hipStream_t s);
template <typename T>
hipError_t launch_inverse(const DevPlan& p, void* Fh, T* f, hipStream_t s, bool x_done = false);
// Gather (GATHER_IMAGE or GATHER_ADJOINT) fused with the inverse transform
// along x: leaves what launch_gather + the x pass of launch_inverse would;
// finish with launch_inverse(..., x_done = true).
template <typename T>
hipError_t launch_gather_x(const DevPlan& p, const void* Gh, void* F, int mode, hipStream_t s);

// Forward model. f -> Dh (real-to-complex along z, forward FFTs along y, x)
template <typename T>
hipError_t launch_forward3d(const DevPlan& p, const T* f, void* Dh, hipStream_t s);
// Dh -> Gh' (deriv 0: A; 1: d/dx_m; 2: d/dy_m); LDS bytes it needs
template <typename T>
hipError_t launch_scatter(const DevPlan& p, const void* Dh, void* Gh, int deriv, hipStream_t s);
template <typename T>
size_t scatter_lds_bytes(const DevPlan& p);
// Gh'[j][k][b] -> V'[b][j][py]
template <typename T>
hipError_t launch_fft_y_t(const DevPlan& p, const void* Gh, void* V, hipStream_t s);
// V'[b][j][py] -> U'[b - b_begin][py][px] for bins [b_begin, b_end)
template <typename T>
hipError_t launch_fft_x_t(const DevPlan& p, const void* V, void* U, int b_begin, int b_end, hipStream_t s);
// U' (bins [b_begin, b_end)) -> Gt'[m][b] at the sensors
template <typename T>
hipError_t launch_interp(const DevPlan& p, const void* U, void* Gt, int b_begin, int b_end, hipStream_t s);
// k_fft_x_t and k_interp in one kernel over all bins (no grid buffer); usable
// when fused_interp_ok: n_x <= 1024 and the strip of 16 + w - 1 rows fits the
// work-group LDS limit.
template <typename T>
hipError_t launch_fft_x_interp(const DevPlan& p, const void* V, void* Gt, hipStream_t s);
// Static LDS that the fused kernel and the transposed interpolation hold
// beside their dynamic LDS (row and run tables); the plan's fit checks add it.
constexpr size_t kStaticLdsMargin = 512;

// LDS of the fused kernel for a strip of strip_tiles rows of home tiles
template <typename T>
size_t fused_interp_lds(const DevPlan& p, int strip_tiles);
template <typename T>
bool fused_interp_ok(const DevPlan& p, size_t lds_limit);
// Gt' -> g[m][n] (unit weights)
template <typename T>
hipError_t launch_temporal_t(const DevPlan& p, const void* Gt, T* g, hipStream_t s);

// ---------------------------------------------------------------------------
// Batched launches: one launch per stage serves up to kBatchMax problems of
// different sizes. The work items of a stage are the blocks of every
// problem, numbered problem after problem; prefix[p] is the first item of
// problem p (prefix[nprob] = total). Each problem's arguments sit in a device
// table; only the per-call input and output pointers travel in BatchIO (a
// kernel argument), so a batched call allocates and synchronises nothing.
// ---------------------------------------------------------------------------
constexpr int kBatchMax = 64;
constexpr int kGroupMax = 32;  // problems per batched launch

struct BatchIO {
  const void* in[kGroupMax];
  void* out[kGroupMax];
};

struct FftView {  // plain data (it also lives in LDS)
  int n, npass;
  const void* pass;
  const void* tw;
};

struct TemporalBA {
  const void* hw; const void* deap; FftView fd; int M, Nt, n0, b_lo, nb; void* Gt;
};
struct SpreadBA {
  const void* Gt; const int* slot_off; const int* slot_sens; const void* slot_w; const unsigned* slot_k;
  int nb, n_x, n_y, tiles_x, nchunks; void* U;
};
struct FftXBA {
  const void* U; FftView fd; int n_y, Nx, rows, gx; void* V; const int* brange;
};
struct FftYBA {
  const void* V; const void* dcx; const void* dcy; FftView fd; int nb, Nx, Ny, bins, gx; void* Gh;
  const int* jrange;  // per x-mode band range (bin groups outside it are skipped)
  const int* ylist;   // the work items inside the ranges (jj << 16 | bin group), or nullptr: gx * Nx items
};
struct GatherBA {  // the gather fused with the inverse transform along x
  const void* Gh; const void* hcoef; int nb, b_lo, Nx, Ny, Nz, wt, deg;
  int wt_ct, pad;  // compile-time tap count to run (kBatchTaps member equal to wt, else 0: runtime taps)
  double s_per_k, kxu, kyu, kzu, two_c, n0_over_nt, scale; void* Fh;
  FftView fd; int lchunk, gx;  // x transform (length Nx), z modes per group, groups along z
};
struct CfftBA {
  void* F; FftView fd; int Ny, Lh, lchunk, gx;  // Ny is used by the x pass only
};
struct C2rBA {
  const void* F; FftView fd; long long nrows; int rows;
};

// One stage of a batched call: its argument table (one entry per problem),
// prefix sums of work items, the dynamic LDS bytes (maximum over problems)
// and the grid (0: one block per work item; otherwise blocks that loop over
// the work items).
struct BatchStage {
  const void* args = nullptr;
  const int* prefix = nullptr;
  int nprob = 0;
  int total = 0;
  size_t lds = 0;
  int grid = 0;
  bool kahan = false;  // spread with compensated summation
};

// tap counts the batched gather instantiates at compile time (each problem
// runs its own; other counts take the runtime-tap form)
constexpr int kBatchTaps[4] = {6, 8, 10, 12};

// temporal tap polynomials staged in LDS: at most 16 taps of degree <= 24
constexpr int kMaxTapCoefs = 16 * 25;

template <typename T> hipError_t launch_temporal_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_spread_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_fft_x_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_fft_y_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_gather_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_cfft_y_inv_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);
template <typename T> hipError_t launch_c2r_z_batch(const BatchStage& st, const BatchIO& io, hipStream_t s);

}  // namespace patk
