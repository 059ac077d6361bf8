// Batched reconstruction: up to kBatchMax independent problems (each its own
// sensor geometry, trace length and output grid) reconstructed with one
// launch per stage and group of problems. Every stage's work items are the
// blocks of the group's problems (problem after problem); per-problem
// arguments are uploaded once at creation, so a call only enqueues eight
// kernels per group.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "kernels_common.hpp"
#include "pat_nufft.h"
#include "plan_internal.hpp"

using namespace patint;

namespace {
constexpr int kStages = 7;  // temporal, spread, fft x, fft y, gather + inverse x, inverse y, c2r z
// default persistent grid: 64 work-groups per CU of a 256-CU MI355X, each
// looping over the work items after loading the group's arguments once
// (measured best among 0, 4096, 16384 and 65536 on the 32-problem batch)
constexpr int kPersistentBlocks = 16384;
}

// Problems are run in groups of at most kGroupMax, optionally also bounded by
// a byte budget on their oversampled grids (so that a group's stages could
// hand their intermediate arrays on through the last-level cache). Groups run
// one after another and share one workspace.
struct BatchGroup {
  std::vector<int> members;   // problem indices, ascending grid size
  void* tables = nullptr;     // argument tables and prefix sums
  size_t table_bytes = 0;
  patk::BatchStage st[kStages];
};

struct pat_batch {
  int count = 0;
  int device = 0;
  bool fp64 = false;
  pat_plan* plans[patk::kBatchMax] = {};
  pat_plan_desc alloc_desc{};  // allocator used for the batch's own memory
  std::vector<BatchGroup> groups;
  void* ws = nullptr;          // workspace of the largest group
  size_t ws_bytes = 0;
  size_t group_bytes = 0;
};

namespace {

struct Blob {
  std::vector<unsigned char> bytes;
  size_t add(const void* src, size_t n) {
    const size_t off = align_up(bytes.size());
    bytes.resize(off + n);
    if (n) std::memcpy(bytes.data() + off, src, n);
    return off;
  }
};

void destroy_batch(pat_batch* B) {
  if (!B) return;
  {
    DeviceGuard guard(B->device);
    (void)hipDeviceSynchronize();
    dev_free(B->alloc_desc, B->ws);
    for (auto& g : B->groups) dev_free(B->alloc_desc, g.tables);
  }
  for (int i = 0; i < B->count; ++i) nufft_plan_destroy(B->plans[i]);
  delete B;
}

// Workspace bytes of one problem: A = grid U (all bins) / lateral spectra,
// B = x rows / spectrum, C = band values (each 256-byte aligned).
template <typename T>
void problem_regions(const patk::DevPlan& d, size_t& a, size_t& b, size_t& cc) {
  const size_t c = sizeof(patk::cx<T>);
  const size_t lh = size_t(d.Nz / 2 + 1);
  a = align_up(std::max(size_t(d.nb) * d.n_y * d.n_x * c, size_t(d.Nx) * d.Ny * d.nb * c));
  b = align_up(std::max(size_t(d.nb) * d.Nx * d.n_y * c, size_t(d.Nx) * d.Ny * lh * c));
  cc = align_up(size_t(d.M) * d.nb * c);
}

// Stage tables of one group, with workspace pointers into `ws`.
template <typename T>
pat_status build_group(pat_batch* B, BatchGroup& G, unsigned char* ws, hipStream_t stream) {
  using patk::cx;
  const int P = int(G.members.size());
  const size_t c = sizeof(cx<T>);
  const patk::FftCfg cfg = patk::fft_cfg();
  const patk::FftCfg icfg = patk::inv_cfg();
  std::vector<patk::TemporalBA> a0(P);
  std::vector<patk::SpreadBA> a1(P);
  std::vector<patk::FftXBA> a2(P);
  std::vector<patk::FftYBA> a3(P);
  std::vector<patk::GatherBA> a4(P);
  std::vector<patk::CfftBA> a5(P);
  std::vector<patk::C2rBA> a6(P);
  std::vector<int> pre[kStages];
  for (auto& v : pre) v.assign(P + 1, 0);
  size_t lds[kStages] = {};
  const int kFft = patk::kFftMaxV * cfg.threads;
  size_t off = 0;
  for (int p = 0; p < P; ++p) {
    const patk::DevPlan& d = B->plans[G.members[p]]->dp;
    size_t ra, rb, rc;
    problem_regions<T>(d, ra, rb, rc);
    void* A = ws + off;
    void* Bw = ws + off + ra;
    void* C = ws + off + ra + rb;
    off += ra + rb + rc;
    const int Lh = d.Nz / 2 + 1;
    if (d.n_t > patk::kFftMaxV * 512) return PAT_ERR_UNSUPPORTED;
    // stage 0: temporal FFT, one block per sensor pair
    a0[p] = patk::TemporalBA{d.hw, d.deap, patk::as_view(d.f_nt), d.M, d.Nt, d.n0, d.b_lo, d.nb, C};
    pre[0][p + 1] = (d.M + 1) / 2;
    lds[0] = std::max(lds[0], size_t(patk::temporal_lds_slots(d.n_t)) * c);
    // stage 1: spread, all bins in one round
    const int nchunks = (d.nb + 15) / 16;
    a1[p] = patk::SpreadBA{C, d.slot_off, d.slot_sens, d.slot_w, d.slot_k, d.nb, d.n_x, d.n_y, d.tiles_x, nchunks, A};
    pre[1][p + 1] = d.tiles_x * d.patches_y * ((nchunks + patk::kSpreadGroups - 1) / patk::kSpreadGroups);
    // stage 2: FFT along x
    const int rows = patk::fft_batch<T>(d.n_x, cfg.threads, cfg.cap);
    if (rows * d.n_x > kFft || rows * d.Nx > kFft) return PAT_ERR_UNSUPPORTED;
    const int gx2 = (d.n_y + rows - 1) / rows;
    a2[p] = patk::FftXBA{A, patk::as_view(d.f_nx), d.n_y, d.Nx, rows, gx2, Bw, d.jrange ? d.brange : nullptr};
    pre[2][p + 1] = gx2 * d.nb;
    lds[2] = std::max(lds[2], (size_t(rows) * patk::lseq(d.n_x) + d.n_x) * c);
    // stage 3: FFT along y with deconvolution
    const int bins = patk::fft_batch<T>(d.n_y, cfg.threads, cfg.cap);
    if (bins * d.n_y > kFft || bins * d.Ny > kFft) return PAT_ERR_UNSUPPORTED;
    const int gx3 = (d.nb + bins - 1) / bins;
    const bool listed = d.ylist && d.ylist_n > 0 && d.jrange;
    a3[p] = patk::FftYBA{Bw, d.dcx, d.dcy, patk::as_view(d.f_ny), d.nb, d.Nx, d.Ny, bins, gx3, A, d.jrange,
                         listed ? d.ylist : nullptr};
    pre[3][p + 1] = listed ? d.ylist_n : gx3 * d.Nx;
    lds[3] = std::max(lds[3], (size_t(bins) * patk::lseq(d.n_y) + d.n_y) * c);
    // stage 4: temporal interpolation and weight (image-ready spectrum) fused
    // with the inverse transform along x
    const int lcx = patk::fft_batch<T>(d.Nx, icfg.threads, patk::kGatherCap);
    const int gx5 = (Lh + lcx - 1) / lcx;
    int wt_ct = 0;
    for (int t : patk::kBatchTaps)
      if (d.w_t == t && d.w_t * (d.hdeg + 1) <= patk::kMaxTapCoefs) wt_ct = t;
    a4[p] = patk::GatherBA{A, d.hcoef, d.nb, d.b_lo, d.Nx, d.Ny, d.Nz, d.w_t, d.hdeg, wt_ct, 0,
                           d.s_per_k, d.kxu, d.kyu, d.kzu, d.two_c, d.n0_over_nt, d.inv_vol, Bw,
                           patk::as_view(d.f_Nx), lcx, gx5};
    pre[4][p + 1] = gx5 * d.Ny;
    lds[4] = std::max(lds[4], (size_t(lcx) * patk::lseq(d.Nx) + d.Nx) * c);
    // stage 5: inverse transform along y (in place on the spectrum)
    const int lcy = patk::fft_batch<T>(d.Ny, icfg.threads, icfg.cap);
    const int gx6 = (Lh + lcy - 1) / lcy;
    a5[p] = patk::CfftBA{Bw, patk::as_view(d.f_Ny), d.Ny, Lh, lcy, gx6};
    pre[5][p + 1] = gx6 * d.Nx;
    lds[5] = std::max(lds[5], (size_t(lcy) * patk::lseq(d.Ny) + d.Ny) * c);
    // stage 6: complex-to-real along z into the caller's image
    const int rz = patk::fft_batch<T>(d.Nz, icfg.threads, icfg.cap);
    const long long nrows = (long long)d.Nx * d.Ny;
    a6[p] = patk::C2rBA{Bw, patk::as_view(d.f_Nz), nrows, rz};
    pre[6][p + 1] = int((nrows + rz - 1) / rz);
    if ((rz + 1) / 2 * (d.Nz / 2 + 1) > patk::kC2rStage * icfg.threads) return PAT_ERR_UNSUPPORTED;
    lds[6] = std::max(lds[6], size_t(patk::c2r_lds_slots(rz, d.Nz)) * c);
  }
  for (auto& v : pre) {
    for (int p = 0; p < P; ++p) {
      const long long next = (long long)v[p] + v[p + 1];
      if (next > 0x7fffffffLL) return PAT_ERR_UNSUPPORTED;
      v[p + 1] = int(next);
    }
  }
  Blob blob;
  size_t oa[kStages], op[kStages];
  oa[0] = blob.add(a0.data(), a0.size() * sizeof(a0[0]));
  oa[1] = blob.add(a1.data(), a1.size() * sizeof(a1[0]));
  oa[2] = blob.add(a2.data(), a2.size() * sizeof(a2[0]));
  oa[3] = blob.add(a3.data(), a3.size() * sizeof(a3[0]));
  oa[4] = blob.add(a4.data(), a4.size() * sizeof(a4[0]));
  oa[5] = blob.add(a5.data(), a5.size() * sizeof(a5[0]));
  oa[6] = blob.add(a6.data(), a6.size() * sizeof(a6[0]));
  for (int i = 0; i < kStages; ++i) op[i] = blob.add(pre[i].data(), pre[i].size() * sizeof(int));
  G.table_bytes = align_up(blob.bytes.size());
  G.tables = dev_alloc(B->alloc_desc, G.table_bytes);
  if (!G.tables) return PAT_ERR_ALLOC;
  if (hipMemcpyAsync(G.tables, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    (void)hipGetLastError();
    return PAT_ERR_HIP;
  }
  unsigned char* tb = static_cast<unsigned char*>(G.tables);
  const bool kahan = B->plans[0]->dp.kahan;
  for (int i = 0; i < kStages; ++i) {
    G.st[i].args = tb + oa[i];
    G.st[i].prefix = reinterpret_cast<const int*>(tb + op[i]);
    G.st[i].nprob = P;
    G.st[i].total = pre[i][P];
    G.st[i].lds = lds[i];
    G.st[i].grid = kPersistentBlocks;
    G.st[i].kahan = kahan;
  }
  return PAT_OK;
}

template <typename T>
pat_status build_batch(pat_batch* B, hipStream_t stream) {
  const int P = B->count;
  // group by the oversampled grid's size (the array handed from the spread to the x-FFT)
  std::vector<size_t> grid(P), total(P);
  for (int p = 0; p < P; ++p) {
    size_t a, b, c;
    problem_regions<T>(B->plans[p]->dp, a, b, c);
    const patk::DevPlan& d = B->plans[p]->dp;
    grid[p] = size_t(d.nb) * d.n_y * d.n_x * sizeof(patk::cx<T>);
    total[p] = a + b + c;
  }
  std::vector<int> order(P);
  for (int p = 0; p < P; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return grid[x] < grid[y]; });
  B->groups.clear();
  size_t sum = 0;
  for (int p : order) {
    if (B->groups.empty() || int(B->groups.back().members.size()) == patk::kGroupMax ||
        (sum + grid[p] > B->group_bytes && !B->groups.back().members.empty())) {
      B->groups.emplace_back();
      sum = 0;
    }
    B->groups.back().members.push_back(p);
    sum += grid[p];
  }
  size_t ws = 0;
  for (auto& g : B->groups) {
    size_t t = 0;
    for (int p : g.members) t += total[p];
    ws = std::max(ws, t);
  }
  B->ws_bytes = ws;
  B->ws = dev_alloc(B->alloc_desc, ws);
  if (!B->ws) return PAT_ERR_ALLOC;
  for (auto& g : B->groups) {
    const pat_status st = build_group<T>(B, g, static_cast<unsigned char*>(B->ws), stream);
    if (st != PAT_OK) return st;
  }
  return PAT_OK;
}

template <typename T>
pat_status run_batch(pat_batch* B, const void* const* g, void* const* f, hipStream_t s) {
  for (const BatchGroup& G : B->groups) {
    patk::BatchIO io{};
    for (size_t i = 0; i < G.members.size(); ++i) {
      io.in[i] = g[G.members[i]];
      io.out[i] = f[G.members[i]];
    }
    hipError_t e;
    if ((e = patk::launch_temporal_batch<T>(G.st[0], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_spread_batch<T>(G.st[1], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_fft_x_batch<T>(G.st[2], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_fft_y_batch<T>(G.st[3], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_gather_batch<T>(G.st[4], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_cfft_y_inv_batch<T>(G.st[5], io, s)) != hipSuccess) return to_status(e);
    if ((e = patk::launch_c2r_z_batch<T>(G.st[6], io, s)) != hipSuccess) return to_status(e);
  }
  return PAT_OK;
}

}  // namespace

extern "C" {

pat_status pat_batch_create(const pat_plan_desc* descs, int32_t count, size_t group_bytes, void* stream,
                            pat_batch** out) {
  if (!out) return PAT_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!descs || count < 1 || count > patk::kBatchMax) return PAT_ERR_INVALID_ARGUMENT;
  for (int i = 1; i < count; ++i) {
    const bool fp64_i = descs[i].precision == PAT_FP64, fp64_0 = descs[0].precision == PAT_FP64;
    if (fp64_i != fp64_0 || (descs[i].precision == PAT_FP32_KAHAN) != (descs[0].precision == PAT_FP32_KAHAN))
      return PAT_ERR_INVALID_ARGUMENT;
  }
  pat_batch* B = new (std::nothrow) pat_batch();
  if (!B) return PAT_ERR_ALLOC;
  if (hipGetDevice(&B->device) != hipSuccess) {
    (void)hipGetLastError();
    delete B;
    return PAT_ERR_HIP;
  }
  B->alloc_desc = descs[0];
  B->alloc_desc.sensor_xy = nullptr;
  B->alloc_desc.sensor_h = nullptr;
  B->fp64 = descs[0].precision == PAT_FP64;
  B->group_bytes = group_bytes ? group_bytes : SIZE_MAX;
  for (int i = 0; i < count; ++i) {
    pat_status st = nufft_plan(&descs[i], stream, &B->plans[i]);
    if (st != PAT_OK) {
      destroy_batch(B);
      return st;
    }
    B->count = i + 1;
  }
  const pat_status st = B->fp64 ? build_batch<double>(B, static_cast<hipStream_t>(stream))
                                : build_batch<float>(B, static_cast<hipStream_t>(stream));
  if (st != PAT_OK) {
    destroy_batch(B);
    return st;
  }
  *out = B;
  return PAT_OK;
}

pat_status pat_batch_get_plan(const pat_batch* B, int32_t index, const pat_plan** plan) {
  if (!B || !plan || index < 0 || index >= B->count) return PAT_ERR_INVALID_ARGUMENT;
  *plan = B->plans[index];
  return PAT_OK;
}

pat_status pat_batch_set_grid(pat_batch* B, int32_t blocks) {
  if (!B || blocks < 0) return PAT_ERR_INVALID_ARGUMENT;
  for (auto& g : B->groups)
    for (auto& s : g.st) s.grid = blocks;
  return PAT_OK;
}

pat_status pat_batch_groups(const pat_batch* B, int32_t* groups) {
  if (!B || !groups) return PAT_ERR_INVALID_ARGUMENT;
  *groups = int32_t(B->groups.size());
  return PAT_OK;
}

pat_status pat_batch_reconstruct(pat_batch* B, const void* const* g, void* const* f, void* stream) {
  if (!B || !g || !f) return PAT_ERR_INVALID_ARGUMENT;
  for (int p = 0; p < B->count; ++p)
    if (!g[p] || !f[p]) return PAT_ERR_INVALID_ARGUMENT;
  DeviceGuard guard(B->device);
  if (!guard.ok) return PAT_ERR_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return B->fp64 ? run_batch<double>(B, g, f, s) : run_batch<float>(B, g, f, s);
}

pat_status pat_batch_destroy(pat_batch* B) {
  destroy_batch(B);
  return PAT_OK;
}

}  // extern "C"
