/*
 * pat_nufft.h -- C ABI of the MI355X (gfx950) NEDNER-NUFFT library for planar
 * photoacoustic reconstruction.
 *
 * Problem (Schmid, Glatz, Zabihian, Liu, Drexler, Scherzer, "Non-Equispaced
 * Grid Sampling in Photoacoustics with a Non-Uniform FFT", Section 2):
 * pressure traces g[m][n] are recorded at M sensors x_m = (x_m, y_m) on the
 * plane z = 0 (not necessarily equispaced, each with detector area h_m,
 * sum h_m = X*Y) at times t_n = n*dt. The initial pressure f on the cube
 * [-X/2,X/2) x [-Y/2,Y/2) x [0,Z) follows from the exact Fourier inversion
 * (Section 2, eq. exact), discretised over non-equispaced sensors
 * (Section 2, eq. disc_rec):
 *
 *   F(K) = W(K) * sum_n e^{-i omega(K) t_n} sum_m h_m dt g[m][n] e^{-i(Kx x_m + Ky y_m)}
 *   omega(K) = c sign(Kz) |K|,  W(K) = 2 c |Kz| / |K|   (W = 0 on Kz = 0)
 *   f(x_a, y_b, z_e) = 1/(XYZ) sum_K F(K) e^{i(Kx x_a + Ky y_b + Kz z_e)}
 *
 * on the lattice Kx = 2 pi j/X, Ky = 2 pi k/Y, Kz = 2 pi l/Z with
 * j in [-Nx/2, Nx/2), k in [-Ny/2, Ny/2), l in [-Nz/2, Nz/2); the planes
 * j = -Nx/2, k = -Ny/2, l = -Nz/2 are set to zero. The output voxels are
 * x_a = (a - Nx/2) X/Nx, y_b = (b - Ny/2) Y/Ny, z_e = e Z/Nz.
 *
 * The library evaluates this with the NEDNER-NUFFT of Section 3: a
 * non-equispaced-range NUFFT in time (eqs. NUDFT1, NER_NUFFT, PSI), a
 * non-equispaced-data NUFFT over the sensor plane (eqs. NUDFT2, NED_NUFFT)
 * and an equispaced inverse FFT, with precomputed window tables
 * (Section 5.2: precomputing the window values for a fixed discretisation).
 * The result approximates the sum above within the window error for the
 * chosen oversampling and width.
 *
 * Memory and execution model
 *  - All data pointers passed to pat_reconstruct / pat_spectrum /
 *    pat_forward / pat_adjoint / pat_forward_dxy are DEVICE pointers on the device that was
 *    current when the plan was created. The plan descriptor's sensor arrays
 *    are HOST pointers; the plan copies them.
 *  - Element type: float for PAT_FP32 and PAT_FP32_KAHAN, double for PAT_FP64.
 *    Complex values are (re, im) pairs of that type.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream). Every
 *    compute call only enqueues work on it: no host synchronisation and no
 *    device allocation, so calls can be captured into a HIP graph.
 *  - The caller owns g, f, fhat, the workspace and the stream. The plan owns
 *    its device tables (allocated through the descriptor's callbacks, or
 *    hipMalloc when they are NULL) and frees them in nufft_plan_destroy.
 *  - A plan is immutable after creation; concurrent calls on one plan are
 *    allowed when each uses its own workspace (timing, when enabled, is not
 *    thread-safe).
 *  - Errors are returned as status codes; nothing throws across the ABI.
 *    Argument validation happens before anything is enqueued, so a call that
 *    fails validation leaves its outputs untouched. NaN inputs propagate.
 */
#ifndef PAT_NUFFT_H
#define PAT_NUFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PAT_OK = 0,
  PAT_ERR_INVALID_ARGUMENT = 1, /* NULL pointer, bad size, sensor outside the plane, ... */
  PAT_ERR_UNSUPPORTED = 2,      /* size the FFTs or kernels cannot represent */
  PAT_ERR_ALLOC = 3,            /* device allocation (or the alloc callback) failed */
  PAT_ERR_HIP = 4,              /* a HIP runtime call or kernel launch failed */
  PAT_ERR_NOT_IMPLEMENTED = 5,
  PAT_ERR_WORKSPACE_TOO_LARGE = 6 /* pat_reconstruct_noalloc: the plan's workspace exceeds
                                     PAT_NOALLOC_SCRATCH_BYTES */
} pat_status;

typedef enum {
  PAT_FP64 = 0,       /* double data, double tables: the plain comparison form */
  PAT_FP32 = 1,       /* float data and arithmetic; tables and omega(K) map computed in double */
  PAT_FP32_KAHAN = 2  /* as PAT_FP32 with compensated (Kahan) summation in the spread */
} pat_precision;

/* Window Psi of Section 3.1 (eq. NUFFT1): compactly supported, positive on
 * the band, with an analytic or quadrature Fourier transform. */
typedef enum {
  PAT_KERNEL_GAUSSIAN = 0,       /* truncated Gaussian (Greengard-Lee width rule) */
  PAT_KERNEL_KAISER_BESSEL = 1   /* Kaiser-Bessel, the window named in Section 3.1 */
} pat_kernel;

/* Temporal interpolation at omega(K) (the NER step, Section 3.1). */
typedef enum {
  PAT_INTERP_WINDOW = 0,  /* NER-NUFFT: deapodised, centred FFT and the window's width_t taps */
  PAT_INTERP_LINEAR = 1   /* comparison baseline of Section 5.1 (Table 1): zeros appended after the
                             trace, FFT of length smooth(sigma_t*Nt), linear interpolation between the
                             two nearest bins; width_t is ignored and sigma_t may be 1 */
} pat_temporal_interp;

typedef struct pat_plan_desc {
  int32_t n_sensors;         /* M >= 1 */
  int32_t n_t;               /* Nt >= 2, samples per trace */
  double dt;                 /* sampling step in s, > 0 */
  double c;                  /* speed of sound in m/s, > 0 */
  const double* sensor_xy;   /* HOST [M][2] sensor positions in metres, plane-centred;
                                each must satisfy -X/2 <= x < X/2 and -Y/2 <= y < Y/2 */
  const double* sensor_h;    /* HOST [M] detector areas in m^2 (sum = X*Y), or NULL for X*Y/M */
  int32_t nx, ny, nz;        /* output grid, each even and >= 4 */
  double lx, ly, lz;         /* extents X, Y, Z in metres, > 0 */
  double sigma_xy;           /* lateral oversampling factor, >= 1.1 (grid = smooth(sigma*N)) */
  int32_t width_xy;          /* lateral window footprint w in grid points, even, 2..16 */
  double sigma_t;            /* temporal oversampling factor, >= 1.1 (>= 1.0 for PAT_INTERP_LINEAR); a
                                minimum: short traces get a longer FFT when the band of bins the
                                interpolation reads needs it (see pat_plan_info.nt_over) */
  int32_t width_t;           /* temporal window footprint, even, 2..16 */
  pat_kernel kernel;
  pat_precision precision;
  pat_temporal_interp temporal_interp;
  /* Optional device allocator (e.g. a framework's caching allocator). Both
   * NULL: the library uses hipMalloc/hipFree. alloc must return memory on the
   * current device aligned to at least 256 bytes, or NULL on failure. */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* alloc_ctx;
} pat_plan_desc;

typedef struct pat_plan pat_plan;

/* Sizes the plan derived; filled by pat_plan_get_info. */
typedef struct pat_plan_info {
  int32_t nx_over, ny_over;  /* oversampled lateral grid: the smallest even 2,3,5-smooth lengths
                                >= max(sigma_xy * n, width_xy) */
  int32_t nt_over;           /* oversampled temporal FFT length */
  int32_t band_lo;           /* first oversampled temporal bin kept (may be < 0) */
  int32_t band_bins;         /* number of temporal bins kept */
  int32_t time_origin;       /* centring offset n0 = Nt/2 of the temporal window */
  int32_t element_bytes;     /* 4 or 8 */
  int32_t spread_tiles;      /* 16 x 16 tiles of the oversampled lateral grid */
  int64_t spread_pairs;      /* (sensor, patch) incidences: footprints meeting each 16 x 4 patch */
  size_t workspace_bytes;
  size_t table_bytes;        /* device bytes owned by the plan */
  int32_t chunk_bins;        /* temporal bins per spread / x-FFT round */
  int32_t rounds;            /* spread / x-FFT rounds per call */
  double deconv_range_xy;    /* largest / smallest lateral deconvolution factor over the kept modes */
  double deconv_range_t;     /* the same for the temporal deapodisation */
  int32_t forward_fused;     /* 1: the forward model's x-FFT and interpolation to the sensors run as one
                                kernel with no grid buffer (oversampled x length <= 1024 and a strip of
                                16 + width_xy - 1 grid rows fits the work-group LDS); 0: two kernels in
                                rounds of chunk_bins bins */
  int32_t pad0;
  int64_t spread_slots;      /* packed slots of the single-problem spread: groups of up to 4 sensors whose
                                footprints share no point of a 16 x 4 patch of the oversampled grid */
  int64_t band_pairs;        /* (x-mode, band bin) pairs inside the per-x-mode ranges of bins the temporal
                                interpolation reads (at most Nx * band_bins): the pairs the lateral FFT along
                                y transforms and the interpolation reads from; the others are skipped */
} pat_plan_info;

/* Fill `desc` with defaults: sigma 2, width 8, Kaiser-Bessel, FP32, window
 * interpolation, NULL pointers, zero sizes. Returns PAT_ERR_INVALID_ARGUMENT if desc is NULL. */
pat_status pat_plan_desc_init(pat_plan_desc* desc);

/* Build a plan for one sensor geometry and output grid (the precomputation
 * of window tables of Section 5.2). Validates the descriptor, computes in
 * double precision on the host each sensor's oversampled-grid coordinates
 * and window weights, the spread tile lists, the deconvolution and
 * deapodisation vectors and the FFT twiddles, and copies them to the device
 * with hipMemcpyAsync on `stream` (hipStream_t) followed by a stream
 * synchronisation. On success *out owns the plan; on failure *out is NULL.
 * PAT_ERR_UNSUPPORTED also when the lattice's largest |omega| dt is so close
 * to or beyond pi that no temporal FFT up to 8192 points holds the band, and
 * for FP32 plans whose deconvolution dynamic range exceeds 1e4 (oversampling
 * near 1 with wide windows: FP32 rounding would be amplified beyond use; the
 * FP64 form accepts them). */
pat_status nufft_plan(const pat_plan_desc* desc, void* stream, pat_plan** out);

/* Workspace bytes every compute call on this plan needs (>= 256-byte aligned). */
pat_status nufft_plan_workspace_size(const pat_plan* plan, size_t* bytes);

pat_status pat_plan_get_info(const pat_plan* plan, pat_plan_info* info);

/* Release the plan and its device tables. NULL is accepted and ignored.
 * Synchronises the device before freeing. */
pat_status nufft_plan_destroy(pat_plan* plan);

/* f = R g: reconstruction (Section 2, eq. disc_rec; Section 3, NEDNER steps).
 * g: DEVICE [M][Nt] real, one trace per sensor in descriptor order.
 * f: DEVICE [Nx][Ny][Nz] real, depth-contiguous; overwritten.
 * workspace: DEVICE, nufft_plan_workspace_size bytes, 256-byte aligned.
 * g, f and workspace must not overlap. */
pat_status pat_reconstruct(pat_plan* plan, const void* g, void* f, void* workspace, void* stream);

/* fhat = F: the weighted spectrum before the inverse transform (the Fourier
 * coefficients of f that eq. disc_rec approximates), as the non-negative
 * half along z: DEVICE complex [Nx][Ny][Nz/2+1] indexed [j mod Nx][k mod Ny][l],
 * l = 0..Nz/2; the l = 0, l = Nz/2, j = -Nx/2 and k = -Ny/2 entries are 0.
 * F(-K) = conj F(K) gives the rest. */
pat_status pat_spectrum(pat_plan* plan, const void* g, void* fhat, void* workspace, void* stream);

/* g = A f: the forward model on the reconstruction's Fourier lattice. The
 * image f launches the free-space wave of Section 2 (zero initial velocity)
 * written as a Fourier series with depth period Z:
 *
 *   D(K) = dV sum_r f(r) e^{-i K.r},  dV = (X/Nx)(Y/Ny)(Z/Nz),
 *   g[m][n] = 1/(XYZ) sum_K D(K) e^{i(Kx x_m + Ky y_m)} cos(c|K| t_n),
 *
 * K over the lattice minus the planes j = -Nx/2, k = -Ny/2, l = -Nz/2. A
 * source at depth z also arrives from z - Z; pad the depth so that those
 * arrivals come after the last sample. Evaluated with the NUFFT steps of the
 * reconstruction transposed (type-2 interpolation to the sensors), within
 * the window error of the plan's settings; the sensor areas h_m are not used.
 * f: DEVICE [Nx][Ny][Nz] real (as pat_reconstruct's output); g: DEVICE [M][Nt]
 * real, overwritten. Returns PAT_ERR_UNSUPPORTED if the per-column LDS of the
 * temporal step (Nz/2 * (4 + (2 + width_t) * element size) bytes) exceeds the
 * device limit. */
pat_status pat_forward(pat_plan* plan, const void* f, void* g, void* workspace, void* stream);

/* f = A* g: the adjoint of pat_forward for the plain Euclidean inner products
 * sum_{m,n} g g' and sum_r f f'. It is the reconstruction's pipeline with unit
 * trace weights (no h_m dt) and the weight W replaced by the constant dV with
 * e^{-i omega t} averaged over both signs of Kz, i.e. cos(c|K| t), on every
 * l including l = 0:
 *   f(r) = 1/(XYZ) sum_K dV sum_n cos(c|K| t_n) sum_m g[m][n] e^{-i(Kx x_m + Ky y_m)} e^{i K.r}.
 * The device kernels of pat_forward are the exact transposes of these, so
 * <A f, g> = <f, A* g> holds to rounding. Layouts as pat_reconstruct. */
pat_status pat_adjoint(pat_plan* plan, const void* g, void* f, void* workspace, void* stream);

/* g = d(A f)/d(x_m) (axis 0) or d(A f)/d(y_m) (axis 1): each trace
 * differentiated with respect to its own sensor's position, i.e. pat_forward
 * with i Kx (i Ky) in front of every lattice term. The gradient of a loss
 * L(A f) with respect to sensor m's x is sum_n dL/dg[m][n] * g[m][n]. Layouts
 * and errors as pat_forward; PAT_ERR_INVALID_ARGUMENT for another axis. */
pat_status pat_forward_dxy(pat_plan* plan, const void* f, int32_t axis, void* g, void* workspace, void* stream);

/* ------------------------------------------------------------------------
 * Batched reconstruction: count (1..64) independent problems, each with its
 * own descriptor (geometry, trace length, output grid, window settings; all
 * with the same element type), reconstructed with one kernel launch per
 * stage for the whole batch: every stage's work items are the blocks of all
 * problems, so small problems share the device instead of running one after
 * another. Results equal pat_reconstruct's for each problem bit for bit.
 *
 * Problems are run in groups of at most 32 (one group per 32 problems by
 * default). With group_bytes > 0 a group also takes problems, sorted by the
 * size of their oversampled lateral grid, only while their grids together
 * stay within group_bytes (meant for handing each stage's output to the next
 * through the last-level cache; on MI355X this measured slower than one
 * group, so 0, no budget, is the default). Groups run one after another
 * (eight launches each) and share one workspace (the largest group's).
 *
 * pat_batch_create builds one plan per descriptor (as nufft_plan), uploads
 * per-group argument tables and allocates the workspace through descs[0]'s
 * allocator (or hipMalloc), then synchronises `stream`. The batch owns its
 * plans, tables and workspace, so calls on one batch must not overlap in
 * time (they share the workspace).
 * ------------------------------------------------------------------------ */
typedef struct pat_batch pat_batch;

pat_status pat_batch_create(const pat_plan_desc* descs, int32_t count, size_t group_bytes, void* stream,
                            pat_batch** out);

/* Number of problem groups the batch runs (each: eight launches). */
pat_status pat_batch_groups(const pat_batch* batch, int32_t* groups);

/* Plan of problem `index` (read-only, e.g. for pat_plan_get_info). */
pat_status pat_batch_get_plan(const pat_batch* batch, int32_t index, const pat_plan** plan);

/* Grid of the batched launches: blocks > 0 (default 16384) launches at most
 * that many work-groups, each loading the group's arguments into LDS once and
 * looping over the work items (a persistent launch); 0 launches one
 * work-group per work item. Results do not depend on it. */
pat_status pat_batch_set_grid(pat_batch* batch, int32_t blocks);

/* f[p] = R g[p] for every problem p: g and f are HOST arrays of `count`
 * DEVICE pointers with the layouts of pat_reconstruct. Enqueues eight kernels
 * per group on `stream` (no allocation, no synchronisation), so the call can
 * be captured into a HIP graph. Inputs and outputs must not overlap. */
pat_status pat_batch_reconstruct(pat_batch* batch, const void* const* g, void* const* f, void* stream);

/* Synchronises the device, then releases the batch. NULL is ignored. */
pat_status pat_batch_destroy(pat_batch* batch);

/* f = R g, as pat_reconstruct, for callers that cannot allocate device
 * memory when they reconstruct (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): no workspace argument, and the
 * call allocates nothing (no hipMalloc, no allocator callback, no host
 * allocation). The workspace is a fixed array of PAT_NOALLOC_SCRATCH_BYTES
 * bytes inside the library, one per GPU the library runs on, reserved when
 * the library's device code is loaded on that GPU and held until the process
 * ends; its device address is looked up (hipGetSymbolAddress) on the first
 * call on each device. g, f, stream and the result as pat_reconstruct (same
 * kernels, same bits). Returns PAT_ERR_WORKSPACE_TOO_LARGE, before enqueueing
 * anything, when nufft_plan_workspace_size exceeds PAT_NOALLOC_SCRATCH_BYTES
 * (use pat_reconstruct with a caller workspace then). Every call on one GPU
 * uses that GPU's one array: calls that overlap in time on the same GPU
 * (other streams, other threads, other plans) race and give undefined
 * results; serialise them. Nothing in the array needs clearing between
 * calls (every stage writes what the next reads). */
#define PAT_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
pat_status pat_reconstruct_noalloc(pat_plan* plan, const void* g, void* f, void* stream);

/* Per-stage device timing with HIP events recorded on the call's stream.
 * pat_timing_begin(plan, n) creates events for up to n subsequent compute
 * calls (allocation happens here, not in the compute calls). pat_timing_end
 * synchronises on the last event, writes the summed milliseconds of each
 * stage to ms[0..nstage-1] (nstage <= PAT_TIMING_STAGES), the number of
 * recorded calls to *calls, and destroys the events. Stages: 0 temporal FFT,
 * 1 lateral spread, 2 lateral FFT along x, 3 lateral FFT along y with
 * deconvolution, 4 temporal interpolation and weight fused with the inverse
 * FFT along x (pat_spectrum: the interpolation alone), 5 the inverse FFT's
 * y and z passes (the spread and x-FFT run in rounds over bins; their rounds
 * are summed). Calls
 * of pat_forward and pat_forward_dxy add each kernel's time to the stage it
 * transposes (5: forward 3-D FFT, 4: transposed interpolation, 3 and 2:
 * transposed lateral FFTs, 1: interpolation to the sensors, 0: transposed
 * temporal FFT); with pat_plan_info.forward_fused the fused x-FFT and
 * interpolation kernel counts under stage 1 and stage 2 reads 0. */
#define PAT_TIMING_STAGES 6
pat_status pat_timing_begin(pat_plan* plan, int32_t max_calls);
/* The same for the stages in stage_mask only (bit s = stage s, nonzero,
 * below 1 << PAT_TIMING_STAGES): events are recorded only at the two ends
 * of those stages, so the other kernels run back to back as in an untimed
 * call (every event between two kernels costs a few microseconds), and
 * pat_timing_end reports 0 for the other stages. pat_timing_begin is this
 * call with every stage's bit set. PAT_ERR_INVALID_ARGUMENT for a mask
 * outside that range. */
pat_status pat_timing_begin_stages(pat_plan* plan, int32_t max_calls, uint32_t stage_mask);
pat_status pat_timing_end(pat_plan* plan, double* ms, int32_t nstage, int32_t* calls);

const char* pat_status_str(pat_status status);

/* Library version string. */
const char* pat_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PAT_NUFFT_H */
