/*
 * rtmi.h -- C ABI of the MI355X (gfx950) emission-absorption ray march.
 *
 * The method is the time-dependent ray tracer of Ray-trax (arXiv 2511.09389), Sec. 2:
 * from each source, N_Omega rays on a Fibonacci (golden-angle) lattice march
 * N_s = ceil(c dt / ds) substeps. At substep k a ray at x_k reads j by trilinear
 * interpolation and kappa from the nearest voxel, applies Eq. (2)
 *     x_{k+1} = x_k + n ds,  tau_{k+1} = tau_k + kappa ds,
 *     I_{k+1} = I_k exp(-kappa ds) + j exp(-tau_k) ds,
 * and deposits the post-attenuation I_{k+1} back onto the grid with the same trilinear
 * weights, scaled by 4 pi / N_Omega. Indexing is clamped to the box: rays that leave it
 * keep marching and deposit on the nearest boundary voxels.
 *
 * Conventions shared by every entry point:
 *  - Maps and fields are DEVICE memory owned by the caller: contiguous float32, C order
 *    [nx][ny][nz] (z fastest). Voxel (a, b, c) sits at grid coordinate (a, b, c), and
 *    source positions are given in these grid coordinates (Appendix A, "source_pos").
 *    The library never frees or retains caller memory beyond the call's stream work.
 *  - Per-source arrays (source_pos, num_rays, substep_cap) and kappa_scale are HOST
 *    memory; they are read during the call and may be reused as soon as it returns.
 *  - All device work is enqueued on `stream` (a hipStream_t; NULL = the default stream).
 *    Calls return without synchronising the stream.
 *  - Output fields are OVERWRITTEN: zeroed, then accumulated, in stream order.
 *  - Directions: the FP64 lattice rounded to binary32, cached per (device, N_Omega) in
 *    device memory the library owns for the life of the process. The first call with a
 *    new N_Omega on a device allocates and uploads that table; call rtmi_prepare() first
 *    to keep later calls free of allocation (e.g. under stream capture).
 *  - Sample points: x_k = fl(src + fl(fl(k ds) n)) in binary32, computed without fused
 *    multiply-add, so that floor/round index decisions are reproducible by an
 *    independent implementation.
 *  - Status: RTMI_OK (0) or a negative RTMI_ERR_* code. Arguments are validated before
 *    any work is enqueued; on error nothing is enqueued and rtmi_last_error() returns a
 *    message for the calling thread. Map contents are not scanned for NaN/Inf.
 *  - Limits: 1 <= nx, ny, nz and nx*ny*nz < 2^31; 1 <= num_rays <= 2^24; N_s <= 2^24.
 */
#ifndef RTMI_H
#define RTMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RTMI_OK = 0,
  RTMI_ERR_INVALID_ARG = -1, /* null pointer, count <= 0, ds <= 0, c < 0 or dt < 0 */
  RTMI_ERR_SHAPE = -2,       /* a grid dimension < 1 or nx*ny*nz >= 2^31 */
  RTMI_ERR_NONFINITE = -3,   /* a scalar argument or source position is NaN or Inf */
  RTMI_ERR_HIP = -4,         /* a HIP runtime call failed (message names it) */
  RTMI_ERR_UNSUPPORTED = -5, /* a combination this build does not implement */
  RTMI_ERR_RANGE = -6        /* N_s or num_rays beyond 2^24 */
};

/* Accumulation modes (rtmi_options.accum_mode). */
enum {
  /* Float32 atomic adds; results agree with the FP64 oracle to the tolerances of the
   * tests, but the last bits depend on the order the hardware performs the adds. */
  RTMI_ACCUM_ATOMIC = 0,
  /* Deposits are rounded to 64-bit fixed point (a power-of-two scale chosen on the
   * device from max|j| and the worst-case sum) and added with integer atomics, so the
   * field is bitwise reproducible from run to run and does not depend on the order of
   * the sources or on scheduling. (Short per-lane partial sums are formed in a fixed
   * order set by the build before rounding.) The worst-case sum uses each source's ray
   * weight times its N_Omega; negative kappa values in the maps widen it by
   * exp(N_s ds max(-kappa)), so the integers cannot wrap. A negative kappa_scale is
   * refused in this mode (RTMI_ERR_INVALID_ARG). */
  RTMI_ACCUM_DETERMINISTIC = 1
};

/* Optional settings; pass NULL for the defaults (all fields zero). */
typedef struct rtmi_options {
  int32_t accum_mode;       /* RTMI_ACCUM_ATOMIC or RTMI_ACCUM_DETERMINISTIC */
  /* Explicit HOST direction table [num_rays][3] (unit vectors, any order) replacing the
   * Fibonacci lattice for every source; then every source must use the same num_rays.
   * Uploaded per call (allocates): a test hook for closed forms and symmetry checks. */
  const float* directions;
  float ray_weight;         /* weight per ray with explicit directions; <= 0: 4 pi/num_rays */
  int32_t path;             /* RTMI_PATH_TILED (default) or RTMI_PATH_DIRECT */
  /* Tiled path: size of a tile work item in chunks (a chunk is one ray's substeps inside
   * one aligned block of 8, for one tile). A tile whose rays bring C chunks is split into
   * ceil(C / tile_item_chunks) work items (at most 64), which separate work-groups take
   * and add atomically. 0 picks 1024. Changes the speed, not the field (in the
   * deterministic mode, not a bit of it). Ignored by the direct path. */
  int32_t tile_item_chunks;
  /* Test hook of the tiled path's stateless calls: > 0 caps each chunk-record buffer at
   * this many records instead of the library's upper bound, so that the overflow report
   * (rtmi_dropped_records) can be exercised. 0: the bound. Plans ignore it (they count
   * their records exactly). */
  int64_t record_capacity;
  /* Tiled path with j and kappa shared by the bins: where the record pass gathers them.
   * 1: a table built per call holding, per voxel, the eight corners of j and of kappa in
   * one 64-byte line (one line per sample; 64 bytes of workspace per voxel). 2: the maps
   * themselves (nine 4-byte loads per sample, no table). 3: a gather pass before the
   * record pass gathers j and kappa tile by tile (the tile's maps staged in LDS) into
   * per-sample rows (8 bytes per ray-substep of workspace instead of the table), which the
   * record pass reads in whole 64-byte pieces. 0 picks the table. Changes the speed, and
   * the field only by rounding (the maps round the interpolation of a sample clamped on a
   * box face differently from the table and the gather pass, also in the deterministic
   * mode). */
  int32_t gather_table;
  /* Tiled path: > 0 caps the sources one record launch (and its tile passes) covers;
   * the sources are then marched in consecutive groups of at most this many, each group's
   * tile passes adding into the field. 0: every source in one launch unless their deposit
   * rows pass 4 GiB. Changes the speed and the workspace, not the field. */
  int32_t sources_per_launch;
  /* Tiled path: > 0 caps the work-groups of the persistent tile pass at this many per
   * compute unit (0: as many as fit, three). A tuning knob: changes the speed only. */
  int32_t tile_groups_per_cu;
} rtmi_options;

/* Execution paths (rtmi_options.path). Both compute the same field.
 *  RTMI_PATH_TILED: two kernels. A record kernel runs each ray's recurrence and writes
 *    the deposit value of every substep to a workspace; a tile kernel then lets each
 *    work-group own a 16^3 block of the output, accumulate the deposits landing in it
 *    in LDS and add it to the field. Workspace: 4 bytes per (ray, substep, bin), plus
 *    64 bytes per voxel (a gather table of j and kappa) when j and kappa are shared by
 *    the bins, plus the chunk records that list each tile's work (8 bytes per chunk of
 *    up to 8 substeps and tile it reaches; sized by an upper bound, 8 tiles per chunk
 *    for step_size <= 0.9, two such buffers when the sources or bins need several
 *    launches), taken from a stream-ordered pool the library owns per device. The
 *    library keeps one such workspace per (device, stream) and reuses it for the next
 *    call on that stream, growing it when a call needs more; it is held until
 *    rtmi_release_workspaces or the process ends. Host threads that call on one stream
 *    must take turns (one call at a time per stream), as they must for any stream-ordered
 *    work that shares memory. During graph capture a call takes its own
 *    stream-ordered allocation instead, which the graph owns. The tile schedules and records, which
 *    depend on the geometry only, are computed on a library-owned stream of the same
 *    device, ordered by events after the caller's earlier work on `stream` and before
 *    the tile passes that read them; the call's results are still ordered on `stream`
 *    like any other enqueued work.
 *  RTMI_PATH_DIRECT: one kernel; each lane sums its ray's consecutive deposits into a
 *    2x2x2 register window and flushes it with global atomics. No workspace. */
enum { RTMI_PATH_TILED = 0, RTMI_PATH_DIRECT = 1 };

/* Message describing the last error on the calling thread ("" if none). */
const char* rtmi_last_error(void);

/* ABI version of this library (major * 100 + minor). */
int32_t rtmi_version(void);

/* N_s = ceil(c dt / ds) (Sec. 2 after Eq. (2)), the quotient taken in binary64 on the
 * binary32 arguments; when cap > 0 the result is min(N_s, cap). Returns N_s >= 0, or a
 * negative RTMI_ERR_* code for ds <= 0, c < 0, dt < 0, non-finite input, or N_s > 2^24. */
int64_t rtmi_num_substeps(float step_size, float radiation_velocity, float time_step,
                          int32_t cap);

/* Fibonacci (golden-angle) lattice of Sec. 2, written to HOST memory host_xyz[n][3] in
 * lattice order: z_i = 1 - (2i+1)/n, r_i = sqrt(1 - z_i^2), phi_i = 2 pi frac(i g) with
 * g = (3 - sqrt(5))/2, n_i = (r_i cos phi_i, r_i sin phi_i, z_i) on array axes (0,1,2),
 * evaluated in binary64 and rounded to binary32. This is the table the march uses. */
int32_t rtmi_fibonacci_directions(int32_t n, float* host_xyz);

/* Build (once) the device direction table for n rays on the current device, so that
 * later calls with this N_Omega allocate nothing. */
int32_t rtmi_prepare(int32_t num_rays);

/* Grow the current device's workspace pool so that tiled calls needing up to `bytes`
 * of workspace allocate nothing from the system (their pool allocations, the first on
 * each stream and those made during graph capture, are then served from memory the pool
 * already holds). */
int32_t rtmi_reserve(int64_t bytes);

/* Chunk records that the tiled path's stateless calls on the current device could not
 * store since the last query (their buffers are sized by an upper bound on the records,
 * see RTMI_PATH_TILED; the tile passes of those calls then missed those deposits). Waits
 * for all work on the device, writes the count to *count and resets it. Returns RTMI_OK
 * when the count is 0, RTMI_ERR_RANGE (with a message) when deposits were dropped, or
 * RTMI_ERR_HIP. Plans never drop records. */
int32_t rtmi_dropped_records(int64_t* count);

/* Free the workspaces that stateless calls keep per stream on the current device (see
 * RTMI_PATH_TILED), after waiting for all work on the device. Call it to return that
 * memory, and before a stream that still had calls pending is destroyed if a stream
 * created later might receive the same handle (a cached workspace is keyed by the
 * handle; reusing it from a new stream while the old stream's work still runs would
 * race). Returns RTMI_OK or RTMI_ERR_HIP. */
int32_t rtmi_release_workspaces(void);

/* The single-source kernel of Sec. 2: advance the field over one dt for one source.
 * Arguments mirror the paper's (j_map, kappa_map, source_pos, num_rays, step_size,
 * radiation_velocity, time_step). source_pos: HOST float[3]. out_field: DEVICE
 * float[nx][ny][nz], overwritten with J = sum over rays of the deposits. */
int32_t rtmi_trace_single(const float* j_map, const float* kappa_map,
                          int32_t nx, int32_t ny, int32_t nz,
                          const float* source_pos, int32_t num_rays, float step_size,
                          float radiation_velocity, float time_step,
                          float* out_field, void* stream);

/* The multi-source routine of Sec. 2 ("loop-and-sum"): out_field = sum over sources of
 * rtmi_trace_single with a shared j_map, each source with its own N_Omega and, if
 * substep_cap is not NULL, its own cap (cap <= 0: none). source_pos: HOST
 * float[n_src][3]; num_rays, substep_cap: HOST int32[n_src]. Work for all sources is
 * one pass over the device; the order of the sum over sources is not specified. */
int32_t rtmi_trace_multi(const float* j_map, const float* kappa_map,
                         int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                         const float* source_pos, const int32_t* num_rays,
                         const int32_t* substep_cap, float step_size,
                         float radiation_velocity, float time_step,
                         float* out_field, void* stream);

/* Frequency bins as a batch axis (Sec. 2, "Frequency-bin agnosticism"): bin b is an
 * independent multi-source problem with emissivity j_b and opacity kappa_b, written to
 * out_fields + b * nx*ny*nz.
 *   j_b     = j_maps + b * j_bin_stride          (stride 0: one j shared by all bins)
 *   kappa_b = kappa_maps + b * kappa_bin_stride  (stride > 0: per-bin maps), or, with
 *             stride 0, kappa_maps * kappa_scale[b] (kappa_scale HOST float[n_bins];
 *             NULL means all ones), the product rounded to binary32.
 * Strides are in elements. opts may be NULL. */
int32_t rtmi_trace_bins(const float* j_maps, int64_t j_bin_stride,
                        const float* kappa_maps, int64_t kappa_bin_stride,
                        const float* kappa_scale, int32_t n_bins,
                        int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                        const float* source_pos, const int32_t* num_rays,
                        const int32_t* substep_cap, float step_size,
                        float radiation_velocity, float time_step,
                        float* out_fields, const rtmi_options* opts, void* stream);

/* For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. The same call as rtmi_trace_bins (same
 * arguments, the same field; in the deterministic mode the same bits), with no
 * allocation of any kind: every buffer the call needs beyond its inputs and outputs (the
 * tiled path's gather table, deposit rows, tile schedules and chunk records, or the
 * deterministic mode's fixed-point field) is carved from one static device array of
 * rtmi_static_scratch_bytes() bytes (384 MiB) that the library holds on each device it
 * runs on until the process ends. The geometry passes run on `stream` itself (no side
 * stream, no events), and kernel timing (rtmi_timing_enable) does not record these calls.
 * Errors, all before anything is enqueued:
 *  - RTMI_ERR_RANGE when the call needs more scratch than the array holds (the message
 *    gives the size it needs; a 128^3 grid with 16 sources x 4096 rays x 256 substeps
 *    fits);
 *  - RTMI_ERR_UNSUPPORTED when a source's N_Omega has no direction table on this device
 *    (call rtmi_prepare(N_Omega) first) or when opts->directions is set (that table is
 *    uploaded per call).
 * Every call on one device shares that device's array and leaves its contents behind
 * (the call clears what must start at zero itself). Calls ordered on one stream are safe;
 * calls that may overlap on one device (concurrent streams, several host threads) race on
 * the array and must be serialised by the caller. */
int32_t rtmi_trace_bins_static(const float* j_maps, int64_t j_bin_stride,
                               const float* kappa_maps, int64_t kappa_bin_stride,
                               const float* kappa_scale, int32_t n_bins,
                               int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                               const float* source_pos, const int32_t* num_rays,
                               const int32_t* substep_cap, float step_size,
                               float radiation_velocity, float time_step,
                               float* out_fields, const rtmi_options* opts, void* stream);

/* Size in bytes of the static scratch of rtmi_trace_bins_static, per device. */
int64_t rtmi_static_scratch_bytes(void);

/* ---- Plans: the batched multi-source, multi-bin march set up once, run many times ----
 *
 * The multi-source routine (Sec. 2, "loop-and-sum") and the frequency bins (Sec. 2,
 * "Frequency-bin agnosticism") as one prepared execution: sources with their own N_Omega
 * and substep caps, times bins, exactly as rtmi_trace_bins computes them (same field, and
 * in the deterministic mode the same bits). Creation validates the geometry, uploads the
 * direction tables, allocates the whole workspace (rtmi_plan_workspace_bytes) and
 * computes the tile schedules and chunk records, which depend on the geometry only (the
 * records are counted first and allocated exactly); it synchronises and may allocate. Execution takes new maps and only enqueues kernels: it allocates nothing,
 * does not synchronise and reads no device data on the host, so it may be captured into
 * a HIP graph and replayed. Executions of one plan share its workspace: they must be
 * ordered on one stream (or otherwise serialised), never run concurrently. A plan
 * belongs to the device current at creation, which must be current when it executes.
 * Tiled path only (opts->path = RTMI_PATH_DIRECT is refused with RTMI_ERR_UNSUPPORTED).
 * Kernel timing (rtmi_timing_enable) must be off while a graph is being captured. */
typedef struct rtmi_plan rtmi_plan;

/* Arguments as rtmi_trace_bins without the maps and field; the host arrays are copied.
 * On success *plan receives the plan, else NULL and a negative RTMI_ERR_* code. */
int32_t rtmi_plan_create(int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                         const float* source_pos, const int32_t* num_rays,
                         const int32_t* substep_cap, int32_t n_bins,
                         int64_t j_bin_stride, int64_t kappa_bin_stride,
                         const float* kappa_scale, float step_size,
                         float radiation_velocity, float time_step,
                         const rtmi_options* opts, rtmi_plan** plan);

/* out_fields [n_bins][nx][ny][nz] (DEVICE, overwritten) from j_maps and kappa_maps
 * (DEVICE, laid out as the bin strides given at creation), on `stream`. */
int32_t rtmi_plan_execute(const rtmi_plan* plan, const float* j_maps,
                          const float* kappa_maps, float* out_fields, void* stream);

/* Device bytes the plan holds. */
int64_t rtmi_plan_workspace_bytes(const rtmi_plan* plan);

/* Frees the plan (NULL is accepted). No execution of it may still be pending. */
int32_t rtmi_plan_destroy(rtmi_plan* plan);

/* ---- Learned surrogate (not part of the paper; the march is its fallback) ----
 *
 * Building blocks of a small 3-D convolutional network that predicts the march's field
 * from its inputs: 3x3x3 "same" convolutions with zero padding over 32 channels, bf16
 * operands on the matrix cores with fp32 accumulation, GELU (error-function form) and
 * residual connections, their gradients, a squared-error loss and an Adam step.
 * Layout: activations channels-last bf16 [n][d][h][w][32] (DEVICE; a channel count
 * below 32 is zero-padded by the caller); weights bf16 [27][32 co][32 ci] with
 * tap = ((dz+1)*3 + (dy+1))*3 + (dx+1), the input read at voxel + (dz, dy, dx); bias fp32
 * [32]. All pointers are DEVICE memory owned by the caller; calls enqueue on `stream`
 * and return RTMI_ERR_* on bad arguments without enqueueing.
 *
 * forward: z = conv(x, w) + bias; y = (gelu ? GELU(z) : z) + residual (bf16, or NULL);
 *   writes y (bf16) and, if z != NULL, z (fp32, for the backward pass). */
int32_t rtmi_conv3d_forward(const void* x, const void* w, const float* bias,
                            const void* residual, int32_t gelu, int32_t n, int32_t d,
                            int32_t h, int32_t w_dim, void* y, float* z, void* stream);

/* backward-data: g = conv^T(dz, w) + residual (fp32, or NULL), i.e.
 *   g[u][ci] = sum_tap sum_co w[tap][co][ci] dz[u - off(tap)][co] + residual[u][ci];
 *   writes g to dh (fp32, or NULL) and g * GELU'(zprev) (or g when zprev is NULL) to
 *   dz_prev (bf16, or NULL). */
int32_t rtmi_conv3d_backward_data(const void* dz, const void* w, const float* residual,
                                  const float* zprev, int32_t n, int32_t d, int32_t h,
                                  int32_t w_dim, float* dh, void* dz_prev, void* stream);

/* backward-weight: dw[tap][co][ci] += sum_v dz[v][co] x[v + off(tap)][ci] and
 *   db[co] += sum_v dz[v][co] (fp32; the caller zeroes them). Needs w_dim a multiple of
 *   16, else RTMI_ERR_UNSUPPORTED. Uses about 110 KB of scratch per compute unit from the
 *   library's stream-ordered pool (per-work-group partial sums, added up in a fixed order,
 *   so the result is the same bits on every call). */
int32_t rtmi_conv3d_backward_weight(const void* x, const void* dz, int32_t n, int32_t d,
                                    int32_t h, int32_t w_dim, float* dw, float* db,
                                    void* stream);

/* Squared error of channel 0 of y (bf16 [n_voxels][32]) against target (fp32
 * [n_voxels]): *loss += scale * sum (y - t)^2, and dz (bf16 [n_voxels][32], overwritten)
 * = its gradient in channel 0, zero in the others. */
int32_t rtmi_mse_loss(const void* y, const float* target, int64_t n_voxels, float scale,
                      void* dz, float* loss, void* stream);

/* Network input of one sample (cells voxels; DEVICE fp32 j, kappa and `cheap`, the march
 * with few rays). First scale_sums (DEVICE fp32 [2]) is reset and scale_sums[0] = sum of
 * cheap^2, giving the sample's scale s = sqrt(scale_sums[0] / cells); then x (bf16
 * [cells][32], overwritten) = ((log kappa - stats[0]) * stats[1], j * stats[2], cheap / s,
 * (log(cheap + stats[5]) - stats[3]) * stats[4], 0, ...). stats: HOST float[6], stats[5] > 0. */
int32_t rtmi_surrogate_features(const float* j, const float* kappa, const float* cheap,
                                int64_t cells, const float* stats, float* scale_sums, void* x,
                                void* stream);

/* Prediction from the network's output y (bf16 [cells][32], channel 0 read) and the
 * scale_sums that rtmi_surrogate_features left: field = max(0, cheap + s y) (fp32,
 * overwritten); check_sums[0] += sum (field - cheap)^2 and check_sums[1] += sum cheap^2
 * (DEVICE fp32 [2]): the relative L2 distance from the cheap field that the fallback test
 * reads. */
int32_t rtmi_surrogate_output(const void* y, const float* cheap, int64_t cells,
                              const float* scale_sums, float* field, float* check_sums,
                              void* stream);

/* One Adam step (bias-corrected, step >= 1) on fp32 weights w with moments m, v and
 * gradient g (count elements each); also writes the bf16 copy w_bf16 when not NULL. */
int32_t rtmi_adam_step(float* w, float* m, float* v, const float* g, void* w_bf16,
                       int64_t count, float lr, float beta1, float beta2, float eps,
                       int32_t step, void* stream);

/* Adjoint of rtmi_trace_multi (Sec. 4: gradients of a loss through the tracer, here
 * written out by the chain rule on Eq. (2) instead of automatic differentiation): given
 * grad_field = dL/dJ (DEVICE float[nx][ny][nz]), writes dL/dj to grad_j and dL/dkappa to
 * grad_kappa (DEVICE float[nx][ny][nz] each, overwritten). The reverse sweep recomputes
 * each ray's forward state from checkpoints kept every few substeps rather than storing
 * trajectories. Per ray and substep k, in reverse order:
 *   g = (4 pi/N) * trilinear gather of G at x_k;  Ibar_{k+1} = g + Ibar_{k+2} a_{k+1};
 *   dL/dj     += trilinear deposit of Ibar_{k+1} E_k ds at x_k;
 *   dL/dkappa[nearest voxel of x_k] += -ds (Ibar_{k+1} I_k a_k + sum_{k'>k} Ibar_{k'+1} j_{k'} E_{k'} ds).
 * Other arguments as rtmi_trace_multi; workspace from the library pool (about 12 bytes
 * per ray-substep plus 8 bytes per voxel). */
int32_t rtmi_trace_vjp(const float* j_map, const float* kappa_map,
                       int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                       const float* source_pos, const int32_t* num_rays,
                       const int32_t* substep_cap, float step_size,
                       float radiation_velocity, float time_step, const float* grad_field,
                       float* grad_j, float* grad_kappa, void* stream);

/* Adjoint of rtmi_trace_bins (Sec. 4, "Gradient-based inversion", with the frequency
 * bins of Sec. 2, "Frequency-bin agnosticism": each bin is an independent problem, so its
 * gradient is the one-bin adjoint above at (j_b, kappa_b), and inputs shared by the bins
 * collect every bin's contribution). grad_fields = dL/dJ_b (DEVICE float[n_bins][cells]).
 * Outputs (DEVICE, overwritten):
 *  - grad_j: dL/dj, float[cells] when j is shared (j_bin_stride 0: the sum over bins),
 *    else float[n_bins][cells] (dL/dj_b);
 *  - grad_kappa: with a shared kappa and kappa_b = kappa_scale[b] kappa (kappa_bin_stride
 *    0), float[cells] holding sum_b kappa_scale[b] dL/dkappa_b; with per-bin kappa maps,
 *    float[n_bins][cells] holding dL/dkappa_b;
 *  - grad_kappa_scale: NULL, or (shared kappa only) float[n_bins] holding
 *    dL/dkappa_scale[b] = sum_v kappa[v] dL/dkappa_b[v], summed in binary64.
 * Other arguments as rtmi_trace_bins (options are not taken: the float tiled path with the
 * Fibonacci directions). RTMI_ERR_INVALID_ARG when grad_kappa_scale is given with per-bin
 * kappa maps. Workspace as rtmi_trace_vjp, reused bin after bin. */
int32_t rtmi_trace_bins_vjp(const float* j_maps, int64_t j_bin_stride,
                            const float* kappa_maps, int64_t kappa_bin_stride,
                            const float* kappa_scale, int32_t n_bins,
                            int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                            const float* source_pos, const int32_t* num_rays,
                            const int32_t* substep_cap, float step_size,
                            float radiation_velocity, float time_step, const float* grad_fields,
                            float* grad_j, float* grad_kappa, float* grad_kappa_scale, void* stream);

/* Helpers of the parameter fits (Sec. 4: a scalar amplitude recovered through the
 * tracer; here also a global opacity scale). rtmi_dot: out[0] = sum_i a[i] b[i] (DEVICE
 * float[count] each; out DEVICE float[1], overwritten), summed in binary64 by one
 * work-group in a fixed order. rtmi_scaled_copy: out[i] = scale[0] * in[i] with the
 * scale read from DEVICE memory (so a fitted parameter never leaves the device). */
int32_t rtmi_dot(const float* a, const float* b, int64_t count, float* out, void* stream);
int32_t rtmi_scaled_copy(const float* in, const float* scale, float* out, int64_t count,
                         void* stream);

/* Squared field error of the inverse problem (Sec. 4, "Gradient-based inversion": a
 * loss on the traced field, minimised through the tracer's gradient): *loss =
 * scale * sum_i (field[i] - target[i])^2 (DEVICE float[1], overwritten) and grad[i] =
 * 2 scale (field[i] - target[i]) = dL/dfield (DEVICE float[count], overwritten; it may
 * be passed as grad_field to rtmi_trace_vjp). field, target: DEVICE float[count]. With
 * scale = 1 / count this is the mean squared error. */
int32_t rtmi_field_mse(const float* field, const float* target, int64_t count, float scale,
                       float* grad, float* loss, void* stream);

/* Per-ray intensities of one source (a check of Eq. (2) on the device): writes
 * I_{k+1} for ray i (lattice order) and substep k to out_rays[i * n_s + k] (DEVICE
 * float[num_rays][n_s], n_s = rtmi_num_substeps(ds, c, dt, cap)) and, if out_tau is
 * not NULL, tau_{k+1} to out_tau in the same layout. No field is written. */
int32_t rtmi_debug_rays(const float* j_map, const float* kappa_map,
                        int32_t nx, int32_t ny, int32_t nz, const float* source_pos,
                        int32_t num_rays, float step_size, float radiation_velocity,
                        float time_step, int32_t cap, float* out_rays, float* out_tau,
                        void* stream);

/* Measurement hooks. While enabled (on != 0), every launch of a march kernel is bracketed
 * by a pair of HIP events recorded on its launch stream, tallied per kernel kind:
 * RTMI_KERNEL_RECORD (a record dispatch with its segment fix-up, if any),
 * RTMI_KERNEL_TILE (one tile-pass dispatch: one bin of one source launch),
 * RTMI_KERNEL_DIRECT, RTMI_KERNEL_TABLE (the gather-table build of a tiled call),
 * RTMI_KERNEL_GATHER (one gather-pass dispatch, gather_table = 3). Reading
 * waits for that kind's recorded events, returns the summed elapsed milliseconds and the
 * number of launches since the last enable or read of that kind, and resets them. Do
 * not enable timing while a stream is being captured. */
enum { RTMI_KERNEL_RECORD = 0, RTMI_KERNEL_TILE = 1, RTMI_KERNEL_DIRECT = 2, RTMI_KERNEL_TABLE = 3,
       RTMI_KERNEL_GATHER = 4 };
int32_t rtmi_timing_enable(int32_t on);
int32_t rtmi_timing_read(int32_t kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* RTMI_H */
