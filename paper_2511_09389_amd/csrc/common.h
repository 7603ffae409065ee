// Internal declarations shared by the host layer and the kernels of librtmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmi {

constexpr int kBlock = 256;          // lanes (rays) per work-group
constexpr int kMaxSrcPerLaunch = 32; // sources described in one launch's arguments
constexpr int kMaxBinsPerLaunch = 4; // bins a lane carries at once
constexpr int kPatch = 64;           // rays per coherent patch (one wavefront)
constexpr int kTile = 16;            // output tile edge, voxels
constexpr int kTileVox = kTile * kTile * kTile;
constexpr int kTileThreads = 512;    // lanes per tile work-group
constexpr int kPairBlock = 128;      // (source, patch) pairs per work-group of the tile geometry passes
constexpr int kChunk = 8;            // consecutive substeps one tile lane sums in registers
constexpr int kSeg = 4;              // substeps per recomputed segment of the adjoint sweep
// Per-patch record of the direction table: min x, y, z, max x, y, z, -, -, cone axis
// x, y, z, cos and sin of the cone's half-angle, -, -, -.
constexpr int kPatchRec = 16;
constexpr int kMaxParts = 64;        // work items (work-groups) sharing one output tile
constexpr int kRowAlign = 8;         // workspace rows are padded to this many substeps
constexpr int kXcds = 8;             // accelerator complex dies; work-groups go round-robin

// Everything one launch of the march needs, passed by value as kernel arguments so a
// call needs no per-call device buffer (and no allocation) for its source table.
struct MarchArgs {
  const float* j;          // j of bin 0 of this launch
  long long j_stride;      // elements between bins' j (0: shared)
  const float* kap;        // kappa of bin 0 of this launch
  long long k_stride;      // elements between bins' kappa (0: shared, scaled)
  float kscale[kMaxBinsPerLaunch];
  float* out;              // field of bin 0 of this launch (float mode)
  unsigned long long* acc; // fixed-point field of bin 0 (deterministic mode)
  const double* det_scale; // device scalar: fixed-point scale (deterministic mode)
  long long out_stride;    // elements between bins' fields (= cells)
  int nx, ny, nz;
  float ds;
  int n_src;
  int blk_begin[kMaxSrcPerLaunch + 1];
  float sx[kMaxSrcPerLaunch], sy[kMaxSrcPerLaunch], sz[kMaxSrcPerLaunch];
  float wray[kMaxSrcPerLaunch];
  int nrays[kMaxSrcPerLaunch];
  int nsub[kMaxSrcPerLaunch];
  const float4* dirs[kMaxSrcPerLaunch];
};

// One source of a tiled launch as the record and tile kernels read it, from a table in
// the launch's workspace (so that one launch can cover any number of sources). The table
// is written on the device by launch_write_sources from host data passed by value, which
// keeps a call free of host-to-device copies (and capturable in a graph).
struct alignas(16) SrcRec {
  float sx, sy, sz;           // position
  float tmax;                 // distance of the last substep (written on the device)
  float marg;                 // tile-geometry position margin (written on the device)
  float wray;                 // ray weight, 4 pi / N_Omega
  int nrays, nsub;            // rays (0 when N_s = 0), substeps
  long long vbase;            // workspace row base of the source's rays
  long long sbase;            // segment mode: first run end state of the source
  const float4* dirs;         // directions, one float4 per ray
  const float* pbounds;       // per 64-ray patch: kPatchRec floats (bounds and cone)
  int blk_begin;              // first record block, counted within the source's XCD group
  int pbegin;                 // first (source, patch) pair of the source in the launch
  int nseg;                   // segment mode: runs per ray
  int fbegin;                 // segment mode: first fix-up wave
};

constexpr int kSrcPerWrite = 24;    // sources one table-writing launch carries by value
struct SrcWrite {
  SrcRec rec[kSrcPerWrite];
  SrcRec* table;              // destination: table[first + i] = rec[i]
  int first, count;
  float ds;
};
constexpr int kMaxSrcPerTiledLaunch = 1 << 13;   // the chunk records hold 13 bits of source

// Phase 1 of the two-phase march: per-ray recurrence, deposit values to the workspace.
struct RecordArgs {
  const float4* med;          // gather table (8 corners of j, then of kappa, per voxel), or null
  const float2* jk;           // or: (j_k, kappa_k) rows of the gather pass, shaped like bin 0's V rows
  const float* j;
  long long j_stride;
  const float* kap;
  long long k_stride;
  float kscale[kMaxBinsPerLaunch];
  float* V;                   // workspace rows of bin 0
  long long v_bin_stride;     // elements between bins' rows
  float* corner;              // [NB][8] sums of samples collapsed onto a box corner
  unsigned long long* corner_q;  // the same in fixed point (deterministic mode)
  const double* det_scale;
  int nx, ny, nz;
  float ds;
  // The launch's sources, grouped by the XCD their record blocks run on: work-group i
  // runs on XCD i mod kXcds and takes block i / kXcds of that XCD's group, whose sources
  // are src[xcd_src[x] .. xcd_src[x + 1]) with xcd_blocks[x] blocks in all, most costly
  // first.
  const SrcRec* src;
  int n_src;
  int xcd_src[kXcds + 1];
  int xcd_blocks[kXcds];
  // Segments: with seg_len > 0 each ray's substeps are cut into runs of seg_len (a
  // multiple of kRowAlign) marched by separate lanes from I = 0, E = 1. Eq. (2) is linear
  // in the entry state (I0, E0): I_k = I0 P_k + E0 Q_k with P, Q the run's values from
  // (0, 1), so a later pass (fixup) turns the stored wray Q_k and P_k into the deposit
  // values once the runs' end states are chained.
  int seg_len;                // 0: whole rays
  int fix_waves;              // fix-up waves of the launch (sum of nrays (nseg - 1))
  float* P;                   // rows like V: P_k of runs after the first
  float2* segtot;             // [(sbase + ray * nseg + run) * NB + bin]: (Q, P) at the run's end
};

// Phase 2: tile-owned accumulation of the recorded deposit values.
struct TileArgs {
  const float* V;
  long long v_bin_stride;
  const float* corner;
  const unsigned long long* corner_q;
  float* out;
  unsigned long long* out_q;
  const double* det_scale;
  long long out_stride;
  int n_bins = 1;                 // tile kernel: bins of one launch (V, out and corner strided)
  int nx, ny, nz;
  int tiles_x, tiles_y, tiles_z;
  float ds;
  const SrcRec* src;              // the launch's sources (any order)
  int n_src;
  int n_pairs;                    // (source, 64-ray patch) pairs of the launch
  // Schedule, written by the cost, schedule and fill kernels and read by the tile kernel
  // (the field must be zeroed before the tile kernel adds into it).
  unsigned long long* tile_cost;  // [tiles] chunks per tile
  long long* tile_begin;          // [tiles] first chunk record of the tile
  long long* tile_count;          // [tiles] its records (clipped to rec_capacity)
  long long* tile_fill;           // [tiles] fill cursor: records below it are written
  unsigned* pair_mask;            // [tiles][pair blocks][kPairBlock / 32]: pairs with chunks in the tile
  long long* rec_total;           // chunk records of all tiles (before clipping)
  uint2* recs;                    // chunk records, grouped by tile
  long long rec_capacity;
  unsigned long long* dropped;    // device counter of records beyond rec_capacity, or null
  int2* item_map;                 // [tiles * kMaxParts] work item -> (tile, part | parts << 16)
  int* item_total;                // number of work items
  int* item_next;                 // next unclaimed work item
  int* item_done;                 // work-groups finished (the last one rewinds the counters)
  int item_chunks;                // target chunk records per work item
  int groups_per_cu;              // persistent tile grid: work-groups per compute unit (0: all that fit)
  // Gather pass: j (trilinear) and kappa (nearest voxel) of every sample from the shared
  // maps, written to rows shaped like bin 0's V rows.
  const float* gj;
  const float* gk;
  float2* jk;
  long long jk_bytes;             // bytes of the launch's rows (< 4 GiB: the stores take 32-bit offsets)
};

// Adjoint of the march: per-ray reverse sweep with checkpointed recomputation.
struct AdjointArgs {
  const float4* med;          // gather table: 8 corners of j, then of kappa, per voxel
  const float* grad;          // dL/dJ, [nx][ny][nz]
  float* Vj;                  // rows: dL/dj contribution of each sample (I-bar E ds)
  float* Vk;                  // rows: dL/dkappa of each sample, deposited at its nearest voxel
  float2* ckpt;               // (I, E) at the start of every segment of every ray
  float* corner_j;            // [8] sums of collapsed samples per box corner
  float* corner_k;            // [8]
  float kscale;               // this bin's opacity: table kappa x kscale (binary32, as the forward)
  float kgrad_scale;          // dL/dkappa deposits are multiplied by this (the bin scale of a shared kappa)
  double* dscale;             // or null: += sum over samples of table kappa(nearest) x dL/dkappa_bin
  int nx, ny, nz;
  float ds;
  int n_src;
  int blk_begin[kMaxSrcPerLaunch + 1];
  float sx[kMaxSrcPerLaunch], sy[kMaxSrcPerLaunch], sz[kMaxSrcPerLaunch];
  float wray[kMaxSrcPerLaunch];
  int nrays[kMaxSrcPerLaunch];
  int nsub[kMaxSrcPerLaunch];
  long long vbase[kMaxSrcPerLaunch];
  int cstride[kMaxSrcPerLaunch];
  long long cbase[kMaxSrcPerLaunch];
  const float4* dirs[kMaxSrcPerLaunch];
};

struct DebugArgs {
  const float* j;
  const float* kap;
  float* out_rays;
  float* out_tau;
  int nx, ny, nz;
  float ds;
  float sx, sy, sz;
  int nrays, nsub;
  const float4* dirs;
};

// Launchers (march.hip). They only enqueue; the host layer validates everything first.
hipError_t launch_march(const MarchArgs& a, int n_bins, bool shared_j, bool deterministic,
                        int n_blocks, hipStream_t s);
hipError_t launch_debug(const DebugArgs& a, hipStream_t s);
// Deposit values of the runs after the first (segment mode): one wave per run.
hipError_t launch_fixup(const RecordArgs& a, int n_bins, bool deterministic, int waves, hipStream_t s);
hipError_t launch_record(const RecordArgs& a, int n_bins, bool shared_j, bool deterministic,
                         int n_blocks, hipStream_t s);   // uses a.jk, else a.med, when not null
// Gather pass over the launch's chunk records (a.gj, a.gk -> a.jk); shares the tile pass's
// schedule and work-item counters (and rewinds them).
hipError_t launch_gather_pass(const TileArgs& a, hipStream_t s);
// Surrogate network: 3x3x3 convolutions over channels-last bf16 activations.
constexpr int kConvChannels = 32;

struct ConvArgs {
  const void* x;              // bf16 [n][d][h][w][32]: input (forward), dz (backward-data)
  const void* w;              // bf16 [27][32][32] forward weights
  const float* bias;          // forward, or null
  const void* residual;       // forward: bf16 tensor added after the activation, or null
  int gelu;                   // forward: apply GELU to conv + bias
  float* z;                   // forward: fp32 pre-activation out, or null
  void* y;                    // forward: bf16 out; backward-data: bf16 dz of the previous layer
  const float* residual_f32;  // backward-data: fp32 gradient added to the result, or null
  const float* zprev;         // backward-data: previous layer's pre-activation (GELU'), or null
  float* dh;                  // backward-data: fp32 gradient out, or null
  const void* dz;             // backward-weight: bf16 dz [n][d][h][w][32]
  float* dw;                  // backward-weight: fp32 [27][32][32], accumulated
  float* db;                  // backward-weight: fp32 [32], accumulated
  int n, d, h, w_dim;
};

// Input standardisation of the surrogate (fixed from its training set).
struct SurrogateStats {
  float log_kappa_mean, log_kappa_inv_std;
  float j_inv_scale;
  float log_cheap_mean, log_cheap_inv_std;
  float floor;                // added to the cheap field before the log
};

hipError_t launch_features(const float* j, const float* kap, const float* cheap, long long cells,
                           const SurrogateStats& st, float* sums, unsigned short* x, hipStream_t s);
hipError_t launch_surrogate_output(const unsigned short* y, const float* cheap, long long cells,
                                   const float* sums, float* field, float* check, hipStream_t s);
hipError_t launch_conv(const ConvArgs& a, bool backward, hipStream_t s);
// Weight gradient (adds into a.dw and a.db); `part` is scratch of wgrad_scratch_bytes(a).
size_t wgrad_scratch_bytes(const ConvArgs& a);
hipError_t launch_wgrad(const ConvArgs& a, float* part, hipStream_t s);
hipError_t launch_mse(const unsigned short* y, const float* target, long long nvox, float scale,
                      unsigned short* dz, float* loss, hipStream_t s);
hipError_t launch_adam(float* w, float* m, float* v, const float* g, unsigned short* w_bf16,
                       long long count, float lr, float b1, float b2, float eps, float c1, float c2,
                       hipStream_t s);

// Tile launches: the schedule (per-tile cost, work items; depends on the geometry only)
// and the persistent tile kernel, which leaves the schedule ready for another run.
// Per tile: chunk counts, the work items and the record offsets (cost + schedule kernels).
hipError_t launch_tile_schedule(const TileArgs& a, int tiles, hipStream_t s);
// Writes the chunk records of every tile (after launch_tile_schedule on the same buffers).
hipError_t launch_tile_fill(const TileArgs& a, int tiles, hipStream_t s);
hipError_t launch_tile_run(const TileArgs& a, int n_bins, bool deterministic, bool nearest,
                           hipStream_t s);
// The tile pass of one bin of a launch (launch_tile_run runs every bin's in turn).
hipError_t launch_tile_bin(const TileArgs& a, int bin, bool deterministic, bool nearest, hipStream_t s);
// All n_bins bins of the launch in one persistent kernel: its work-groups claim (item, bin)
// pairs, the bins of an item one after another.
hipError_t launch_tile_bins(const TileArgs& a, int n_bins, bool deterministic, bool nearest, hipStream_t s);
hipError_t launch_adjoint_record(const AdjointArgs& a, int n_blocks, hipStream_t s);
// out[i] = (float) in[i], i < n (the scale gradients, summed in binary64)
hipError_t launch_f64_to_f32(const double* in, float* out, int n, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, long long n, float* out, hipStream_t s);
hipError_t launch_scaled_copy(const float* in, const float* scale, float* out, long long n, hipStream_t s);
// loss[0] = scale * sum (field - target)^2 (overwritten), grad = 2 scale (field - target).
hipError_t launch_field_mse(const float* field, const float* target, long long n, float scale, float* grad,
                            float* loss, hipStream_t s);
// Gather table of j and kappa (64 bytes per voxel) for the record and adjoint kernels.
hipError_t launch_cell_table(const float* j, const float* kap, float4* table, int nx, int ny, int nz,
                             hipStream_t s);
// Writes w.rec[0 .. count) to w.table[first ..), completing tmax and marg.
hipError_t launch_write_sources(const SrcWrite& w, hipStream_t s);
hipError_t launch_fill_zero(float* p, long long n, hipStream_t s);
hipError_t launch_fill_zero_u64(unsigned long long* p, long long n, hipStream_t s);
// scale_out[0] = the fixed-point scale, a power of two with bound * scale <= 2^62, where
// bound = max|j| * bound_per_unit_j * exp(growth_per_neg_kappa * max(0, -min kappa));
// scale_out[1] is scratch.
hipError_t launch_det_scale(const float* j, long long j_count, const float* kap, long long k_count,
                            double growth_per_neg_kappa, double bound_per_unit_j, double* scale_out,
                            hipStream_t s);
hipError_t launch_det_convert(const unsigned long long* acc, const double* scale, float* out,
                              long long n, hipStream_t s);

}  // namespace rtmi
