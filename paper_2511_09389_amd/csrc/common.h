// Internal declarations shared by the host layer and the kernels of librtmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtmi {

constexpr int kBlock = 256;          // lanes (rays) per work-group
constexpr int kMaxSrcPerLaunch = 32; // sources described in one launch's arguments
constexpr int kMaxBinsPerLaunch = 4; // bins a lane carries at once

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
hipError_t launch_fill_zero(float* p, long long n, hipStream_t s);
hipError_t launch_fill_zero_u64(unsigned long long* p, long long n, hipStream_t s);
hipError_t launch_det_scale(const float* j, long long j_count, double bound_per_unit_j,
                            double* scale_out, hipStream_t s);
hipError_t launch_det_convert(const unsigned long long* acc, const double* scale, float* out,
                              long long n, hipStream_t s);

}  // namespace rtmi
