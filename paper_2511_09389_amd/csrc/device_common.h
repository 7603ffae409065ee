// Device helpers shared by the march kernels: sample points and the clamped stencil.
#pragma once

#include <hip/hip_runtime.h>

namespace rtmi {

// One axis of the clamped trilinear stencil and of the nearest-voxel pick at x.
struct Axis {
  int lo, hi;    // clamped corner indices (lo == hi when x < 0 or x >= n - 1)
  float w0, w1;  // 1-D weights of lo and hi (they sum to 1)
  int nearest;   // clamped round-half-to-even index
};

__device__ __forceinline__ Axis axis_stencil(float x, int n) {
  const float fl = floorf(x);
  const float f = x - fl;  // exact for binary32 x
  const int i = static_cast<int>(fminf(fmaxf(fl, -1.0f), static_cast<float>(n - 1)));
  Axis a;
  a.lo = max(i, 0);
  a.hi = min(i + 1, n - 1);
  a.w0 = 1.0f - f;
  a.w1 = f;
  a.nearest = static_cast<int>(fminf(fmaxf(rintf(x), 0.0f), static_cast<float>(n - 1)));
  return a;
}

// x = fl(src + fl(t * n)): two separately rounded binary32 operations, never fused, so
// that every implementation takes its floor/round decisions on the same numbers.
__device__ __forceinline__ float sample_axis(float src, float t, float n) {
#pragma clang fp contract(off)
  const float p = t * n;
  return src + p;
}

// t = fl(k ds), the distance of substep k from the source.
__device__ __forceinline__ float sample_distance(int k, float ds) {
#pragma clang fp contract(off)
  return static_cast<float>(k) * ds;
}

// True when the stencil collapses onto one voxel along this axis (x < 0 or x >= n - 1).
__device__ __forceinline__ bool axis_clamped(float x, int n) {
  return x < 0.0f || x >= static_cast<float>(n - 1);
}

// Workspace rows of one source: the value of (ray, substep k) sits at
//   base + ((k / 8) * nrays + ray) * 8 + k % 8,
// so the rays of a wavefront write one 8-substep chunk as one contiguous run, and a
// chunk of one ray is 32 contiguous, 32-byte-aligned bytes.
__device__ __forceinline__ long long row_slot(long long base, int nrays, int ray, int k) {
  return base + (static_cast<long long>(k >> 3) * nrays + ray) * 8 + (k & 7);
}

}  // namespace rtmi
