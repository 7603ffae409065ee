// Microbenchmarks of the device rates that bound the march (librtmi_peaks.so): device
// copy, random 64-byte line gathers at a chosen footprint, LDS atomic adds and global
// float atomic adds. Each call times `reps` launches with HIP events and keeps the best.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/rtmi_peaks.h"

namespace {

constexpr int kThreads = 256;
constexpr int kLdsThreads = 512;
constexpr int kLdsRounds = 12;                       // distinct slots per lane
constexpr int kLdsSlots = kLdsThreads * kLdsRounds;  // 48 KB of binary64: three groups per CU

__device__ __forceinline__ unsigned lcg(unsigned h) { return h * 1664525u + 1013904223u; }

__device__ __forceinline__ unsigned seed(unsigned i) {
  // (a 32-bit integer hash, so that neighbouring lanes start far apart)
  i ^= i >> 16;
  i *= 0x7feb352du;
  i ^= i >> 15;
  i *= 0x846ca68bu;
  i ^= i >> 16;
  return i;
}

__global__ void __launch_bounds__(kThreads) copy_kernel(const float4* __restrict__ a, float4* __restrict__ b,
                                                        long long n) {
  const long long stride = static_cast<long long>(gridDim.x) * kThreads;
  for (long long i = blockIdx.x * static_cast<long long>(kThreads) + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// Each lane reads `iters` whole 64-byte lines at pseudo-random line indices below `lines`
// (the addresses do not depend on the loaded values, so the loads overlap).
__global__ void __launch_bounds__(kThreads) gather_kernel(const float4* __restrict__ t, unsigned lines, int iters,
                                                          float* __restrict__ out) {
  const unsigned tid = blockIdx.x * kThreads + threadIdx.x;
  unsigned h = seed(tid);
  float acc = 0.0f;
  for (int it = 0; it < iters; it += 4) {
    float4 v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      h = lcg(h);
      const float4* p = t + 4ull * (h % lines);
#pragma unroll
      for (int q = 0; q < 4; ++q) v[u][q] = p[q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u][0].x + v[u][1].y + v[u][2].z + v[u][3].w;
  }
  out[tid] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kLdsThreads) lds_atomic_kernel(int iters, T* __restrict__ out) {
  __shared__ T acc[kLdsSlots];
  const int tid = static_cast<int>(threadIdx.x);
  for (int i = tid; i < kLdsSlots; i += kLdsThreads) acc[i] = T(0);
  __syncthreads();
  const T one = T(1);
  for (int it = 0; it < iters; it += kLdsRounds) {
#pragma unroll
    for (int q = 0; q < kLdsRounds; ++q) atomicAdd(&acc[tid + kLdsThreads * q], one);
  }
  __syncthreads();
  T s = T(0);
#pragma unroll
  for (int q = 0; q < kLdsRounds; ++q) s += acc[tid + kLdsThreads * q];
  out[blockIdx.x * kLdsThreads + tid] = s;
}

// The same adds at pseudo-random slots of the 48 KB array (each lane draws its kLdsRounds
// slots once, so the loop issues nothing but the adds): the bank conflicts and occasional
// same-address collisions of lanes whose addresses are unrelated, as in a tile pass whose
// lanes deposit along different rays. Only one lane in EVERY of each wave adds, as in a
// tile pass where only the lanes whose ray left a cell flush their sums.
template <typename T, int EVERY>
__global__ void __launch_bounds__(kLdsThreads) lds_atomic_random_kernel(int iters, T* __restrict__ out) {
  __shared__ T acc[kLdsSlots];
  const int tid = static_cast<int>(threadIdx.x);
  for (int i = tid; i < kLdsSlots; i += kLdsThreads) acc[i] = T(0);
  int slot[kLdsRounds];
#pragma unroll
  for (int q = 0; q < kLdsRounds; ++q)
    slot[q] = static_cast<int>(seed(static_cast<unsigned>((blockIdx.x * kLdsThreads + tid) * kLdsRounds + q)) %
                               static_cast<unsigned>(kLdsSlots));
  __syncthreads();
  if ((tid & 63) % EVERY == 0) {
    for (int it = 0; it < iters; it += kLdsRounds) {
#pragma unroll
      for (int q = 0; q < kLdsRounds; ++q) atomicAdd(&acc[slot[q]], T(1));
    }
  }
  __syncthreads();
  T s = T(0);
#pragma unroll
  for (int q = 0; q < kLdsRounds; ++q) s += acc[tid + kLdsThreads * q];
  out[blockIdx.x * kLdsThreads + tid] = s;
}

// scattered: each lane adds to the first word of a pseudo-random 64-byte line;
// otherwise lane i of round r adds to word (i + r * lanes) mod words.
__global__ void __launch_bounds__(kThreads) global_atomic_kernel(float* __restrict__ buf, unsigned words,
                                                                 int scattered, int iters) {
  const unsigned tid = blockIdx.x * kThreads + threadIdx.x;
  const unsigned lanes = gridDim.x * kThreads;
  const unsigned lines = words / 16u;
  unsigned h = seed(tid);
  for (int it = 0; it < iters; ++it) {
    unsigned w;
    if (scattered) {
      h = lcg(h);
      w = (h % lines) * 16u;
    } else {
      w = static_cast<unsigned>((static_cast<unsigned long long>(tid) + static_cast<unsigned long long>(it) * lanes) %
                                words);
    }
    unsafeAtomicAdd(buf + w, 1.0f);
  }
}

int compute_units() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 256;
  return cus;
}

// Time `reps` calls of `launch` (after one untimed call); the shortest, in seconds.
template <typename F>
int32_t best_time(F launch, int32_t reps, double* seconds) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -4;
  int32_t rc = 0;
  double best = 1e30;
  launch();
  for (int r = 0; r < std::max(reps, 1) && rc == 0; ++r) {
    float ms = 0.0f;
    if (hipEventRecord(a, nullptr) != hipSuccess) rc = -4;
    launch();
    if (rc == 0 && (hipGetLastError() != hipSuccess || hipEventRecord(b, nullptr) != hipSuccess ||
                    hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess))
      rc = -4;
    best = std::min(best, 1e-3 * static_cast<double>(ms));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *seconds = best;
  return rc;
}

struct Buffers {
  void* p[2] = {nullptr, nullptr};
  ~Buffers() {
    (void)hipDeviceSynchronize();
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
};

}  // namespace

extern "C" {

int32_t rtmi_peak_copy(int64_t bytes, int32_t reps, double* rate, double* bytes_or_ops) {
  if (!rate || bytes < 16 * 1024) return -1;
  const long long n = bytes / 16;
  Buffers B;
  if (hipMalloc(&B.p[0], n * 16) != hipSuccess || hipMalloc(&B.p[1], n * 16) != hipSuccess) return -4;
  if (hipMemset(B.p[0], 0, n * 16) != hipSuccess) return -4;
  const int grid = compute_units() * 8;
  double t = 0.0;
  const int32_t rc = best_time([&] {
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kThreads), 0, nullptr, static_cast<const float4*>(B.p[0]),
                       static_cast<float4*>(B.p[1]), n);
  }, reps, &t);
  if (rc) return rc;
  *rate = 2.0 * 16.0 * static_cast<double>(n) / t;
  if (bytes_or_ops) *bytes_or_ops = 2.0 * 16.0 * static_cast<double>(n);
  return 0;
}

int32_t rtmi_peak_gather(int64_t footprint, int32_t iters, int32_t reps, double* rate, double* bytes_or_ops) {
  if (!rate || footprint < 4096 || footprint > (int64_t(1) << 36) || iters < 4 || iters % 4) return -1;
  const unsigned lines = static_cast<unsigned>(footprint / 64);
  const int grid = compute_units() * 16;
  const long long lanes = static_cast<long long>(grid) * kThreads;
  Buffers B;
  if (hipMalloc(&B.p[0], static_cast<size_t>(lines) * 64) != hipSuccess ||
      hipMalloc(&B.p[1], lanes * sizeof(float)) != hipSuccess)
    return -4;
  if (hipMemset(B.p[0], 0, static_cast<size_t>(lines) * 64) != hipSuccess) return -4;
  double t = 0.0;
  const int32_t rc = best_time([&] {
    hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(kThreads), 0, nullptr, static_cast<const float4*>(B.p[0]),
                       lines, iters, static_cast<float*>(B.p[1]));
  }, reps, &t);
  if (rc) return rc;
  const double moved = 64.0 * static_cast<double>(lanes) * iters;
  *rate = moved / t;
  if (bytes_or_ops) *bytes_or_ops = moved;
  return 0;
}

int32_t rtmi_peak_lds_atomic(int32_t kind, int32_t iters, int32_t reps, double* rate, double* bytes_or_ops) {
  if (!rate || kind < 0 || kind > 7 || iters < kLdsRounds || iters % kLdsRounds) return -1;
  const int grid = compute_units() * 3;
  Buffers B;
  if (hipMalloc(&B.p[0], static_cast<size_t>(grid) * kLdsThreads * 8) != hipSuccess) return -4;
  double t = 0.0;
  const int32_t rc = best_time([&] {
    if (kind == 0)
      hipLaunchKernelGGL(lds_atomic_kernel<double>, dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<double*>(B.p[0]));
    else if (kind == 2)
      hipLaunchKernelGGL(lds_atomic_kernel<float>, dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<float*>(B.p[0]));
    else if (kind == 3)
      hipLaunchKernelGGL((lds_atomic_random_kernel<double, 1>), dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<double*>(B.p[0]));
    else if (kind == 4)
      hipLaunchKernelGGL((lds_atomic_random_kernel<unsigned long long, 1>), dim3(grid), dim3(kLdsThreads), 0,
                         nullptr, iters, static_cast<unsigned long long*>(B.p[0]));
    else if (kind == 5)
      hipLaunchKernelGGL((lds_atomic_random_kernel<double, 2>), dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<double*>(B.p[0]));
    else if (kind == 6)
      hipLaunchKernelGGL((lds_atomic_random_kernel<double, 4>), dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<double*>(B.p[0]));
    else if (kind == 7)
      hipLaunchKernelGGL((lds_atomic_random_kernel<double, 8>), dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<double*>(B.p[0]));
    else
      hipLaunchKernelGGL(lds_atomic_kernel<unsigned long long>, dim3(grid), dim3(kLdsThreads), 0, nullptr, iters,
                         static_cast<unsigned long long*>(B.p[0]));
  }, reps, &t);
  if (rc) return rc;
  const int every = kind == 5 ? 2 : kind == 6 ? 4 : kind == 7 ? 8 : 1;   // (adds of the active lanes)
  const double ops = static_cast<double>(grid) * kLdsThreads * iters / every;
  *rate = ops / t;
  if (bytes_or_ops) *bytes_or_ops = ops;
  return 0;
}

int32_t rtmi_peak_global_atomic(int64_t footprint, int32_t scattered, int32_t iters, int32_t reps, double* rate,
                                double* bytes_or_ops) {
  if (!rate || footprint < 4096 || footprint > (int64_t(1) << 32) || iters < 1) return -1;
  const unsigned words = static_cast<unsigned>(footprint / 64) * 16u;
  const int grid = compute_units() * 16;
  Buffers B;
  if (hipMalloc(&B.p[0], static_cast<size_t>(words) * 4) != hipSuccess) return -4;
  if (hipMemset(B.p[0], 0, static_cast<size_t>(words) * 4) != hipSuccess) return -4;
  double t = 0.0;
  const int32_t rc = best_time([&] {
    hipLaunchKernelGGL(global_atomic_kernel, dim3(grid), dim3(kThreads), 0, nullptr, static_cast<float*>(B.p[0]),
                       words, scattered ? 1 : 0, iters);
  }, reps, &t);
  if (rc) return rc;
  const double ops = static_cast<double>(grid) * kThreads * iters;
  *rate = ops / t;
  if (bytes_or_ops) *bytes_or_ops = ops;
  return 0;
}

}  // extern "C"
