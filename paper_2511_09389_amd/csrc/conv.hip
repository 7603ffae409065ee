// 3x3x3 "same" convolutions of the surrogate network on bf16 matrix cores (MFMA), fp32
// accumulation. Activations are channels-last bf16 [n][z][y][x][32]; weights bf16
// [27][32 co][32 ci] with tap = ((dz+1)*3 + (dy+1))*3 + (dx+1); zero padding.
//
// conv_kernel (forward and backward-data): an implicit GEMM, out[v][co] = sum over taps
// and ci of x[v + off(tap)][ci] W[tap][co][ci], one wave per 32 output voxels x 32
// channels: 27 taps x 2 MFMA 32x32x16 steps. The weights sit in LDS (staged flipped and
// transposed for the backward-data pass, where dx[u][ci] = sum W[tap][co][ci]
// dz[u - off(tap)][co]). The A operand (8 consecutive channels of one voxel) is one
// 16-byte load straight from global memory.
// wgrad_kernel: dW[tap][co][ci] = sum_v dz[v][co] x[v + off(tap)][ci]; the K dimension is
// voxels, so an x-row of dz and the nine neighbouring rows of x (three shifted copies
// each) are staged transposed in LDS; three waves own the taps with dx = -1, 0, +1.
#include "common.h"

namespace rtmi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kC = kConvChannels;   // 32
constexpr int kConvThreads = 256;   // 4 waves, 32 output voxels each per round

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(static_cast<unsigned>(h) << 16);
}

// Round to nearest even (inputs here are finite).
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// MFMA 32x32 accumulator layout (wave64): element i of lane l is row
// 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
__device__ __forceinline__ int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

template <bool BACKWARD>
__global__ void __launch_bounds__(kConvThreads) conv_kernel(const ConvArgs a) {
  // B operand: Bs[tap][half][column][16 k], k contiguous (forward: column co, k = ci;
  // backward: column ci, k = co, taps mirrored)
  __shared__ __attribute__((aligned(16))) unsigned short Bs[27 * 2 * kC * 16];
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const unsigned short* W = static_cast<const unsigned short*>(a.w);
  for (int i = tid; i < 27 * kC * kC; i += kConvThreads) {
    const int tap = i / (kC * kC), col = (i / kC) % kC, k = i % kC;
    // forward: W[tap][co = col][ci = k]; backward: W[26 - tap][co = k][ci = col]
    const unsigned short v = BACKWARD ? W[((26 - tap) * kC + k) * kC + col] : W[(tap * kC + col) * kC + k];
    Bs[((tap * 2 + (k >> 4)) * kC + col) * 16 + (k & 15)] = v;
  }
  __syncthreads();

  const unsigned short* X = static_cast<const unsigned short*>(a.x);
  const int D = a.d, H = a.h, Wd = a.w_dim;
  const long long nvox = static_cast<long long>(a.n) * D * H * Wd;
  const int r = lane & 31, kg = lane >> 5;
  const int co = lane & 31;   // this lane's output column
  for (long long blk = (static_cast<long long>(blockIdx.x) * 4 + wave) * 32; blk < nvox;
       blk += static_cast<long long>(gridDim.x) * 4 * 32) {
    // this lane's A row: voxel blk + r
    const long long v = blk + r;
    const bool vin = v < nvox;
    long long t = vin ? v : 0;
    const int x = static_cast<int>(t % Wd); t /= Wd;
    const int y = static_cast<int>(t % H); t /= H;
    const int z = static_cast<int>(t % D);
    const long long nbase = t / D * D;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
#pragma unroll 3
    for (int tap = 0; tap < 27; ++tap) {
      const int oz = tap / 9 - 1, oy = (tap / 3) % 3 - 1, ox = tap % 3 - 1;
      const int zz = z + oz, yy = y + oy, xx = x + ox;
      const bool in = vin && zz >= 0 && zz < D && yy >= 0 && yy < H && xx >= 0 && xx < Wd;
      const long long nb = ((nbase + zz) * H + yy) * Wd + xx;
      u16x8 a0 = {0, 0, 0, 0, 0, 0, 0, 0}, a1 = {0, 0, 0, 0, 0, 0, 0, 0};
      if (in) {
        const u16x8* src = reinterpret_cast<const u16x8*>(X + nb * kC);
        a0 = src[kg];
        a1 = src[2 + kg];
      }
      const u16x8 b0 = *reinterpret_cast<const u16x8*>(&Bs[((tap * 2 + 0) * kC + co) * 16 + kg * 8]);
      const u16x8 b1 = *reinterpret_cast<const u16x8*>(&Bs[((tap * 2 + 1) * kC + co) * 16 + kg * 8]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0), acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1), __builtin_bit_cast(bf16x8, b1), acc, 0, 0, 0);
    }
    // epilogue: lane holds column co of rows acc_row(i, lane)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const long long vo = blk + acc_row(i, lane);
      if (vo >= nvox) continue;
      const long long e = vo * kC + co;
      float s = acc[i];
      if constexpr (!BACKWARD) {
        if (a.bias) s += a.bias[co];
        if (a.z) a.z[e] = s;
        float y_out = a.gelu ? gelu_f(s) : s;
        if (a.residual) y_out += bf16_to_f32(static_cast<const unsigned short*>(a.residual)[e]);
        static_cast<unsigned short*>(a.y)[e] = f32_to_bf16(y_out);
      } else {
        if (a.residual_f32) s += a.residual_f32[e];
        if (a.dh) a.dh[e] = s;
        if (a.y) {
          const float g = a.zprev ? s * gelu_grad_f(a.zprev[e]) : s;
          static_cast<unsigned short*>(a.y)[e] = f32_to_bf16(g);
        }
      }
    }
  }
}

// dW (and db) of one layer; rows = (n, z, y) x-rows of length a.w_dim (a multiple of 16,
// at most kMaxRow).
constexpr int kMaxRow = 64;
constexpr int kWgradThreads = 192;

__global__ void __launch_bounds__(kWgradThreads) wgrad_kernel(const ConvArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned short dzT[kC][kMaxRow];       // [co][x]
  __shared__ __attribute__((aligned(16))) unsigned short xs[3][kC][kMaxRow];     // [dx+1][ci][x]
  __shared__ float db_part[kC];
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;   // wave: dx + 1
  const unsigned short* X = static_cast<const unsigned short*>(a.x);
  const unsigned short* DZ = static_cast<const unsigned short*>(a.dz);
  const int D = a.d, H = a.h, Wd = a.w_dim;
  const long long rows = static_cast<long long>(a.n) * D * H;
  const int kb_count = Wd / 16;
  if (tid < kC) db_part[tid] = 0.0f;
  f32x16 acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.0f;
  float db_acc = 0.0f;

  for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
    const int y = static_cast<int>(row % H);
    const int z = static_cast<int>((row / H) % D);
    const long long n = row / (static_cast<long long>(H) * D);
    __syncthreads();
    // dz of the row, transposed
    for (int i = tid; i < Wd * kC; i += kWgradThreads) {
      const int x = i / kC, c = i % kC;
      dzT[c][x] = DZ[(row * Wd + x) * kC + c];
    }
    __syncthreads();
    if (tid < kC) {
      float s = 0.0f;
      for (int x = 0; x < Wd; ++x) s += bf16_to_f32(dzT[tid][x]);
      db_acc += s;
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int oz = t / 3 - 1, oy = t % 3 - 1;
      const int zz = z + oz, yy = y + oy;
      const bool row_in = zz >= 0 && zz < D && yy >= 0 && yy < H;
      const long long src_row = (n * D + zz) * H + yy;
      __syncthreads();
      // the neighbouring row at (dz, dy), in three copies shifted by dx = -1, 0, +1
      for (int i = tid; i < 3 * Wd * kC; i += kWgradThreads) {
        const int s = i / (Wd * kC), rem = i % (Wd * kC), x = rem / kC, c = rem % kC;
        const int xx = x + s - 1;
        unsigned short v = 0;
        if (row_in && xx >= 0 && xx < Wd) v = X[(src_row * Wd + xx) * kC + c];
        xs[s][c][x] = v;
      }
      __syncthreads();
      const int col = lane & 31, kg = lane >> 5;
      for (int kb = 0; kb < kb_count; ++kb) {
        const u16x8 av = *reinterpret_cast<const u16x8*>(&dzT[col][kb * 16 + kg * 8]);
        const u16x8 bv = *reinterpret_cast<const u16x8*>(&xs[wave][col][kb * 16 + kg * 8]);
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc[t], 0, 0, 0);
      }
    }
  }
  // this wave's taps (dz, dy, dx = wave - 1): rows co, columns ci
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int tap = t * 3 + wave;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int co = acc_row(i, lane), ci = lane & 31;
      if (acc[t][i] != 0.0f) unsafeAtomicAdd(a.dw + (tap * kC + co) * kC + ci, acc[t][i]);
    }
  }
  if (tid < kC && db_acc != 0.0f) unsafeAtomicAdd(a.db + tid, db_acc);
}

// Loss of the surrogate (mean squared error of channel 0 against the target) and its
// gradient, seeded into a zeroed 32-channel bf16 tensor for the last layer's backward.
__global__ void mse_kernel(const unsigned short* __restrict__ y, const float* __restrict__ target,
                           long long nvox, float scale, unsigned short* __restrict__ dz,
                           float* __restrict__ loss) {
  float part = 0.0f;
  for (long long v = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; v < nvox;
       v += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float d = bf16_to_f32(y[v * kC]) - target[v];
    part += d * d;
#pragma unroll
    for (int c = 0; c < kC; ++c) dz[v * kC + c] = c == 0 ? f32_to_bf16(2.0f * scale * d) : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0 && part != 0.0f) unsafeAtomicAdd(loss, part * scale);
}

// Adam on fp32 master weights; writes the bf16 copy the convolutions read.
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, unsigned short* __restrict__ w_bf16,
                            long long count, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (w_bf16) w_bf16[i] = f32_to_bf16(wi);
  }
}

// sums[0] += sum of cheap^2 over the sample (the scale s = sqrt(sums[0] / cells) of the
// linear features and of the prediction).
__global__ void sumsq_kernel(const float* __restrict__ cheap, long long cells, float* __restrict__ sums) {
  float part = 0.0f;
  for (long long v = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; v < cells;
       v += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float c = fmaxf(cheap[v], 0.0f);
    part += c * c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0 && part != 0.0f) unsafeAtomicAdd(sums, part);
}

__global__ void fill_sums_kernel(float* sums) {
  if (threadIdx.x < 2) sums[threadIdx.x] = 0.0f;
}

__device__ __forceinline__ float sample_scale(const float* sums, long long cells) {
  return fmaxf(sqrtf(sums[0] / static_cast<float>(cells)), 1e-30f);
}

// Network input of one sample: channel 0 standardised log kappa, 1 scaled j, 2 the cheap
// (few-ray) field over its scale s, 3 the standardised log of the cheap field, the rest 0.
__global__ void features_kernel(const float* __restrict__ j, const float* __restrict__ kap,
                                const float* __restrict__ cheap, long long cells, SurrogateStats st,
                                const float* __restrict__ sums, unsigned short* __restrict__ x) {
  const float inv_s = 1.0f / sample_scale(sums, cells);
  for (long long v = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; v < cells;
       v += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float c = fmaxf(cheap[v], 0.0f);
    const float f[4] = {(logf(fmaxf(kap[v], 1e-30f)) - st.log_kappa_mean) * st.log_kappa_inv_std,
                        j[v] * st.j_inv_scale, c * inv_s,
                        (logf(c + st.floor) - st.log_cheap_mean) * st.log_cheap_inv_std};
#pragma unroll
    for (int ch = 0; ch < kC; ++ch) x[v * kC + ch] = ch < 4 ? f32_to_bf16(f[ch]) : 0;
  }
}

// Prediction: the network's channel 0 corrects the cheap field in units of its scale,
// J = max(0, cheap + s y); also sums, for the error check, (J - cheap)^2 and cheap^2 into
// check[0], check[1].
__global__ void output_kernel(const unsigned short* __restrict__ y, const float* __restrict__ cheap,
                              long long cells, const float* __restrict__ sums, float* __restrict__ field,
                              float* __restrict__ check) {
  const float scale = sample_scale(sums, cells);
  float s0 = 0.0f, s1 = 0.0f;
  for (long long v = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; v < cells;
       v += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float c = fmaxf(cheap[v], 0.0f);
    const float J = fmaxf(c + scale * bf16_to_f32(y[v * kC]), 0.0f);
    field[v] = J;
    s0 += (J - c) * (J - c);
    s1 += c * c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    unsafeAtomicAdd(check, s0);
    unsafeAtomicAdd(check + 1, s1);
  }
}

int grid_for(long long work, int per_block) {
  long long g = (work + per_block - 1) / per_block;
  return static_cast<int>(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t launch_conv(const ConvArgs& a, bool backward, hipStream_t s) {
  const long long nvox = static_cast<long long>(a.n) * a.d * a.h * a.w_dim;
  const int grid = grid_for(nvox, 4 * 32 * 4);   // about four rounds of 128 voxels per group
  if (backward) hipLaunchKernelGGL(conv_kernel<true>, dim3(grid), dim3(kConvThreads), 0, s, a);
  else hipLaunchKernelGGL(conv_kernel<false>, dim3(grid), dim3(kConvThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(const ConvArgs& a, hipStream_t s) {
  const long long rows = static_cast<long long>(a.n) * a.d * a.h;
  const int grid = static_cast<int>(rows < 1024 ? (rows < 1 ? 1 : rows) : 1024);
  hipLaunchKernelGGL(wgrad_kernel, dim3(grid), dim3(kWgradThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mse(const unsigned short* y, const float* target, long long nvox, float scale,
                      unsigned short* dz, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(grid_for(nvox, 256 * 4)), dim3(256), 0, s, y, target, nvox, scale, dz, loss);
  return hipGetLastError();
}

hipError_t launch_features(const float* j, const float* kap, const float* cheap, long long cells,
                           const SurrogateStats& st, float* sums, unsigned short* x, hipStream_t s) {
  hipLaunchKernelGGL(fill_sums_kernel, dim3(1), dim3(64), 0, s, sums);
  hipLaunchKernelGGL(sumsq_kernel, dim3(grid_for(cells, 256 * 4)), dim3(256), 0, s, cheap, cells, sums);
  hipLaunchKernelGGL(features_kernel, dim3(grid_for(cells, 256 * 4)), dim3(256), 0, s, j, kap, cheap, cells, st,
                     sums, x);
  return hipGetLastError();
}

hipError_t launch_surrogate_output(const unsigned short* y, const float* cheap, long long cells, const float* sums,
                                   float* field, float* check, hipStream_t s) {
  hipLaunchKernelGGL(output_kernel, dim3(grid_for(cells, 256 * 4)), dim3(256), 0, s, y, cheap, cells, sums,
                     field, check);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, float* m, float* v, const float* g, unsigned short* w_bf16, long long count,
                       float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(count, 256 * 4)), dim3(256), 0, s, w, m, v, g, w_bf16, count,
                     lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace rtmi
