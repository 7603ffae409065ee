// 3x3x3 "same" convolutions of the surrogate network on bf16 matrix cores (MFMA), fp32
// accumulation. Activations are channels-last bf16 [n][z][y][x][32]; weights bf16
// [27][32 co][32 ci] with tap = ((dz+1)*3 + (dy+1))*3 + (dx+1); zero padding.
//
// conv_tile_kernel (forward and backward-data): an implicit GEMM, out[v][co] = sum over
// taps and ci of x[v + off(tap)][ci] W[tap][co][ci], 32 output voxels x 32 channels per
// MFMA 32x32x16 accumulator: 27 taps x 2 steps. The weights sit in LDS (staged flipped and
// transposed for the backward-data pass, where dx[u][ci] = sum W[tap][co][ci]
// dz[u - off(tap)][co]), and so does each block's input with its halo.
// wgrad: dW[tap][co][ci] = sum_v dz[v][co] x[v + off(tap)][ci], a GEMM over the voxels on
// channel-major copies of dz and of x (three, shifted by dx = -1, 0, +1), so that a row
// shift is a whole number of rows and every operand an aligned 16-byte load.
#include "common.h"

namespace rtmi {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int kC = kConvChannels;   // 32

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(static_cast<unsigned>(h) << 16);
}

// Round to nearest even (inputs here are finite).
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return static_cast<unsigned short>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// erf by the rational approximation of Abramowitz and Stegun (Handbook of Mathematical
// Functions, 7.1.26): erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2) with
// t = 1 / (1 + p x) for x >= 0, odd in x; absolute error below 1.5e-7, far under the bf16
// rounding of the activations it feeds.
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * ax);
  const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float r = 1.0f - poly * __expf(-ax * ax);
  return copysignf(r, x);
}

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

// MFMA 32x32 accumulator layout (wave64): element i of lane l is row
// 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
__device__ __forceinline__ int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// conv_tile_kernel: a persistent work-group of eight waves stages the weights once, then
// takes blocks of 2 (z) x 8 (y) x 32 (x) output voxels in turn; it loads a block's input
// with its one-voxel halo (4 x 10 x 34 voxels, 64 bytes each) once, and every wave
// computes two 32-voxel rows (two accumulators sharing each weight fragment) reading its
// A operands from that halo for all 27 taps. The halo's 16-byte chunks are XOR-swizzled
// by voxel, chunk c of voxel v at c ^ ((v >> 2) & 3), so that any 16 consecutive voxels
// a fragment reads (256 bytes, one pass over the 64 banks) hit distinct banks; the weights' fragments are laid out with the
// lanes' columns consecutive for the same reason.
constexpr int kBz = 2, kBy = 8, kBx = 32;
constexpr int kHz = kBz + 2, kHy = kBy + 2, kHx = kBx + 2;
constexpr int kHaloVox = kHz * kHy * kHx;          // 1360 voxels, 87,040 bytes
constexpr int kTileConvThreads = 512;              // eight waves, two output rows each

__device__ __forceinline__ int halo_slot(int v, int c) {   // in 16-byte chunks
  return v * 4 + (c ^ ((v >> 2) & 3));
}

template <bool BACKWARD>
__global__ void __launch_bounds__(kTileConvThreads) conv_tile_kernel(const ConvArgs a) {
  // weights: fragment (tap, half h, k-group g) of column col at chunk ((tap * 2 + h) * 2 + g) * 32 + col
  __shared__ __attribute__((aligned(16))) u16x8 Bs[27 * 2 * 2 * kC];
  __shared__ __attribute__((aligned(16))) u16x8 Hs[kHaloVox * 4];
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const u16x8* W8 = static_cast<const u16x8*>(a.w);   // W[tap][co][ci] as 16-byte chunks of ci
  // (all of a thread's loads are issued before any is stored, so that their latencies
  // overlap instead of adding up)
  constexpr int kWChunks = 27 * 2 * 2 * kC;
  constexpr int kWIters = (kWChunks + kTileConvThreads - 1) / kTileConvThreads;
  u16x8 wv[kWIters];
  if constexpr (!BACKWARD) {
    // forward fragment (tap, h, g, col = co) is W[tap][co][16 h + 8 g ..]: one chunk
#pragma unroll
    for (int q = 0; q < kWIters; ++q) {
      const int i = tid + q * kTileConvThreads;
      const int col = i % kC, g = (i / kC) % 2, h = (i / (2 * kC)) % 2, tap = i / (4 * kC);
      if (i < kWChunks) wv[q] = W8[(tap * kC + col) * 4 + h * 2 + g];
    }
#pragma unroll
    for (int q = 0; q < kWIters; ++q)
      if (tid + q * kTileConvThreads < kWChunks) Bs[tid + q * kTileConvThreads] = wv[q];
  } else {
    // backward fragment (tap, h, g, col = ci) is W[26 - tap][16 h + 8 g ..][ci]: a column,
    // transposed through LDS (the halo's space, before the halo is loaded)
    const unsigned short* Wraw = reinterpret_cast<const unsigned short*>(Hs);
#pragma unroll
    for (int q = 0; q < kWIters; ++q)
      if (tid + q * kTileConvThreads < kWChunks) wv[q] = W8[tid + q * kTileConvThreads];
#pragma unroll
    for (int q = 0; q < kWIters; ++q)
      if (tid + q * kTileConvThreads < kWChunks) Hs[tid + q * kTileConvThreads] = wv[q];
    __syncthreads();
    for (int i = tid; i < 27 * 2 * 2 * kC; i += kTileConvThreads) {
      const int col = i % kC, g = (i / kC) % 2, h = (i / (2 * kC)) % 2, tap = i / (4 * kC);
      u16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = Wraw[((26 - tap) * kC + h * 16 + g * 8 + e) * kC + col];
      Bs[i] = v;
    }
  }
  const int D = a.d, H = a.h, Wd = a.w_dim;
  const int nbx = (Wd + kBx - 1) / kBx, nby = (H + kBy - 1) / kBy, nbz = (D + kBz - 1) / kBz;
  const long long nblocks = static_cast<long long>(a.n) * nbz * nby * nbx;
  const u16x8* X = static_cast<const u16x8*>(a.x);
  // Work-group i runs on XCD i mod kXcds: each XCD takes a contiguous range of blocks (a
  // slab of the volume), so that neighbouring blocks' halos meet in its L2.
  const long long per_xcd = (nblocks + kXcds - 1) / kXcds;
  const int xcd = static_cast<int>(blockIdx.x) % kXcds;
  const long long groups_per_xcd = (gridDim.x + kXcds - 1) / kXcds;
  for (long long j = blockIdx.x / kXcds; j < per_xcd; j += groups_per_xcd) {
  const long long blk = xcd * per_xcd + j;
  if (blk >= nblocks) break;
  long long b = blk;
  const int bx = static_cast<int>(b % nbx) * kBx;
  b /= nbx;
  const int by = static_cast<int>(b % nby) * kBy;
  b /= nby;
  const int bz = static_cast<int>(b % nbz) * kBz;
  const long long n = b / nbz;
  __syncthreads();   // the weights are staged, and every wave is done with the previous halo
  // the block's input with its halo, zero outside the volume: all of a thread's loads are
  // issued before any is stored
  constexpr int kHaloIters = (kHaloVox * 4 + kTileConvThreads - 1) / kTileConvThreads;
  u16x8 hval[kHaloIters];
#pragma unroll
  for (int q = 0; q < kHaloIters; ++q) {
    const int i = tid + q * kTileConvThreads;
    const int c = i & 3, v = i >> 2;
    const int hx = v % kHx, hy = (v / kHx) % kHy, hz = v / (kHx * kHy);
    const int x = bx - 1 + hx, y = by - 1 + hy, z = bz - 1 + hz;
    hval[q] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (i < kHaloVox * 4 && x >= 0 && x < Wd && y >= 0 && y < H && z >= 0 && z < D)
      hval[q] = X[(((n * D + z) * H + y) * static_cast<long long>(Wd) + x) * 4 + c];
  }
#pragma unroll
  for (int q = 0; q < kHaloIters; ++q) {
    const int i = tid + q * kTileConvThreads;
    if (i < kHaloVox * 4) Hs[halo_slot(i >> 2, i & 3)] = hval[q];
  }
  __syncthreads();

  const int r = lane & 31, g = lane >> 5, col = lane & 31;
  const int lz = wave >> 2, ly0 = (wave & 3) * 2;   // this wave's rows: (lz, ly0) and (lz, ly0 + 1)
  f32x16 acc[2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[m][i] = 0.0f;
#pragma unroll 3
  for (int tap = 0; tap < 27; ++tap) {
    const int oz = tap / 9, oy = (tap / 3) % 3, ox = tap % 3;   // halo offsets (tap offset + 1)
    const u16x8 b0 = Bs[((tap * 2 + 0) * 2 + g) * kC + col];
    const u16x8 b1 = Bs[((tap * 2 + 1) * 2 + g) * kC + col];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int hv = ((lz + oz) * kHy + (ly0 + m + oy)) * kHx + (r + ox);
      const u16x8 a0 = Hs[halo_slot(hv, g)];
      const u16x8 a1 = Hs[halo_slot(hv, 2 + g)];
      acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0), __builtin_bit_cast(bf16x8, b0), acc[m], 0, 0, 0);
      acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a1), __builtin_bit_cast(bf16x8, b1), acc[m], 0, 0, 0);
    }
  }
  // epilogue: lane holds column col of rows acc_row(i, lane), row = voxel x offset in the tile
  const float bcol = (!BACKWARD && a.bias) ? a.bias[col] : 0.0f;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int z = bz + lz, y = by + ly0 + m;
    if (z >= D || y >= H) continue;
    const long long rowbase = ((n * D + z) * H + y) * static_cast<long long>(Wd);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int x = bx + acc_row(i, lane);
      if (x >= Wd) continue;
      const long long e = (rowbase + x) * kC + col;
      float sv = acc[m][i];
      if constexpr (!BACKWARD) {
        sv += bcol;
        if (a.z) a.z[e] = sv;
        float y_out = a.gelu ? gelu_f(sv) : sv;
        if (a.residual) y_out += bf16_to_f32(static_cast<const unsigned short*>(a.residual)[e]);
        static_cast<unsigned short*>(a.y)[e] = f32_to_bf16(y_out);
      } else {
        if (a.residual_f32) sv += a.residual_f32[e];
        if (a.dh) a.dh[e] = sv;
        if (a.y) {
          const float gg = a.zprev ? sv * gelu_grad_f(a.zprev[e]) : sv;
          static_cast<unsigned short*>(a.y)[e] = f32_to_bf16(gg);
        }
      }
    }
  }
  }
}

// Weight gradient, dW[tap][co][ci] = sum_v dz[v][co] x[v + off(tap)][ci]: a GEMM whose K
// dimension is the voxels, while the matrix cores want eight consecutive K values per
// lane. So dz and x are first copied channel-major (x three times, shifted by dx = -1, 0,
// +1 within its row, zero past the row's ends); a row shift by (dz, dy) is then a whole
// number of rows and every operand is one aligned 16-byte load.
constexpr int kTrVox = 64;      // voxels per transpose block
constexpr int kTrThreads = 256;

__global__ void __launch_bounds__(kTrThreads) wgrad_transpose_kernel(
    const unsigned short* __restrict__ x, const unsigned short* __restrict__ dz, long long nvox,
    int w_dim, unsigned short* __restrict__ xc, unsigned short* __restrict__ dzc, float* __restrict__ db) {
  __shared__ unsigned short tx[kTrVox + 2][kC + 2];   // voxels v0 - 1 .. v0 + 64
  __shared__ unsigned short tz[kTrVox][kC + 2];
  const int tid = static_cast<int>(threadIdx.x);
  float db_part = 0.0f;
  for (long long v0 = static_cast<long long>(blockIdx.x) * kTrVox; v0 < nvox;
       v0 += static_cast<long long>(gridDim.x) * kTrVox) {
    __syncthreads();
    for (int i = tid; i < (kTrVox + 2) * kC; i += kTrThreads) {
      const long long v = v0 - 1 + i / kC;
      tx[i / kC][i % kC] = (v >= 0 && v < nvox) ? x[v * kC + i % kC] : 0;
    }
    for (int i = tid; i < kTrVox * kC; i += kTrThreads) {
      const long long v = v0 + i / kC;
      tz[i / kC][i % kC] = v < nvox ? dz[v * kC + i % kC] : 0;
    }
    __syncthreads();
    for (int i = tid; i < kC * kTrVox; i += kTrThreads) {
      const int c = i / kTrVox, jv = i % kTrVox;
      const long long v = v0 + jv;
      if (v >= nvox) continue;
      dzc[c * nvox + v] = tz[jv][c];
      const int xpos = static_cast<int>(v % w_dim);
#pragma unroll
      for (int sh = 0; sh < 3; ++sh) {
        const int xx = xpos + sh - 1;
        xc[(sh * kC + c) * nvox + v] = (xx >= 0 && xx < w_dim) ? tx[jv + sh][c] : 0;
      }
    }
    if (tid < kC)
      for (int jv = 0; jv < kTrVox && v0 + jv < nvox; ++jv) db_part += bf16_to_f32(tz[jv][tid]);
  }
  if (tid < kC && db_part != 0.0f) unsafeAtomicAdd(db + tid, db_part);
}

constexpr int kGemmThreads = 256;   // four waves; wave w owns the taps w, w + 4, ...
constexpr int kTapsPerWave = 7;

__global__ void __launch_bounds__(kGemmThreads) wgrad_gemm_kernel(
    const unsigned short* __restrict__ xc, const unsigned short* __restrict__ dzc, long long nvox,
    int d, int h, int w_dim, float* __restrict__ dw) {
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const int col = lane & 31, kg = lane >> 5;
  f32x16 acc[kTapsPerWave];
#pragma unroll
  for (int u = 0; u < kTapsPerWave; ++u)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[u][i] = 0.0f;
  const long long rows = nvox / w_dim;
  for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
    const int y = static_cast<int>(r % h), z = static_cast<int>((r / h) % d);
    for (int kb = 0; kb < w_dim / 16; ++kb) {
      const long long v0 = r * w_dim + kb * 16 + kg * 8;
      const u16x8 av = *reinterpret_cast<const u16x8*>(dzc + col * nvox + v0);
#pragma unroll
      for (int u = 0; u < kTapsPerWave; ++u) {
        const int tap = wave + 4 * u;
        if (tap >= 27) continue;
        const int oz = tap / 9 - 1, oy = (tap / 3) % 3 - 1, ox = tap % 3 - 1;
        u16x8 bv = {0, 0, 0, 0, 0, 0, 0, 0};
        if (z + oz >= 0 && z + oz < d && y + oy >= 0 && y + oy < h)
          bv = *reinterpret_cast<const u16x8*>(xc + ((ox + 1) * kC + col) * nvox + v0 +
                                              (static_cast<long long>(oz) * h + oy) * w_dim);
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc[u], 0, 0, 0);
      }
    }
  }
  // rows co (acc_row), columns ci (this lane's col)
#pragma unroll
  for (int u = 0; u < kTapsPerWave; ++u) {
    const int tap = wave + 4 * u;
    if (tap >= 27) continue;
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (acc[u][i] != 0.0f) unsafeAtomicAdd(dw + (tap * kC + acc_row(i, lane)) * kC + col, acc[u][i]);
  }
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
  // a persistent grid of one work-group per compute unit (the LDS holds one), each staging
  // the weights once and then taking blocks in turn
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ? v : 256;
  }
  const long long blocks = static_cast<long long>(a.n) * ((a.d + kBz - 1) / kBz) * ((a.h + kBy - 1) / kBy) *
                           ((a.w_dim + kBx - 1) / kBx);
  // (a multiple of the XCD count, so that every XCD's block range has its work-groups)
  const long long want = blocks < cus ? blocks : cus;
  const unsigned grid = static_cast<unsigned>((want + kXcds - 1) / kXcds * kXcds);
  if (backward) hipLaunchKernelGGL(conv_tile_kernel<true>, dim3(grid), dim3(kTileConvThreads), 0, s, a);
  else hipLaunchKernelGGL(conv_tile_kernel<false>, dim3(grid), dim3(kTileConvThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgrad(const ConvArgs& a, unsigned short* xc, unsigned short* dzc, hipStream_t s) {
  const long long nvox = static_cast<long long>(a.n) * a.d * a.h * a.w_dim;
  const int tgrid = grid_for(nvox, kTrVox);
  hipLaunchKernelGGL(wgrad_transpose_kernel, dim3(tgrid), dim3(kTrThreads), 0, s,
                     static_cast<const unsigned short*>(a.x), static_cast<const unsigned short*>(a.dz), nvox,
                     a.w_dim, xc, dzc, a.db);
  const long long rows = nvox / a.w_dim;
  const int ggrid = static_cast<int>(rows < 256 ? rows : 256);
  hipLaunchKernelGGL(wgrad_gemm_kernel, dim3(ggrid), dim3(kGemmThreads), 0, s, xc, dzc, nvox, a.d, a.h,
                     a.w_dim, a.dw);
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
