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
// channel-major LDS copies of dz and of x (three, shifted by dx = -1, 0, +1), so that a
// row shift is a whole number of rows and every operand an aligned 16-byte read.
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

// Weight gradient, dW[tap][co][ci] = sum_v dz[v][co] x[v + off(tap)][ci]: 27 GEMMs of 32 x 32
// whose K dimension is the voxels, while the matrix cores want eight consecutive K values
// per lane for one channel. wgrad_tile_kernel: a persistent work-group of eight waves takes
// blocks of 1 (z) x 4 (y) x 32 (x) voxels in turn and stages them channel-major in LDS: dz
// once, and x with its one-voxel halo in z and y three times, shifted by dx = -1, 0, +1, so
// that every operand of every tap is one aligned 16-byte LDS read. Wave w accumulates the
// taps w, w + 8, w + 16 (and w + 24) over all its blocks; at the end every work-group writes
// its partial sums (and its dz channel sums for db), and wgrad_reduce_kernel adds them up,
// in a fixed order, into dw and db. Channel rows are padded by one 16-byte chunk (17 per dz
// row, 73 per x plane), so that the 16 lanes of one read pass fall on distinct banks.
constexpr int kWgY = 4, kWgX = 32;
constexpr int kWgVox = kWgY * kWgX;                      // 128 voxels: 8 K steps of 16
constexpr int kWgDzRow = kWgVox / 8 + 1;                 // 17 chunks per dz channel
constexpr int kWgHz = 3, kWgHy = kWgY + 2;               // staged x rows: 3 z x 6 y of 32
constexpr int kWgXPlane = kWgHz * kWgHy * (kWgX / 8) + 1;   // 73 chunks per (shift, channel)
constexpr int kWgThreads = 512;
constexpr int kWgTapsPerWave = 4;
constexpr int kWgPartial = 27 * kC * kC + kC;            // floats of one work-group's partial sums

__global__ void __launch_bounds__(kWgThreads) wgrad_tile_kernel(const ConvArgs a, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) u16x8 dzT[kC * kWgDzRow];
  __shared__ __attribute__((aligned(16))) u16x8 xS[3 * kC * kWgXPlane];
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63, wave = tid >> 6;
  const int D = a.d, H = a.h, Wd = a.w_dim;
  const int nby = (H + kWgY - 1) / kWgY, nbx = (Wd + kWgX - 1) / kWgX;
  const long long nblocks = static_cast<long long>(a.n) * D * nby * nbx;
  const u16x8* X = static_cast<const u16x8*>(a.x);
  const u16x8* DZ = static_cast<const u16x8*>(a.dz);
  f32x16 acc[kWgTapsPerWave];
#pragma unroll
  for (int u = 0; u < kWgTapsPerWave; ++u)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[u][i] = 0.0f;
  float dbp[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // a dz task: sums of its 8 channels
  const int m = lane & 31, g = lane >> 5;
  const int wave_s = __builtin_amdgcn_readfirstlane(wave);   // (uniform: taps in scalar registers)
  const int taps = (27 - wave_s + 7) / 8;                     // taps wave, wave + 8, ... below 27

  // Staging runs as tasks of 8 consecutive voxels x 8 channels: a task loads them (16 bytes
  // per voxel), transposes the 8 x 8 block in registers and writes one 16-byte chunk per
  // channel, 8 voxels of it. A task's bits are ordered (j, row, cq: x group lowest) so that
  // the 16 lanes of one write pass fall on distinct banks. The global data of a block is
  // fetched one block ahead, so that its latency overlaps the previous block's products.
  constexpr int kDzTasks = kWgY * 4 * (kWgX / 8);            // 64: 4 rows x 4 channel groups x 4 x-groups
  constexpr int kXRows = kWgHz * kWgHy;                      // 18 staged x rows
  constexpr int kXTasks = kXRows * 4 * (kWgX / 8);           // 288
  static_assert(kDzTasks + kXTasks <= kWgThreads, "one staging task per thread");
  // (an x task reads voxels 8 j - 1 .. 8 j + 8 of its row: ten, for the three shifted copies)
  u16x8 ld[10];
  int t_row = 0, t_cq = 0, t_j = 0;
  const bool dz_task = tid < kDzTasks, x_task = !dz_task && tid < kDzTasks + kXTasks;
  {
    const int t = dz_task ? tid : tid - kDzTasks;
    t_j = t & 3;
    t_cq = ((t >> 3) & 1) | (((t >> 4) & 1) << 1);
    t_row = ((t >> 2) & 1) | ((t >> 5) << 1);
  }
  auto fetch = [&](long long blk) {
    long long b = blk;
    const int bx = static_cast<int>(b % nbx) * kWgX;
    b /= nbx;
    const int by = static_cast<int>(b % nby) * kWgY;
    b /= nby;
    const int bz = static_cast<int>(b % D);
    const long long n = b / D;
#pragma unroll
    for (int k = 0; k < 10; ++k) ld[k] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (blk >= nblocks) return;
    if (dz_task) {   // dz row t_row, voxels 8 t_j .. + 8, zero outside the volume
      const int y = by + t_row;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int x = bx + 8 * t_j + k;
        if (y < H && x < Wd) ld[k] = DZ[(((n * D + bz) * H + y) * static_cast<long long>(Wd) + x) * 4 + t_cq];
      }
    } else if (x_task) {   // x row (z, y) = t_row (3 z x 6 y, from bz - 1, by - 1), voxels bx - 1 + 8 t_j + k
      const int z = bz - 1 + t_row / kWgHy, y = by - 1 + t_row % kWgHy;
      if (z >= 0 && z < D && y >= 0 && y < H) {
#pragma unroll
        for (int k = 0; k < 10; ++k) {
          const int x = bx - 1 + 8 * t_j + k;
          if (x >= 0 && x < Wd) ld[k] = X[(((n * D + z) * H + y) * static_cast<long long>(Wd) + x) * 4 + t_cq];
        }
      }
    }
  };
  // the 8 x 8 transpose: channel e of voxels ld[base .. base + 8)
  auto column = [&](int base, int e) -> u16x8 {
    u16x8 c;
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = ld[base + k][e];
    return c;
  };
  fetch(blockIdx.x);
  for (long long blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    __syncthreads();   // every wave is done with the previous block
    if (dz_task) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const u16x8 c = column(0, e);
        dzT[(8 * t_cq + e) * kWgDzRow + t_row * 4 + t_j] = c;
#pragma unroll
        for (int k = 0; k < 8; ++k) dbp[e] += bf16_to_f32(c[k]);
      }
    } else if (x_task) {
      // copy s holds x[bx + xi + s - 1] at xi: for xi = 8 t_j + k that is ld[k + s]
#pragma unroll
      for (int sh = 0; sh < 3; ++sh)
#pragma unroll
        for (int e = 0; e < 8; ++e)
          xS[(sh * kC + 8 * t_cq + e) * kWgXPlane + t_row * 4 + t_j] = column(sh, e);
    }
    __syncthreads();
    fetch(blk + gridDim.x);   // (past the last block: nothing read)

    // Two K steps at a time: all their operands are read before the products that use them
    // (the fourth tap of the waves that have only three reads a valid slot and is not used).
#pragma unroll
    for (int step = 0; step < kWgVox / 16; step += 2) {
      u16x8 av[2], bv[2][kWgTapsPerWave];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int r = (step + q) >> 1, h = (step + q) & 1;
        av[q] = dzT[m * kWgDzRow + r * 4 + 2 * h + g];
#pragma unroll
        for (int u = 0; u < kWgTapsPerWave; ++u) {
          const int tap = min(wave_s + 8 * u, 26);
          const int oz = tap / 9, oy = (tap / 3) % 3, ox = tap % 3;   // offsets + 1
          bv[q][u] = xS[(ox * kC + m) * kWgXPlane + (oz * kWgHy + r + oy) * 4 + 2 * h + g];
        }
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < kWgTapsPerWave; ++u)
          if (u < taps)
            acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, av[q]),
                                                             __builtin_bit_cast(bf16x8, bv[q][u]), acc[u], 0, 0, 0);
    }
  }
  // partial sums: rows co (acc_row), columns ci (this lane's column); then the dz channel sums
  float* mine = part + static_cast<long long>(blockIdx.x) * kWgPartial;
#pragma unroll
  for (int u = 0; u < kWgTapsPerWave; ++u) {
    const int tap = wave + 8 * u;
    if (tap >= 27) continue;
#pragma unroll
    for (int i = 0; i < 16; ++i) mine[(tap * kC + acc_row(i, lane)) * kC + m] = acc[u][i];
  }
  __syncthreads();
  float* red = reinterpret_cast<float*>(xS);   // (the staging space, free now): [dz task][8]
  if (dz_task) {
#pragma unroll
    for (int e = 0; e < 8; ++e) red[tid * 8 + e] = dbp[e];
  }
  __syncthreads();
  if (tid < kC) {   // channel tid = 8 cq + e: the dz tasks of channel group cq, in task order
    float sdb = 0.0f;
    for (int t = 0; t < kDzTasks; ++t) {
      const int cq = ((t >> 3) & 1) | (((t >> 4) & 1) << 1);
      if (cq == tid / 8) sdb += red[t * 8 + tid % 8];
    }
    mine[27 * kC * kC + tid] = sdb;
  }
}

// dw[i] += sum over the work-groups' partials of element i (and db), in a fixed order: 16
// lanes per element each sum the partials of every 16th work-group, then the 16 sums are
// added in lane order. (Many short independent sums keep enough loads in flight.)
constexpr int kRedSlices = 16, kRedElems = 16;

__global__ void __launch_bounds__(kRedSlices * kRedElems) wgrad_reduce_kernel(const float* __restrict__ part,
                                                                             int groups, float* __restrict__ dw,
                                                                             float* __restrict__ db) {
  __shared__ float sums[kRedSlices][kRedElems];
  const int e = static_cast<int>(threadIdx.x) % kRedElems, slice = static_cast<int>(threadIdx.x) / kRedElems;
  const int i = static_cast<int>(blockIdx.x) * kRedElems + e;
  float s = 0.0f;
  if (i < kWgPartial)
    for (int q = slice; q < groups; q += kRedSlices) s += part[static_cast<long long>(q) * kWgPartial + i];
  sums[slice][e] = s;
  __syncthreads();
  if (slice == 0 && i < kWgPartial) {
    float t = 0.0f;
#pragma unroll
    for (int q = 0; q < kRedSlices; ++q) t += sums[q][e];
    if (i < 27 * kC * kC) dw[i] += t;
    else db[i - 27 * kC * kC] += t;
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

int wgrad_groups(const ConvArgs& a) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ? v : 256;
  }
  const long long blocks = static_cast<long long>(a.n) * a.d * ((a.h + kWgY - 1) / kWgY) * ((a.w_dim + kWgX - 1) / kWgX);
  return static_cast<int>(blocks < cus ? blocks : cus);
}

size_t wgrad_scratch_bytes(const ConvArgs& a) { return size_t(wgrad_groups(a)) * kWgPartial * sizeof(float); }

hipError_t launch_wgrad(const ConvArgs& a, float* part, hipStream_t s) {
  const int groups = wgrad_groups(a);
  hipLaunchKernelGGL(wgrad_tile_kernel, dim3(groups), dim3(kWgThreads), 0, s, a, part);
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((kWgPartial + kRedElems - 1) / kRedElems), dim3(kRedSlices * kRedElems), 0,
                     s, part, groups, a.dw, a.db);
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
