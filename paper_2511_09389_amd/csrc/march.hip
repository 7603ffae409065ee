// Device code of librtmi: the per-ray emission-absorption march (Ray-trax, Sec. 2).
//
// One lane owns one ray of one source and carries up to kMaxBinsPerLaunch frequency bins
// (Sec. 2, "Frequency-bin agnosticism": bins are a batch axis). The sample point of
// substep k is evaluated in closed form, x_k = src + (k ds) n, so no lane state but
// (I, E = exp(-tau)) per bin is carried from one substep to the next.
#include <type_traits>

#include "common.h"
#include "device_common.h"

namespace rtmi {
namespace {

struct Stencil {
  int off[8];
  float w[8];
  int nearest;
};

__device__ __forceinline__ Stencil make_stencil(float x, float y, float z, int nx, int ny,
                                                int nz) {
  const Axis X = axis_stencil(x, nx);
  const Axis Y = axis_stencil(y, ny);
  const Axis Z = axis_stencil(z, nz);
  const int nyz = ny * nz;
  const int ox[2] = {X.lo * nyz, X.hi * nyz};
  const int oy[2] = {Y.lo * nz, Y.hi * nz};
  const int oz[2] = {Z.lo, Z.hi};
  const float wx[2] = {X.w0, X.w1};
  const float wy[2] = {Y.w0, Y.w1};
  const float wz[2] = {Z.w0, Z.w1};
  Stencil st;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int cx = c >> 2, cy = (c >> 1) & 1, cz = c & 1;
    st.off[c] = ox[cx] + oy[cy] + oz[cz];
    st.w[c] = (wx[cx] * wy[cy]) * wz[cz];
  }
  st.nearest = X.nearest * nyz + Y.nearest * nz + Z.nearest;
  return st;
}

// Output of one deposit slot: float atomics, or 64-bit fixed-point integer atomics.
__device__ __forceinline__ void emit(float* base, int off, float v) {
  if (v != 0.0f) unsafeAtomicAdd(base + off, v);
}
__device__ __forceinline__ void emit(unsigned long long* base, int off, long long v) {
  if (v != 0) atomicAdd(base + off, static_cast<unsigned long long>(v));
}

// Per-lane deposit window: accumulators for the 8 voxels of the ray's current (clamped)
// trilinear stencil, slot c = (cx << 2) | (cy << 1) | cz. A substep whose stencil equals
// the window's only adds to registers. When the stencil moves by one cell along an axis
// in the ray's direction, the layer the ray leaves is flushed to memory with atomics and
// the shared layer slides over; any other change flushes the whole window. Every deposit
// therefore reaches memory exactly once, summed first along the ray.
template <int NB, typename T>
struct Window {
  T acc[NB][8];
  int lo[3], hi[3];
};

template <int NB, typename T, typename OutT>
__device__ __forceinline__ void flush_slot(Window<NB, T>& w, int c, OutT* out, long long stride,
                                           int nyz, int nz) {
  const int off = ((c & 4) ? w.hi[0] : w.lo[0]) * nyz + ((c & 2) ? w.hi[1] : w.lo[1]) * nz +
                  ((c & 1) ? w.hi[2] : w.lo[2]);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    emit(out + b * stride, off, w.acc[b][c]);
    w.acc[b][c] = T(0);
  }
}

template <int A, int NB, typename T, typename OutT>
__device__ __forceinline__ void advance_axis(Window<NB, T>& w, int lo_new, int hi_new, bool up,
                                             OutT* out, long long stride, int nyz, int nz) {
  constexpr int bit = 4 >> A;
  if (lo_new == w.lo[A] && hi_new == w.hi[A]) return;
  if (up && lo_new == w.hi[A]) {
    // slide one cell up: flush the lower layer, move the upper layer down
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c & bit) continue;
      flush_slot(w, c, out, stride, nyz, nz);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        w.acc[b][c] = w.acc[b][c | bit];
        w.acc[b][c | bit] = T(0);
      }
    }
  } else if (!up && hi_new == w.lo[A]) {
    // slide one cell down: flush the upper layer, move the lower layer up
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c & bit) continue;
      flush_slot(w, c | bit, out, stride, nyz, nz);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        w.acc[b][c | bit] = w.acc[b][c];
        w.acc[b][c] = T(0);
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < 8; ++c) flush_slot(w, c, out, stride, nyz, nz);
  }
  w.lo[A] = lo_new;
  w.hi[A] = hi_new;
}

template <int NB, bool SHARED_J, bool DET>
__global__ void __launch_bounds__(kBlock) march_kernel(const MarchArgs a) {
  using T = typename std::conditional<DET, long long, float>::type;
  using OutT = typename std::conditional<DET, unsigned long long, float>::type;

  const int blk = blockIdx.x;
  int s = 0;
  while (s + 1 < a.n_src && blk >= a.blk_begin[s + 1]) ++s;
  const int ray = (blk - a.blk_begin[s]) * kBlock + static_cast<int>(threadIdx.x);
  if (ray >= a.nrays[s]) return;

  const float4 d = a.dirs[s][ray];
  const float sx = a.sx[s], sy = a.sy[s], sz = a.sz[s];
  const float wray = a.wray[s];
  const int nsub = a.nsub[s];
  const float ds = a.ds;
  const int nx = a.nx, ny = a.ny, nz = a.nz, nyz = ny * nz;
  const bool shared_k = (a.k_stride == 0);
  const bool up[3] = {d.x >= 0.0f, d.y >= 0.0f, d.z >= 0.0f};
  OutT* out;
  double det_scale = 0.0;
  if constexpr (DET) {
    out = a.acc;
    det_scale = *a.det_scale;
  } else {
    out = a.out;
  }

  float I[NB], E[NB];
  Window<NB, T> win;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    I[b] = 0.0f;
    E[b] = 1.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) win.acc[b][c] = T(0);
  }
  win.lo[0] = win.hi[0] = win.lo[1] = win.hi[1] = win.lo[2] = win.hi[2] = -1;

  for (int k = 0; k < nsub; ++k) {
    const float t = __fmul_rn(static_cast<float>(k), ds);
    const Axis X = axis_stencil(sample_axis(sx, t, d.x), nx);
    const Axis Y = axis_stencil(sample_axis(sy, t, d.y), ny);
    const Axis Z = axis_stencil(sample_axis(sz, t, d.z), nz);
    const int ox[2] = {X.lo * nyz, X.hi * nyz};
    const int oy[2] = {Y.lo * nz, Y.hi * nz};
    const int oz[2] = {Z.lo, Z.hi};
    const float wx[2] = {X.w0, X.w1};
    const float wy[2] = {Y.w0, Y.w1};
    const float wz[2] = {Z.w0, Z.w1};
    int off[8];
    float wt[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      off[c] = ox[c >> 2] + oy[(c >> 1) & 1] + oz[c & 1];
      wt[c] = (wx[c >> 2] * wy[(c >> 1) & 1]) * wz[c & 1];
    }
    const int nearest = X.nearest * nyz + Y.nearest * nz + Z.nearest;

    // gather j (trilinear) and kappa (nearest voxel) at x_k
    float jk[NB];
    if constexpr (SHARED_J) {
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < 8; ++c) acc += wt[c] * a.j[off[c]];
#pragma unroll
      for (int b = 0; b < NB; ++b) jk[b] = acc;
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float* jb = a.j + b * a.j_stride;
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) acc += wt[c] * jb[off[c]];
        jk[b] = acc;
      }
    }
    const float k0 = shared_k ? a.kap[nearest] : 0.0f;

    // move the deposit window onto this substep's stencil
    advance_axis<0>(win, X.lo, X.hi, up[0], out, a.out_stride, nyz, nz);
    advance_axis<1>(win, Y.lo, Y.hi, up[1], out, a.out_stride, nyz, nz);
    advance_axis<2>(win, Z.lo, Z.hi, up[2], out, a.out_stride, nyz, nz);

#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float kap = shared_k ? k0 * a.kscale[b] : a.kap[b * a.k_stride + nearest];
      const float att = expf(-kap * ds);
      // Eq. (2): emission uses exp(-tau_k) from before this step's attenuation.
      I[b] = I[b] * att + jk[b] * E[b] * ds;
      E[b] *= att;
      const float v = wray * I[b];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        if constexpr (DET)
          win.acc[b][c] += __double2ll_rn(static_cast<double>(v * wt[c]) * det_scale);
        else
          win.acc[b][c] += v * wt[c];
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) flush_slot(win, c, out, a.out_stride, nyz, nz);
}

// Per-ray trace of one source: I_{k+1} and tau_{k+1} for every substep, lattice order.
__global__ void __launch_bounds__(kBlock) debug_kernel(const DebugArgs a) {
  const int lane = blockIdx.x * kBlock + static_cast<int>(threadIdx.x);
  if (lane >= a.nrays) return;
  const float4 d = a.dirs[lane];
  const long long row = static_cast<long long>(__float_as_int(d.w)) * a.nsub;
  float I = 0.0f, E = 1.0f, tau = 0.0f;
  for (int k = 0; k < a.nsub; ++k) {
    const float t = __fmul_rn(static_cast<float>(k), a.ds);
    const Stencil st = make_stencil(sample_axis(a.sx, t, d.x), sample_axis(a.sy, t, d.y),
                                    sample_axis(a.sz, t, d.z), a.nx, a.ny, a.nz);
    float jk = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) jk += st.w[c] * a.j[st.off[c]];
    const float kap = a.kap[st.nearest];
    const float att = expf(-kap * a.ds);
    I = I * att + jk * E * a.ds;
    E *= att;
    tau += kap * a.ds;
    a.out_rays[row + k] = I;
    if (a.out_tau) a.out_tau[row + k] = tau;
  }
}

__global__ void fill_zero_kernel(float* p, long long n) {
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride)
    p[i] = 0.0f;
}

__global__ void fill_zero_u64_kernel(unsigned long long* p, long long n) {
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride)
    p[i] = 0ull;
}

// max |j| as the bit pattern of a non-negative float (ordered like the value).
__global__ void absmax_kernel(const float* j, long long n, unsigned int* out_bits) {
  __shared__ unsigned int red[kBlock];
  unsigned int m = 0u;
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride)
    m = max(m, __float_as_uint(fabsf(j[i])));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out_bits, red[0]);
}

// max(0, -kappa) as the bit pattern of a non-negative float.
__global__ void negmax_kernel(const float* k, long long n, unsigned int* out_bits) {
  __shared__ unsigned int red[kBlock];
  unsigned int m = 0u;
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride)
    m = max(m, __float_as_uint(fmaxf(0.0f, -k[i])));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out_bits, red[0]);
}

// scale = largest power of two with bound * scale <= 2^62 (1 when the bound is 0 or not finite).
// bits[0]: max |j|; bits[1]: max(0, -kappa).
__global__ void det_scale_kernel(const unsigned int* bits, double growth_per_neg_kappa,
                                 double bound_per_unit_j, double* scale) {
  const double neg = static_cast<double>(__uint_as_float(bits[1]));
  const double growth = neg > 0.0 ? exp(fmin(700.0, neg * growth_per_neg_kappa)) : 1.0;
  const double bound = static_cast<double>(__uint_as_float(bits[0])) * bound_per_unit_j * growth;
  double sc = 1.0;
  if (bound > 0.0 && isfinite(bound)) sc = exp2(floor(62.0 - log2(bound)));
  *scale = sc;
}

__global__ void det_convert_kernel(const unsigned long long* acc, const double* scale,
                                   float* out, long long n) {
  const double inv = 1.0 / *scale;
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += stride)
    out[i] = static_cast<float>(static_cast<double>(static_cast<long long>(acc[i])) * inv);
}

int fill_blocks(long long n) {
  long long b = (n + kBlock * 4 - 1) / (kBlock * 4);
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return static_cast<int>(b);
}

template <int NB>
hipError_t launch_nb(const MarchArgs& a, bool shared_j, bool det, int n_blocks, hipStream_t s) {
  const dim3 grid(n_blocks), block(kBlock);
  if (shared_j) {
    if (det) hipLaunchKernelGGL((march_kernel<NB, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((march_kernel<NB, true, false>), grid, block, 0, s, a);
  } else {
    if (det) hipLaunchKernelGGL((march_kernel<NB, false, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((march_kernel<NB, false, false>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_march(const MarchArgs& a, int n_bins, bool shared_j, bool det, int n_blocks,
                        hipStream_t s) {
  switch (n_bins) {
    case 1: return launch_nb<1>(a, shared_j, det, n_blocks, s);
    case 2: return launch_nb<2>(a, shared_j, det, n_blocks, s);
    case 3: return launch_nb<3>(a, shared_j, det, n_blocks, s);
    case 4: return launch_nb<4>(a, shared_j, det, n_blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_debug(const DebugArgs& a, hipStream_t s) {
  const int blocks = (a.nrays + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(debug_kernel, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero_u64(unsigned long long* p, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_u64_kernel, dim3(fill_blocks(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_det_scale(const float* j, long long j_count, const float* kap, long long k_count,
                            double growth_per_neg_kappa, double bound_per_unit_j, double* scale_out,
                            hipStream_t s) {
  // scale_out[0] receives the scale; the word after it holds the max-|j| and max(0, -kappa) bits.
  unsigned int* bits = reinterpret_cast<unsigned int*>(scale_out + 1);
  hipLaunchKernelGGL(fill_zero_u64_kernel, dim3(1), dim3(kBlock), 0, s,
                     reinterpret_cast<unsigned long long*>(bits), 1ll);
  hipLaunchKernelGGL(absmax_kernel, dim3(fill_blocks(j_count)), dim3(kBlock), 0, s, j, j_count,
                     bits);
  hipLaunchKernelGGL(negmax_kernel, dim3(fill_blocks(k_count)), dim3(kBlock), 0, s, kap, k_count,
                     bits + 1);
  hipLaunchKernelGGL(det_scale_kernel, dim3(1), dim3(1), 0, s, bits, growth_per_neg_kappa,
                     bound_per_unit_j, scale_out);
  return hipGetLastError();
}

hipError_t launch_det_convert(const unsigned long long* acc, const double* scale, float* out,
                              long long n, hipStream_t s) {
  hipLaunchKernelGGL(det_convert_kernel, dim3(fill_blocks(n)), dim3(kBlock), 0, s, acc, scale,
                     out, n);
  return hipGetLastError();
}

}  // namespace rtmi
