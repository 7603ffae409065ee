// Adjoint (vector-Jacobian product) of the march, for gradients with respect to j and kappa.
//
// With G = dL/dJ, a_k = exp(-kappa_k ds), E_k = exp(-tau_k) and c = 4 pi / N_Omega, the chain
// rule on Eq. (2) gives, per ray and in reverse substep order,
//   g_{k+1}    = c * sum_corners w G              (G gathered with the deposit's weights)
//   Ibar_{k+1} = g_{k+1} + Ibar_{k+2} a_{k+1}
//   dL/dj     += w * Ibar_{k+1} E_k ds            (scattered with the same weights)
//   dL/dkappa[nearest voxel] += -ds (Ibar_{k+1} I_k a_k + sum_{k'>k} Ibar_{k'+1} j_{k'} E_{k'} ds)
// The reverse sweep needs I_k, E_k, j_k and a_k again. Instead of storing trajectories, the
// forward sweep keeps (I, E) at the start of every kSeg-substep segment; the reverse sweep
// re-marches one segment forward in registers from its checkpoint, then runs the adjoint
// through it. Per-sample contributions go to workspace rows, which the tile kernel
// deposits (trilinear for dL/dj, nearest voxel for dL/dkappa) exactly like the forward field.
#include "common.h"
#include "device_common.h"

namespace rtmi {
namespace {

struct SampleAD {
  float j;      // trilinear j
  float kap;    // nearest kappa of this bin (table kappa x kscale)
  float kraw;   // nearest kappa as the table holds it
  float g;      // c * trilinear G
  int cid;      // box corner the sample has collapsed onto, or -1
};

__device__ __forceinline__ SampleAD adjoint_sample(const AdjointArgs& a, float sx, float sy,
                                                   float sz, float4 d, int k, float wray) {
  const int nx = a.nx, ny = a.ny, nz = a.nz, nyz = ny * nz;
  const float dist = sample_distance(k, a.ds);
  const float x = sample_axis(sx, dist, d.x);
  const float y = sample_axis(sy, dist, d.y);
  const float z = sample_axis(sz, dist, d.z);
  const Axis X = axis_stencil(x, nx);
  const Axis Y = axis_stencil(y, ny);
  const Axis Z = axis_stencil(z, nz);
  const int ox[2] = {X.lo * nyz, X.hi * nyz};
  const int oy[2] = {Y.lo * nz, Y.hi * nz};
  const int oz[2] = {Z.lo, Z.hi};
  const float wx[2] = {X.w0, X.w1};
  const float wy[2] = {Y.w0, Y.w1};
  const float wz[2] = {Z.w0, Z.w1};
  // j and kappa from the gather table's line of the lower corner; a collapsed axis takes
  // weight 1 on its lower corner (the table's upper corner may be another voxel there)
  const float4* line = a.med + 4ll * (static_cast<long long>(X.lo) * nyz + Y.lo * nz + Z.lo);
  const float4 j0 = line[0], j1 = line[1], k0v = line[2], k1v = line[3];
  const float jc[8] = {j0.x, j0.y, j0.z, j0.w, j1.x, j1.y, j1.z, j1.w};
  const float kc[8] = {k0v.x, k0v.y, k0v.z, k0v.w, k1v.x, k1v.y, k1v.z, k1v.w};
  const float cx[2] = {X.lo == X.hi ? 1.0f : X.w0, X.lo == X.hi ? 0.0f : X.w1};
  const float cy[2] = {Y.lo == Y.hi ? 1.0f : Y.w0, Y.lo == Y.hi ? 0.0f : Y.w1};
  const float cz[2] = {Z.lo == Z.hi ? 1.0f : Z.w0, Z.lo == Z.hi ? 0.0f : Z.w1};
  const int nsel = (X.nearest != X.lo ? 4 : 0) | (Y.nearest != Y.lo ? 2 : 0) | (Z.nearest != Z.lo ? 1 : 0);
  SampleAD r;
  r.j = 0.0f;
  r.kraw = kc[0];
  float gsum = 0.0f;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    r.j += (cx[c >> 2] * cy[(c >> 1) & 1]) * cz[c & 1] * jc[c];
    r.kraw = c == nsel ? kc[c] : r.kraw;
    gsum += (wx[c >> 2] * wy[(c >> 1) & 1]) * wz[c & 1] * a.grad[ox[c >> 2] + oy[(c >> 1) & 1] + oz[c & 1]];
  }
  r.g = wray * gsum;
  r.kap = r.kraw * a.kscale;
  const bool out3 = axis_clamped(x, nx) && axis_clamped(y, ny) && axis_clamped(z, nz);
  r.cid = out3 ? ((x >= 0.0f ? 4 : 0) | (y >= 0.0f ? 2 : 0) | (z >= 0.0f ? 1 : 0)) : -1;
  return r;
}

__global__ void __launch_bounds__(kBlock) adjoint_record_kernel(const AdjointArgs a) {
  __shared__ float ctail[2][8];
  const int tid = static_cast<int>(threadIdx.x);
  if (tid < 16) ctail[tid / 8][tid % 8] = 0.0f;
  __syncthreads();

  const int nblk = a.blk_begin[a.n_src];
  const int per_xcd = (nblk + kXcds - 1) / kXcds;
  const int blk = (static_cast<int>(blockIdx.x) % kXcds) * per_xcd + static_cast<int>(blockIdx.x) / kXcds;
  int s = 0;
  while (s + 1 < a.n_src && blk >= a.blk_begin[s + 1]) ++s;
  const int ray = (blk - a.blk_begin[s]) * kBlock + tid;
  double dsc = 0.0;   // sum of table kappa(nearest) x dL/dkappa_bin over this lane's samples
  if (blk < nblk && ray < a.nrays[s]) {
    const float4 d = a.dirs[s][ray];
    const float sx = a.sx[s], sy = a.sy[s], sz = a.sz[s];
    const float wray = a.wray[s];
    const int nsub = a.nsub[s];
    const float ds = a.ds;
    const long long vb = a.vbase[s];
    const int vn = a.nrays[s];
    float2* ck = a.ckpt + a.cbase[s] + static_cast<long long>(ray) * a.cstride[s];
    const int nseg = (nsub + kSeg - 1) / kSeg;

    // forward sweep: checkpoints only
    float I = 0.0f, E = 1.0f;
    for (int seg = 0; seg < nseg; ++seg) {
      ck[seg] = make_float2(I, E);
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int k = seg * kSeg + t;
        if (k < nsub) {
          const SampleAD q = adjoint_sample(a, sx, sy, sz, d, k, wray);
          const float att = expf(-q.kap * ds);
          I = I * att + q.j * E * ds;
          E *= att;
        }
      }
    }

    // reverse sweep, one recomputed segment at a time
    float ibar_next = 0.0f, a_next = 0.0f, suffix = 0.0f;
    float tail_j = 0.0f, tail_k = 0.0f;
    int corner = -1;
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const float2 c0 = ck[seg];
      float Ir = c0.x, Er = c0.y;
      float jk[kSeg], ak[kSeg], Ik[kSeg], Ek[kSeg], gk[kSeg], kr[kSeg];
      int cid[kSeg];
#pragma unroll
      for (int t = 0; t < kSeg; ++t) {
        const int k = min(seg * kSeg + t, nsub - 1);
        const SampleAD q = adjoint_sample(a, sx, sy, sz, d, k, wray);
        const float att = expf(-q.kap * ds);
        jk[t] = q.j;
        ak[t] = att;
        gk[t] = q.g;
        kr[t] = q.kraw;
        cid[t] = q.cid;
        Ik[t] = Ir;
        Ek[t] = Er;
        Ir = Ir * att + q.j * Er * ds;
        Er *= att;
      }
      float outj[kSeg], outk[kSeg];
#pragma unroll
      for (int t = kSeg - 1; t >= 0; --t) {
        outj[t] = 0.0f;
        outk[t] = 0.0f;
        if (seg * kSeg + t < nsub) {
          const float ibar = gk[t] + ibar_next * a_next;
          float vjv = ibar * Ek[t] * ds;
          float vkv = -ds * (ibar * Ik[t] * ak[t] + suffix);   // dL/dkappa_bin of the sample
          dsc += static_cast<double>(kr[t]) * static_cast<double>(vkv);
          vkv *= a.kgrad_scale;
          suffix += ibar * jk[t] * Ek[t] * ds;
          ibar_next = ibar;
          a_next = ak[t];
          if (cid[t] >= 0) {
            if (cid[t] != corner) {
              if (corner >= 0) {
                atomicAdd(&ctail[0][corner], tail_j);
                atomicAdd(&ctail[1][corner], tail_k);
              }
              tail_j = 0.0f;
              tail_k = 0.0f;
              corner = cid[t];
            }
            tail_j += vjv;
            tail_k += vkv;
            vjv = 0.0f;
            vkv = 0.0f;
          }
          outj[t] = vjv;
          outk[t] = vkv;
        }
      }
      const long long slot = row_slot(vb, vn, ray, seg * kSeg);
      *reinterpret_cast<float4*>(a.Vj + slot) = make_float4(outj[0], outj[1], outj[2], outj[3]);
      *reinterpret_cast<float4*>(a.Vk + slot) = make_float4(outk[0], outk[1], outk[2], outk[3]);
    }
    if (corner >= 0) {
      atomicAdd(&ctail[0][corner], tail_j);
      atomicAdd(&ctail[1][corner], tail_k);
    }
  }
  if (a.dscale) {   // (all lanes here; those without a ray hold zero)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dsc += __shfl_xor(dsc, off, 64);
    if ((tid & 63) == 0 && dsc != 0.0) atomicAdd(a.dscale, dsc);
  }
  __syncthreads();
  if (tid < 16) {
    const float v = ctail[tid / 8][tid % 8];
    if (v != 0.0f) unsafeAtomicAdd((tid < 8 ? a.corner_j : a.corner_k) + (tid % 8), v);
  }
}

// Mean-squared field error of the inverse problem and its gradient: loss[0] +=
// scale * sum (J - T)^2 (the caller's loss word is zeroed first), grad = 2 scale (J - T).
__global__ void field_mse_kernel(const float* __restrict__ field, const float* __restrict__ target,
                                 long long n, float scale, float* __restrict__ grad, float* __restrict__ loss) {
  float part = 0.0f;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x) {
    const float d = field[i] - target[i];
    part += d * d;
    grad[i] = 2.0f * scale * d;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0 && part != 0.0f) unsafeAtomicAdd(loss, part * scale);
}

__global__ void zero_word_kernel(float* p) {
  if (threadIdx.x == 0) *p = 0.0f;
}

}  // namespace

hipError_t launch_field_mse(const float* field, const float* target, long long n, float scale, float* grad,
                            float* loss, hipStream_t s) {
  long long blocks = (n + 1023) / 1024;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  hipLaunchKernelGGL(zero_word_kernel, dim3(1), dim3(64), 0, s, loss);
  hipLaunchKernelGGL(field_mse_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, field, target, n,
                     scale, grad, loss);
  return hipGetLastError();
}

namespace {
constexpr int kDotThreads = 1024;

// out[0] = sum_i a[i] b[i], by one work-group in a fixed order (binary64 partial sums), so
// the result does not depend on scheduling.
__global__ void __launch_bounds__(kDotThreads) dot_kernel(const float* __restrict__ a, const float* __restrict__ b,
                                                          long long n, float* __restrict__ out) {
  __shared__ double part[kDotThreads];
  const int tid = static_cast<int>(threadIdx.x);
  double acc = 0.0;
  for (long long i = tid; i < n; i += kDotThreads) acc += static_cast<double>(a[i]) * static_cast<double>(b[i]);
  part[tid] = acc;
  __syncthreads();
  for (int w = kDotThreads / 2; w > 0; w >>= 1) {
    if (tid < w) part[tid] += part[tid + w];
    __syncthreads();
  }
  if (tid == 0) out[0] = static_cast<float>(part[0]);
}

// out[i] = scale[0] * in[i], the scale read from device memory
__global__ void scaled_copy_kernel(const float* __restrict__ in, const float* __restrict__ scale, float* __restrict__ out,
                                   long long n) {
  const float s = scale[0];
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    out[i] = s * in[i];
}

__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int n) {
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) out[i] = static_cast<float>(in[i]);
}
}  // namespace

hipError_t launch_f64_to_f32(const double* in, float* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_dot(const float* a, const float* b, long long n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_kernel, dim3(1), dim3(kDotThreads), 0, s, a, b, n, out);
  return hipGetLastError();
}

hipError_t launch_scaled_copy(const float* in, const float* scale, float* out, long long n, hipStream_t s) {
  long long blocks = (n + 1023) / 1024;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  hipLaunchKernelGGL(scaled_copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, in, scale, out, n);
  return hipGetLastError();
}

hipError_t launch_adjoint_record(const AdjointArgs& a, int blocks, hipStream_t s) {
  const dim3 grid((blocks + kXcds - 1) / kXcds * kXcds), block(kBlock);
  hipLaunchKernelGGL(adjoint_record_kernel, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace rtmi
