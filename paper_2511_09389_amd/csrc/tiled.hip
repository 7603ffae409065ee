// Two-phase (output-stationary) march of librtmi.
//
// Phase 1, record_kernel: one lane per ray runs the recurrence of Eq. (2) and writes the
// deposit value v_k = (4 pi / N_Omega) I_{k+1} of every substep to a workspace row, in
// whole 32-byte pieces; gathers for a chunk of substeps are issued together and waited
// for once. Samples whose stencil has collapsed onto a single corner voxel of the box
// (outside along all three axes) are summed per lane and reduced per corner instead.
//
// Phase 2, tile_kernel: one work-group owns a 16^3 tile of the output. Beforehand, and
// from the geometry alone, every (source, 64-ray patch) whose swept bounding box reaches
// the tile has each lane find the substep range of its ray that can touch the tile (the
// tile widened by the stencil and, on the box faces, extended to infinity to catch
// clamped samples); that range becomes chunk records of up to 8 substeps, grouped by
// tile. The tile's lanes then stream through its records, recompute the same binary32
// sample points and add v_k times the trilinear weights of the corners inside the tile
// to a binary64 LDS accumulator. The tile is then stored with plain coalesced writes.
// No global float atomics are used for the field.
#include <type_traits>

#include "common.h"
#include "device_common.h"

namespace rtmi {
namespace {

constexpr float kBig = 1.0e30f;
constexpr int kCacheDevices = 64;
constexpr float kCosConeLimit = -0.99913515f;   // cos(3.1)

// The gather table of a shared j and a shared (unscaled) kappa: for every voxel (x, y, z),
// the eight corners (x + cx, y + cy, z + cz), clamped to the box, of j and then of kappa,
// 64 bytes (one cache line) per voxel, corner c = (cx << 2) | (cy << 1) | cz. A sample
// reads its stencil and its nearest kappa (always one of the corners) from the one line of
// its lower corner: four lines per sample become one. The lines of the voxels on the upper
// faces repeat clamped corners; a collapsed axis (lower = upper corner) takes weight 1 on
// its lower corner.
__global__ void cell_table_kernel(const float* __restrict__ j, const float* __restrict__ kap,
                                  float4* __restrict__ table, int nx, int ny, int nz) {
  // four lanes per voxel, one 16-byte quarter of its line each (j corners 0-3, 4-7, then
  // kappa corners 0-3, 4-7), so a wavefront's stores are one contiguous kilobyte
  const long long cells = static_cast<long long>(nx) * ny * nz;
  const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
  for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < 4 * cells; i += stride) {
    const long long v = i >> 2;
    const int q = static_cast<int>(i & 3);
    const int z = static_cast<int>(v % nz), y = static_cast<int>((v / nz) % ny);
    const int x = static_cast<int>(v / (static_cast<long long>(ny) * nz));
    const float* src = (q < 2) ? j : kap;
    const int cx = q & 1;   // corners 4 (q & 1) .. 4 (q & 1) + 3 share cx
    const long long xx = min(x + cx, nx - 1);
    float f[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int yy = min(y + (c >> 1), ny - 1), zz = min(z + (c & 1), nz - 1);
      f[c] = src[(xx * ny + yy) * nz + zz];
    }
    table[i] = make_float4(f[0], f[1], f[2], f[3]);
  }
}

// MED == 1: j and kappa come from the gather table a.med (one 64-byte line per sample).
// MED == 2: from the rows of the gather pass, a.jk (8 bytes per sample, a ray's chunk in
// one 64-byte piece); a sample collapsed onto a box-corner voxel, which no tile lists,
// reads that voxel of the maps.
template <int NB, bool SHARED_J, bool DET, int MED>
__global__ void __launch_bounds__(kBlock) record_kernel(const RecordArgs a) {
  constexpr int C = SHARED_J ? 8 : 4;
  __shared__ float ctail[NB][8];
  __shared__ unsigned long long ctail_q[NB][8];
  const int tid = static_cast<int>(threadIdx.x);
  if (tid < NB * 8) {
    ctail[tid / 8][tid % 8] = 0.0f;
    ctail_q[tid / 8][tid % 8] = 0ull;
  }
  __syncthreads();

  // Work-group i runs on XCD i mod kXcds and takes the (i / kXcds)-th block of that XCD's
  // group of sources (their rays then share the XCD's L2), most costly blocks first.
  const int xcd = static_cast<int>(blockIdx.x) % kXcds;
  const int blk = static_cast<int>(blockIdx.x) / kXcds;
  const bool have = blk < a.xcd_blocks[xcd];
  SrcRec S{};
  if (have) {   // the group's last source whose first block is <= blk
    int lo = a.xcd_src[xcd], hi = a.xcd_src[xcd + 1];
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.src[mid].blk_begin <= blk) lo = mid;
      else hi = mid;
    }
    S = a.src[lo];
  }
  // blocks of a source: run-major, then ray blocks
  const int rblocks = (S.nrays + kBlock - 1) / kBlock;
  const int seg = (a.seg_len > 0 && rblocks > 0) ? (blk - S.blk_begin) / rblocks : 0;
  const int ray = ((blk - S.blk_begin) - seg * rblocks) * kBlock + tid;
  if (have && ray < S.nrays) {
    const float4 d = S.dirs[ray];
    const float sx = S.sx, sy = S.sy, sz = S.sz;
    const float wray = S.wray;
    const int k_begin = a.seg_len > 0 ? seg * a.seg_len : 0;
    const int nsub = a.seg_len > 0 ? min(S.nsub, k_begin + a.seg_len) : S.nsub;   // run end
    const float ds = a.ds;
    const int nx = a.nx, ny = a.ny, nz = a.nz, nyz = ny * nz;
    const bool shared_k = (a.k_stride == 0);
    const long long vb = S.vbase;
    const int vn = S.nrays;
    // runs after the first keep their attenuation P_k, and their samples collapsed onto a
    // box corner are summed by the fixup, which knows the entry state
    float* prow = seg > 0 ? a.P : nullptr;
    const bool tails_here = seg == 0;
    double det_scale = 0.0;
    if constexpr (DET) det_scale = *a.det_scale;

    float I[NB], E[NB], tail[NB];
    long long tail_q[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      I[b] = 0.0f;
      E[b] = 1.0f;
      tail[b] = 0.0f;
      tail_q[b] = 0;
    }
    int corner = -1;
    // A chunk's values are stored only after the next chunk's gathers have been issued:
    // loads and stores share one counter, so the wait for those gathers then also
    // covers stores that were in flight at the same time, not one round trip later.
    float vprev[C][NB];
    int kprev = -1;
    // Settle the loads above (direction, scale) here, once: otherwise the wait for them is
    // placed at the loop head and every iteration also waits for the previous stores.
    __builtin_amdgcn_s_waitcnt(0);

    float pprev[C][NB];
    for (int k0 = k_begin; k0 < nsub; k0 += C) {
      float jv[C][NB][8];
      float kv[C][NB];
      float fx[C], fy[C], fz[C];
      int cid[C];
      float2 rowjk[C];
      if constexpr (MED == 2) {   // (k0 is a multiple of 8 and rows are padded to whole chunks)
        const float4* q = reinterpret_cast<const float4*>(a.jk + row_slot(vb, vn, ray, k0));
#pragma unroll
        for (int h = 0; h < C / 2; ++h) {
          const float4 f = q[h];
          rowjk[2 * h] = make_float2(f.x, f.y);
          rowjk[2 * h + 1] = make_float2(f.z, f.w);
        }
      }
      // issue every gather of the chunk before using any of them
#pragma unroll
      for (int t = 0; t < C; ++t) {
        const int k = min(k0 + t, nsub - 1);
        const float dist = sample_distance(k, ds);
        const float x = sample_axis(sx, dist, d.x);
        const float y = sample_axis(sy, dist, d.y);
        const float z = sample_axis(sz, dist, d.z);
        const Axis X = axis_stencil(x, nx);
        const Axis Y = axis_stencil(y, ny);
        const Axis Z = axis_stencil(z, nz);
        const int ox[2] = {X.lo * nyz, X.hi * nyz};
        const int oy[2] = {Y.lo * nz, Y.hi * nz};
        const int oz[2] = {Z.lo, Z.hi};
        if constexpr (MED == 2) {
          float2 q = rowjk[t];
          if (axis_clamped(x, nx) && axis_clamped(y, ny) && axis_clamped(z, nz)) {
            const int v = X.lo * nyz + Y.lo * nz + Z.lo;
            q = make_float2(a.j[v], a.kap[v]);
          }
          jv[t][0][0] = q.x;
          kv[t][0] = q.y;
        } else if constexpr (MED == 1) {
          const float4* line = a.med + 4ll * (static_cast<long long>(X.lo) * nyz + Y.lo * nz + Z.lo);
          const float4 j0 = line[0], j1 = line[1], k0v = line[2], k1v = line[3];
          jv[t][0][0] = j0.x;
          jv[t][0][1] = j0.y;
          jv[t][0][2] = j0.z;
          jv[t][0][3] = j0.w;
          jv[t][0][4] = j1.x;
          jv[t][0][5] = j1.y;
          jv[t][0][6] = j1.z;
          jv[t][0][7] = j1.w;
          const int nsel = (X.nearest != X.lo ? 4 : 0) | (Y.nearest != Y.lo ? 2 : 0) | (Z.nearest != Z.lo ? 1 : 0);
          const float kc[8] = {k0v.x, k0v.y, k0v.z, k0v.w, k1v.x, k1v.y, k1v.z, k1v.w};
          float kn = kc[0];
#pragma unroll
          for (int q = 1; q < 8; ++q) kn = q == nsel ? kc[q] : kn;
          kv[t][0] = kn;
        } else {
          const int nearest = X.nearest * nyz + Y.nearest * nz + Z.nearest;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if (SHARED_J && b > 0) break;
            const float* jb = a.j + b * a.j_stride;
#pragma unroll
            for (int c = 0; c < 8; ++c) jv[t][b][c] = jb[ox[c >> 2] + oy[(c >> 1) & 1] + oz[c & 1]];
          }
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            if (shared_k && b > 0) break;
            kv[t][b] = a.kap[b * a.k_stride + nearest];
          }
        }
        // (the gather table's upper corner of a collapsed axis may be another voxel)
        fx[t] = (MED != 0 && X.lo == X.hi) ? 0.0f : X.w1;
        fy[t] = (MED != 0 && Y.lo == Y.hi) ? 0.0f : Y.w1;
        fz[t] = (MED != 0 && Z.lo == Z.hi) ? 0.0f : Z.w1;
        const bool out3 = axis_clamped(x, nx) && axis_clamped(y, ny) && axis_clamped(z, nz);
        cid[t] = out3 ? ((x >= 0.0f ? 4 : 0) | (y >= 0.0f ? 2 : 0) | (z >= 0.0f ? 1 : 0)) : -1;
      }
      if (kprev >= 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          float4* dst = reinterpret_cast<float4*>(a.V + b * a.v_bin_stride + row_slot(vb, vn, ray, kprev));
#pragma unroll
          for (int q = 0; q < C / 4; ++q)
            dst[q] = make_float4(vprev[4 * q][b], vprev[4 * q + 1][b], vprev[4 * q + 2][b],
                                 vprev[4 * q + 3][b]);
          if (prow) {
            float4* pdst = reinterpret_cast<float4*>(prow + b * a.v_bin_stride + row_slot(vb, vn, ray, kprev));
#pragma unroll
            for (int q = 0; q < C / 4; ++q)
              pdst[q] = make_float4(pprev[4 * q][b], pprev[4 * q + 1][b], pprev[4 * q + 2][b],
                                    pprev[4 * q + 3][b]);
          }
        }
      }
      float vout[C][NB], pout[C][NB];
#pragma unroll
      for (int t = 0; t < C; ++t) {
        const float wx[2] = {1.0f - fx[t], fx[t]};
        const float wy[2] = {1.0f - fy[t], fy[t]};
        const float wz[2] = {1.0f - fz[t], fz[t]};
        float jk[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int bj = SHARED_J ? 0 : b;
          if constexpr (MED == 2) {
            jk[b] = jv[t][0][0];
          } else {
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              acc += (wx[c >> 2] * wy[(c >> 1) & 1]) * wz[c & 1] * jv[t][bj][c];
            jk[b] = acc;
          }
        }
        const bool live = (k0 + t) < nsub;
        const bool collapsed = tails_here && live && cid[t] >= 0;
        // A ray can pass several corner regions (a source outside the box, a ray that
        // misses it): hand the running sum over whenever the corner changes.
        if (collapsed && cid[t] != corner) {
          if (corner >= 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              if constexpr (DET)
                atomicAdd(&ctail_q[b][corner], static_cast<unsigned long long>(tail_q[b]));
              else
                atomicAdd(&ctail[b][corner], tail[b]);
              tail[b] = 0.0f;
              tail_q[b] = 0;
            }
          }
          corner = cid[t];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const float kap = shared_k ? kv[t][0] * a.kscale[b] : kv[t][b];
          const float att = expf(-kap * ds);
          // Eq. (2): emission uses exp(-tau_k) from before this step's attenuation.
          const float In = I[b] * att + jk[b] * E[b] * ds;
          const float En = E[b] * att;
          I[b] = live ? In : I[b];
          E[b] = live ? En : E[b];
          float v = wray * I[b];
          if (collapsed) {
            if constexpr (DET)
              tail_q[b] += __double2ll_rn(static_cast<double>(v) * det_scale);
            else
              tail[b] += v;
            v = 0.0f;
          }
          vout[t][b] = live ? v : 0.0f;
          pout[t][b] = live ? E[b] : 0.0f;
        }
      }
#pragma unroll
      for (int t = 0; t < C; ++t)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          vprev[t][b] = vout[t][b];
          pprev[t][b] = pout[t][b];
        }
      kprev = k0;
    }
    // the last chunk, in whole 16-byte pieces (rows are padded to a multiple of 8 substeps)
    if (kprev >= 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        float4* dst = reinterpret_cast<float4*>(a.V + b * a.v_bin_stride + row_slot(vb, vn, ray, kprev));
#pragma unroll
        for (int q = 0; q < C / 4; ++q)
          dst[q] = make_float4(vprev[4 * q][b], vprev[4 * q + 1][b], vprev[4 * q + 2][b],
                               vprev[4 * q + 3][b]);
        if (prow) {
          float4* pdst = reinterpret_cast<float4*>(prow + b * a.v_bin_stride + row_slot(vb, vn, ray, kprev));
#pragma unroll
          for (int q = 0; q < C / 4; ++q)
            pdst[q] = make_float4(pprev[4 * q][b], pprev[4 * q + 1][b], pprev[4 * q + 2][b],
                                  pprev[4 * q + 3][b]);
        }
      }
    }
    if (a.seg_len > 0) {   // the run's end state, in units of wray for Q
      float2* st = a.segtot + (S.sbase + static_cast<long long>(ray) * S.nseg + seg) * NB;
#pragma unroll
      for (int b = 0; b < NB; ++b) st[b] = make_float2(I[b], E[b]);
    }
    if (corner >= 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if constexpr (DET)
          atomicAdd(&ctail_q[b][corner], static_cast<unsigned long long>(tail_q[b]));
        else
          atomicAdd(&ctail[b][corner], tail[b]);
      }
    }
  }
  __syncthreads();
  if (tid < NB * 8) {
    const int b = tid / 8, c = tid % 8;
    if constexpr (DET) {
      if (ctail_q[b][c] != 0ull) atomicAdd(a.corner_q + b * 8 + c, ctail_q[b][c]);
    } else {
      if (ctail[b][c] != 0.0f) unsafeAtomicAdd(a.corner + b * 8 + c, ctail[b][c]);
    }
  }
}

// Segment mode: deposit values of the runs after the first. One wave per (ray, run): the
// entry state (I0, E0) chains the earlier runs' end states, then each lane takes samples
// of the run, v_k = E0 (wray Q_k) + I0 wray P_k; samples collapsed onto a box corner go
// to the corner sums instead (the tile kernel skips them).
constexpr int kFixupThreads = 256;

template <int NB, bool DET>
__global__ void __launch_bounds__(kFixupThreads) fixup_kernel(const RecordArgs a) {
  __shared__ float ctail[NB][8];
  __shared__ unsigned long long ctail_q[NB][8];
  const int tid = static_cast<int>(threadIdx.x), lane = tid & 63;
  if (tid < NB * 8) {
    ctail[tid / 8][tid % 8] = 0.0f;
    ctail_q[tid / 8][tid % 8] = 0ull;
  }
  __syncthreads();
  const int w = static_cast<int>(blockIdx.x) * (kFixupThreads / 64) + (tid >> 6);
  if (w < a.fix_waves) {
    int lo = 0, hi = a.n_src;   // the last source whose first fix-up wave is <= w
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.src[mid].fbegin <= w) lo = mid;
      else hi = mid;
    }
    const SrcRec S = a.src[lo];
    const int local = w - S.fbegin;
    const int nrays = S.nrays;
    const int seg = 1 + local / nrays, ray = local % nrays;
    const float2* st = a.segtot + (S.sbase + static_cast<long long>(ray) * S.nseg) * NB;
    float I0[NB], E0[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      I0[b] = 0.0f;
      E0[b] = 1.0f;
    }
    for (int r = 0; r < seg; ++r) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float2 qp = st[r * NB + b];
        I0[b] = I0[b] * qp.y + E0[b] * qp.x;
        E0[b] = E0[b] * qp.y;
      }
    }
    const float wray = S.wray;
    const float4 d = S.dirs[ray];
    const float sx = S.sx, sy = S.sy, sz = S.sz;
    const int k_begin = seg * a.seg_len, k_end = min(S.nsub, k_begin + a.seg_len);
    const long long vb = S.vbase;
    double det_scale = 0.0;
    if constexpr (DET) det_scale = *a.det_scale;
    for (int k = k_begin + lane; k < k_end; k += 64) {
      const float dist = sample_distance(k, a.ds);
      const float x = sample_axis(sx, dist, d.x);
      const float y = sample_axis(sy, dist, d.y);
      const float z = sample_axis(sz, dist, d.z);
      const bool collapsed = axis_clamped(x, a.nx) && axis_clamped(y, a.ny) && axis_clamped(z, a.nz);
      const int cid = (x >= 0.0f ? 4 : 0) | (y >= 0.0f ? 2 : 0) | (z >= 0.0f ? 1 : 0);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const long long slot = row_slot(vb, nrays, ray, k) + b * a.v_bin_stride;
        float* v = a.V + slot;
        const float p = a.P[slot];
        const float val = E0[b] * *v + I0[b] * (wray * p);
        if (collapsed) {
          if constexpr (DET)
            atomicAdd(&ctail_q[b][cid], static_cast<unsigned long long>(__double2ll_rn(static_cast<double>(val) * det_scale)));
          else
            atomicAdd(&ctail[b][cid], val);
          *v = 0.0f;
        } else {
          *v = val;
        }
      }
    }
  }
  __syncthreads();
  if (tid < NB * 8) {
    const int b = tid / 8, c = tid % 8;
    if constexpr (DET) {
      if (ctail_q[b][c] != 0ull) atomicAdd(a.corner_q + b * 8 + c, ctail_q[b][c]);
    } else {
      if (ctail[b][c] != 0.0f) unsafeAtomicAdd(a.corner + b * 8 + c, ctail[b][c]);
    }
  }
}

// Interval of t with s + t n in [lo, hi), from inv = 1/n (approximate reciprocal; the
// callers' margins cover its error); empty when t0 > t1.
__device__ __forceinline__ void axis_span(float s, float n, float inv, float lo, float hi,
                                          float& t0, float& t1) {
  if (n == 0.0f) {
    const bool in = s >= lo && s < hi;
    t0 = in ? -kBig : 1.0f;
    t1 = in ? kBig : 0.0f;
  } else {
    const float ta = (lo - s) * inv, tb = (hi - s) * inv;
    t0 = fminf(ta, tb);
    t1 = fmaxf(ta, tb);
  }
}

// Narrow [t0, t1] to the t where a ray can reach [lo, hi) along one axis.
__device__ __forceinline__ void clip_axis(float s, float n, float inv, float lo, float hi,
                                          float& t0, float& t1) {
  float u0, u1;
  axis_span(s, n, inv, lo, hi, u0, u1);
  t0 = fmaxf(t0, u0);
  t1 = fminf(t1, u1);
}

// Sums reach the LDS tile one corner at a time. In the deterministic mode the tile holds
// 64-bit fixed point: each sum is scaled and rounded to an integer before the
// (order-independent) integer add.
template <typename T, typename V>
__device__ __forceinline__ T tile_value(V v, double scale) {
  if constexpr (std::is_same<T, unsigned long long>::value)
    return static_cast<unsigned long long>(__double2ll_rn(static_cast<double>(v) * scale));
  else
    return static_cast<T>(v);
}

// The LDS tile carries a one-voxel halo: padded coordinates p = l + 1 run over
// [0, kTile + 1], so both corners of every sample that touches the tile have a slot and
// a sample's eight corners sit at fixed offsets from its lower corner (immediate offsets
// of the LDS atomics; no per-corner clamping or index arithmetic). The halo is dropped at
// write-out: its voxels belong to the neighbouring tiles, which collect them from their
// own records. Rows carry one slot of padding: in units of 8 bytes, x then moves the bank
// by 6 (of 16 eight-byte bank pairs), y by 3 and z by 1, which measured faster than
// unpadded rows.
constexpr int kPadRow = kTile + 3;                 // stride of y
constexpr int kPadPlane = kPadRow * (kTile + 2);   // stride of x
constexpr int kPadVox = (kTile + 2) * kPadPlane;

__device__ __forceinline__ int pad_slot(int px, int py, int pz) { return px * kPadPlane + py * kPadRow + pz; }

// ---- output tiles ----
//
// A tile launch runs four kernels. tile_pairs_kernel<false>: per tile, the (source,
// patch) pairs that can reach it and the chunks their rays bring (a chunk is the part of
// one ray's substep range inside one aligned block of kChunk substeps).
// tile_schedule_kernel: each tile's first record (a prefix sum of the counts) and
// ceil(chunks / target) work items (at most kMaxParts; none for an empty tile without a
// box corner); item q of a tile with P items takes the q-th of P equal shares of its
// records. tile_pairs_kernel<true>: the same pass again, writing one 8-byte record per
// chunk. tile_kernel: a persistent grid whose work-groups claim items until none are
// left, so tiles next to sources, several times the mean load, are shared by several
// compute units while light tiles cost one item each. The first three depend on the
// geometry only, so a plan runs them once.

// One 16^3 output tile and the positions whose clamped stencil can reach it:
// [x0 - 1, x0 + ex) per axis, unbounded on the box faces.
struct TileGeom {
  int x0, y0, z0, ex, ey, ez;
  float Ax, Bx, Ay, By, Az, Bz;
  bool interior;           // touches no box face: the cone test applies
  float cx, cy, cz, rad;   // sphere around the tile widened by the stencil
};

__device__ __forceinline__ TileGeom tile_geom(const TileArgs& a, int t) {
  TileGeom g;
  const int tz = t % a.tiles_z, ty = (t / a.tiles_z) % a.tiles_y, tx = t / (a.tiles_z * a.tiles_y);
  g.x0 = tx * kTile;
  g.y0 = ty * kTile;
  g.z0 = tz * kTile;
  g.ex = min(kTile, a.nx - g.x0);
  g.ey = min(kTile, a.ny - g.y0);
  g.ez = min(kTile, a.nz - g.z0);
  g.Ax = g.x0 == 0 ? -kBig : static_cast<float>(g.x0 - 1);
  g.Bx = g.x0 + g.ex == a.nx ? kBig : static_cast<float>(g.x0 + g.ex);
  g.Ay = g.y0 == 0 ? -kBig : static_cast<float>(g.y0 - 1);
  g.By = g.y0 + g.ey == a.ny ? kBig : static_cast<float>(g.y0 + g.ey);
  g.Az = g.z0 == 0 ? -kBig : static_cast<float>(g.z0 - 1);
  g.Bz = g.z0 + g.ez == a.nz ? kBig : static_cast<float>(g.z0 + g.ez);
  g.interior = g.x0 > 0 && g.y0 > 0 && g.z0 > 0 && g.x0 + g.ex < a.nx && g.y0 + g.ey < a.ny &&
               g.z0 + g.ez < a.nz;
  g.cx = static_cast<float>(g.x0) - 1.0f + 0.5f * static_cast<float>(g.ex + 1);
  g.cy = static_cast<float>(g.y0) - 1.0f + 0.5f * static_cast<float>(g.ey + 1);
  g.cz = static_cast<float>(g.z0) - 1.0f + 0.5f * static_cast<float>(g.ez + 1);
  g.rad = 0.5f * sqrtf(static_cast<float>((g.ex + 1) * (g.ex + 1) + (g.ey + 1) * (g.ey + 1) +
                                          (g.ez + 1) * (g.ez + 1))) + 0.01f;
  return g;
}

// Source s of pair p: the last source whose first pair is <= p (sources without rays
// share their successor's first pair).
__device__ __forceinline__ int pair_source(const TileArgs& a, int p) {
  int lo = 0, hi = a.n_src;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.src[mid].pbegin <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The same search over the sources' first pairs staged in LDS.
__device__ __forceinline__ int pair_source(const int* first, int n_src, int p) {
  int lo = 0, hi = n_src;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= p) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Can a ray of patch `patch` of source s reach the tile? The bounding box of the patch's
// segments [0, tmax] (its direction bounds are exact), then, for interior tiles, the
// cone holding the patch's directions against the sphere around the widened tile.
__device__ __forceinline__ bool pair_reaches(const TileArgs& a, const TileGeom& g, int s, int patch) {
  const SrcRec& S = a.src[s];
  const float sx = S.sx, sy = S.sy, sz = S.sz, tmax = S.tmax, m = S.marg;
  const float* pb = S.pbounds + static_cast<long long>(patch) * kPatchRec;
  bool reach = !(sx + fmaxf(0.0f, tmax * pb[3]) + m < g.Ax || sx + fminf(0.0f, tmax * pb[0]) - m >= g.Bx ||
                 sy + fmaxf(0.0f, tmax * pb[4]) + m < g.Ay || sy + fminf(0.0f, tmax * pb[1]) - m >= g.By ||
                 sz + fmaxf(0.0f, tmax * pb[5]) + m < g.Az || sz + fminf(0.0f, tmax * pb[2]) - m >= g.Bz);
  if (reach && g.interior) {
    const float vx = g.cx - sx, vy = g.cy - sy, vz = g.cz - sz;
    const float dist = sqrtf(vx * vx + vy * vy + vz * vz);
    const float rad = g.rad + m;
    if (dist - rad > tmax + 1.0f) {
      reach = false;
    } else if (dist > rad) {
      // the sphere subtends a half-angle alpha (sin alpha = rad / dist); a direction within
      // beta of the axis can meet it only if its angle to the centre is below beta + alpha
      const float sa = fminf(1.0f, rad / dist), ca = sqrtf(fmaxf(0.0f, 1.0f - sa * sa));
      const float cb = pb[11], sb = pb[12];
      const float cos_sum = cb * ca - sb * sa, sin_sum = sb * ca + cb * sa;
      // (beta + alpha beyond ~3.1 rad: the cone covers nearly every direction, keep the pair)
      if (sin_sum >= 0.0f && cos_sum > kCosConeLimit) {
        const float c = (pb[8] * vx + pb[9] * vy + pb[10] * vz) / dist;
        reach = c >= cos_sum - 1.0e-3f;
      }
    }
  }
  return reach;
}

// Substep range [ka, kb] of one ray that can touch the tile (kb < ka: none) and its
// direction (zero for a lane past the source's last ray).
__device__ __forceinline__ void ray_range(const TileArgs& a, const TileGeom& g, int s, int ray, int& ka, int& kb,
                                          float4& d) {
  ka = 0;
  kb = -1;
  d = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const SrcRec& S = a.src[s];
  if (ray >= S.nrays) return;
  const float sx = S.sx, sy = S.sy, sz = S.sz, tmax = S.tmax, m = S.marg;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  d = S.dirs[ray];
  const float ix = __builtin_amdgcn_rcpf(d.x), iy = __builtin_amdgcn_rcpf(d.y),
              iz = __builtin_amdgcn_rcpf(d.z);
  float t0 = 0.0f, t1 = tmax;
  clip_axis(sx, d.x, ix, g.Ax - m, g.Bx + m, t0, t1);
  clip_axis(sy, d.y, iy, g.Ay - m, g.By + m, t0, t1);
  clip_axis(sz, d.z, iz, g.Az - m, g.Bz + m, t0, t1);
  // Samples collapsed onto a corner voxel (clamped along all three axes) belong to the
  // record phase. Along a straight ray each axis is unclamped on one interval of t; only
  // the hull of those intervals can hold samples for the tiles.
  float h0 = kBig, h1 = -kBig, u0, u1;
  if (nx > 1) {
    axis_span(sx, d.x, ix, -m, static_cast<float>(nx - 1) + m, u0, u1);
    if (u0 <= u1) { h0 = fminf(h0, u0); h1 = fmaxf(h1, u1); }
  }
  if (ny > 1) {
    axis_span(sy, d.y, iy, -m, static_cast<float>(ny - 1) + m, u0, u1);
    if (u0 <= u1) { h0 = fminf(h0, u0); h1 = fmaxf(h1, u1); }
  }
  if (nz > 1) {
    axis_span(sz, d.z, iz, -m, static_cast<float>(nz - 1) + m, u0, u1);
    if (u0 <= u1) { h0 = fminf(h0, u0); h1 = fmaxf(h1, u1); }
  }
  t0 = fmaxf(t0, h0);
  t1 = fminf(t1, h1);
  if (t0 <= t1) {
    // one substep of margin on each side covers the rounding of t = k ds
    ka = max(0, static_cast<int>(floorf(t0 / a.ds)) - 1);
    kb = min(S.nsub - 1, static_cast<int>(fminf(ceilf(t1 / a.ds), 1.0e8f)) + 1);
  }
}

__device__ __forceinline__ int range_chunks(int ka, int kb) {
  return kb >= ka ? kb / kChunk - ka / kChunk + 1 : 0;
}

__device__ __forceinline__ long long shfl_up_ll(long long v, int off) {
  const int lo = __shfl_up(static_cast<int>(static_cast<unsigned long long>(v) & 0xffffffffull), off, 64);
  const int hi = __shfl_up(static_cast<int>(static_cast<unsigned long long>(v) >> 32), off, 64);
  return static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                static_cast<unsigned>(lo));
}

// LDS scratch of the schedule pass.
template <int THREADS>
struct ScheduleShared {
  int w_items[THREADS / 64];
  long long w_recs[THREADS / 64];
  int carry;
  long long rec_carry;
};

// One work-group of THREADS lanes, four consecutive tiles per lane: per tile, its first
// record (prefix sums of the counts), its work items and the item -> (tile, part) map;
// also resets the fill cursors and the claim counters of the tile kernel. A tile without
// records keeps one item only if it holds a corner voxel of the box (the record phase's
// corner sums are added there).
template <int THREADS>
__device__ void schedule_tiles(const TileArgs& a, int n_tiles, ScheduleShared<THREADS>& sh) {
  constexpr int kPer = 4;
  const int tid = static_cast<int>(threadIdx.x), wave = tid >> 6, lane = tid & 63;
  if (tid == 0) {
    sh.carry = 0;
    sh.rec_carry = 0;
  }
  __syncthreads();
  for (int t0 = 0; t0 < n_tiles; t0 += THREADS * kPer) {
    int items[kPer];
    long long recs[kPer];
    int isum = 0;
    long long rsum = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = t0 + tid * kPer + q;
      items[q] = 0;
      recs[q] = 0;
      if (t < n_tiles) {
        recs[q] = static_cast<long long>(a.tile_cost[t]);
        if (recs[q] > 0) {
          const long long want = (recs[q] + a.item_chunks - 1) / a.item_chunks;
          items[q] = static_cast<int>(want > kMaxParts ? kMaxParts : want);
        } else {
          const int tz = t % a.tiles_z, ty = (t / a.tiles_z) % a.tiles_y, tx = t / (a.tiles_z * a.tiles_y);
          const bool corner = (tx == 0 || tx == a.tiles_x - 1) && (ty == 0 || ty == a.tiles_y - 1) &&
                              (tz == 0 || tz == a.tiles_z - 1);
          items[q] = corner ? 1 : 0;
        }
      }
      isum += items[q];
      rsum += recs[q];
    }
    int incl = isum;
    long long rincl = rsum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off, 64);
      const long long ro = shfl_up_ll(rincl, off);
      if (lane >= off) {
        incl += o;
        rincl += ro;
      }
    }
    if (lane == 63) {
      sh.w_items[wave] = incl;
      sh.w_recs[wave] = rincl;
    }
    __syncthreads();
    int ib = sh.carry + incl - isum;
    long long rb = sh.rec_carry + rincl - rsum;
    for (int w = 0; w < wave; ++w) {
      ib += sh.w_items[w];
      rb += sh.w_recs[w];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = t0 + tid * kPer + q;
      if (t < n_tiles) {
        a.tile_begin[t] = rb;
        a.tile_count[t] = recs[q];
        a.tile_fill[t] = rb;
      }
      for (int i = 0; i < items[q]; ++i) a.item_map[ib + i] = make_int2(t, i | (items[q] << 16));
      ib += items[q];
      rb += recs[q];
    }
    __syncthreads();
    if (tid == THREADS - 1) {
      sh.carry = ib;
      sh.rec_carry = rb;
    }
    __syncthreads();
  }
  if (tid == 0) {
    *a.item_total = sh.carry;
    *a.item_next = 0;
    *a.item_done = 0;
    *a.rec_total = sh.rec_carry;
    // records beyond the buffer are never written; the tile passes skip them, and the
    // count of such lost records is reported to the host
    if (a.dropped && sh.rec_carry > a.rec_capacity)
      atomicAdd(a.dropped, static_cast<unsigned long long>(sh.rec_carry - a.rec_capacity));
  }
}

constexpr int kScheduleThreads = 256;

// (a small work-group, so that it finds room beside a record pass running concurrently)
__global__ void __launch_bounds__(kScheduleThreads) tile_schedule_kernel(const TileArgs a, int n_tiles) {
  __shared__ ScheduleShared<kScheduleThreads> sh;
  schedule_tiles<kScheduleThreads>(a, n_tiles, sh);
}

// Per (tile, block of kPairBlock pairs): the pairs that can reach the tile, then, one
// wave per pair, the substep range of each of its rays. FILL = false: the chunks are
// summed into tile_cost[t] (zeroed beforehand), and the pairs with chunks are marked in
// pair_mask. FILL = true takes only the marked pairs (no cull, no pair without chunks). FILL = true: a wave reserves the chunks
// of the four pairs it holds with one atomic add at the tile's fill cursor and writes one
// record per chunk,
//   x = (source mod 256) << kRecRayBits | ray,
//   y = (source / 256) << kRecChunkEnd | chunk << 6 | (first substep - chunk start) << 3
//       | (last substep - chunk start),
// never past the tile's count or the record buffer. Both passes run the same code on
// the same inputs, so they agree on every count; the tile kernel also trusts only records
// below the cursor. Blocks hold a modest number of pairs because next to a source every
// pair of a block reaches the tile and each needs its rays' ranges.
constexpr int kCostThreads = 256;
constexpr int kRecRayBits = 24;    // rays per source < 2^24
constexpr int kRecChunkEnd = 27;   // chunk index < 2^21 (N_s <= 2^24); 13 bits of source above it
static_assert(kMaxSrcPerTiledLaunch <= (1 << (32 - kRecChunkEnd + 8)), "source index does not fit the records");

__device__ __forceinline__ long long shfl_ll(long long v, int src) {
  const int lo = __shfl(static_cast<int>(static_cast<unsigned long long>(v) & 0xffffffffull), src, 64);
  const int hi = __shfl(static_cast<int>(static_cast<unsigned long long>(v) >> 32), src, 64);
  return static_cast<long long>((static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) |
                                static_cast<unsigned>(lo));
}

template <bool FILL>
__global__ void __launch_bounds__(kCostThreads) tile_pairs_kernel(const TileArgs a) {
  __shared__ int list[kPairBlock];
  __shared__ int count;
  __shared__ unsigned long long total;
  constexpr int kMaskWords = kPairBlock / 32;
  __shared__ unsigned mask[kMaskWords];   // pairs of the block with chunks in the tile
  const int tid = static_cast<int>(threadIdx.x), wave = tid >> 6, lane = tid & 63;
  if (tid == 0) {
    count = 0;
    total = 0ull;
  }
  const int t = static_cast<int>(blockIdx.x);
  const TileGeom g = tile_geom(a, t);
  const int npairs = a.n_pairs;
  const int nblocks = (npairs + kPairBlock - 1) / kPairBlock;
  long long rec_end = 0;   // records of this tile end here (FILL)
  if constexpr (FILL) {
    rec_end = a.tile_begin[t] + a.tile_count[t];
    rec_end = rec_end < a.rec_capacity ? rec_end : a.rec_capacity;
  }
  unsigned long long sum = 0;
  // With few sources their first pairs sit in LDS for the searches of pair_source (its
  // chain of dependent loads measured a tenth of the count pass).
  __shared__ int first_pair[kCostThreads];
  const bool staged = a.n_src <= kCostThreads;
  if (staged && tid < a.n_src) first_pair[tid] = a.src[tid].pbegin;
  // (blocks beyond the grid's y extent, 65535, are taken in turn)
  for (int q0 = static_cast<int>(blockIdx.y); q0 < nblocks; q0 += static_cast<int>(gridDim.y)) {
    __syncthreads();
    if (tid == 0) count = 0;
    if (tid < kMaskWords) mask[tid] = 0u;
    __syncthreads();
    unsigned* const block_mask = a.pair_mask + (static_cast<long long>(t) * nblocks + q0) * kMaskWords;
    const int p = q0 * kPairBlock + tid;
    if (tid < kPairBlock && p < npairs) {
      if constexpr (FILL) {   // only the pairs the count pass found chunks for
        if ((block_mask[tid >> 5] >> (tid & 31)) & 1u) list[atomicAdd(&count, 1)] = p;
      } else {
        const int s = staged ? pair_source(first_pair, a.n_src, p) : pair_source(a, p);
        if (pair_reaches(a, g, s, p - (staged ? first_pair[s] : a.src[s].pbegin))) list[atomicAdd(&count, 1)] = p;
      }
    }
    __syncthreads();
    // A tile next to a source keeps every pair of the block: each wave then takes many
    // pairs, four at a time so that their direction loads overlap.
    constexpr int kWavesC = kCostThreads / 64, kUnroll = 4;
    for (int i0 = wave; i0 < count; i0 += kWavesC * kUnroll) {
      int ka[kUnroll], kb[kUnroll], src[kUnroll], ray[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int i = i0 + u * kWavesC;
        ka[u] = 0;
        kb[u] = -1;
        src[u] = 0;
        ray[u] = 0;
        if (i < count) {
          const int q = list[i];
          src[u] = staged ? pair_source(first_pair, a.n_src, q) : pair_source(a, q);
          ray[u] = (q - (staged ? first_pair[src[u]] : a.src[src[u]].pbegin)) * kPatch + lane;
          float4 d;
          ray_range(a, g, src[u], ray[u], ka[u], kb[u], d);
        }
      }
      if constexpr (!FILL) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          int cu = range_chunks(ka[u], kb[u]);
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) cu += __shfl_xor(cu, off, 64);
          sum += static_cast<unsigned long long>(cu);
          const int i = i0 + u * kWavesC;
          if (lane == 0 && cu > 0) {
            const int bit = list[i] - q0 * kPairBlock;
            atomicOr(&mask[bit >> 5], 1u << (bit & 31));
          }
        }
      } else {
        // offsets of each lane's chunks within the wave's kUnroll pairs, then one
        // reservation at the tile's cursor for all of them
        int incl[kUnroll], c[kUnroll];
        int run = 0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          c[u] = range_chunks(ka[u], kb[u]);
          incl[u] = c[u];
#pragma unroll
          for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl[u], off, 64);
            if (lane >= off) incl[u] += o;
          }
          incl[u] += run;
          run = __shfl(incl[u], 63, 64);
        }
        if (run == 0) continue;   // (uniform across the wave)
        long long base = 0;
        if (lane == 63)
          base = static_cast<long long>(atomicAdd(reinterpret_cast<unsigned long long*>(a.tile_fill + t),
                                                  static_cast<unsigned long long>(run)));
        base = shfl_ll(base, 63);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          long long idx = base + incl[u] - c[u];
          const unsigned rx = (static_cast<unsigned>(src[u] & 0xff) << kRecRayBits) | static_cast<unsigned>(ray[u]);
          const unsigned ry = static_cast<unsigned>(src[u] >> 8) << kRecChunkEnd;
          for (int q = 0; q < c[u] && idx < rec_end; ++q, ++idx) {
            const int cb = ka[u] / kChunk + q, kblk = cb * kChunk;
            const int ob = max(ka[u], kblk) - kblk, oe = min(kb[u], kblk + kChunk - 1) - kblk;
            a.recs[idx] = make_uint2(rx, ry | (static_cast<unsigned>(cb) << 6) | static_cast<unsigned>(ob << 3) |
                                             static_cast<unsigned>(oe));
          }
        }
      }
    }
    if constexpr (!FILL) {
      __syncthreads();
      if (tid < kMaskWords) block_mask[tid] = mask[tid];
    }
  }
  if constexpr (!FILL) {
    if (lane == 0 && sum) atomicAdd(&total, sum);
    __syncthreads();
    if (tid == 0 && total) atomicAdd(a.tile_cost + t, total);
  }
}

// Axes on which a tile touches a box face: bit 4, 2, 1 for x, y, z.
__device__ __forceinline__ int tile_faces(const TileGeom& g, int nx, int ny, int nz) {
  return (g.x0 > 0 && g.x0 + g.ex < nx ? 0 : 4) | (g.y0 > 0 && g.y0 + g.ey < ny ? 0 : 2) |
         (g.z0 > 0 && g.z0 + g.ez < nz ? 0 : 1);
}

// One axis of a sample's stencil in a tile with origin o: the lower corner's padded index
// (halo at 0), and the corners' weights. FACE: the tile touches a box face on this axis,
// so the sample may be clamped there (a collapsed axis carries its whole weight on the
// lower corner); otherwise it is not clamped if its stencil reaches the tile, and the
// index is only bounded before the conversion (the bound never passes the reach test).
template <bool FACE>
__device__ __forceinline__ int tile_axis(float x, int n, int o, float (&w)[2]) {
  if constexpr (FACE) {
    const Axis A = axis_stencil(x, n);
    w[0] = A.lo == A.hi ? 1.0f : A.w0;
    w[1] = A.lo == A.hi ? 0.0f : A.w1;
    return A.lo - o + 1;
  } else {
    const float f = floorf(x);
    w[1] = x - f;
    w[0] = 1.0f - w[1];
    return static_cast<int>(fminf(fmaxf(f, -1.0f), static_cast<float>(n))) - o + 1;
  }
}

// Every bin of a launch (claimed item by item), 512 lanes per work-group, three
// work-groups per compute unit.
// The tile is accumulated in binary64 (or 64-bit fixed point in the deterministic mode):
// a voxel next to a source collects thousands of deposits, and binary32 running sums of
// that length drift by more than the binary32 field is allowed to differ from the exact one.
// NEAREST: each sample adds its value to its nearest voxel only (the adjoint's kappa
// deposit) instead of the trilinear stencil.
template <bool DET, bool NEAREST>
__global__ void __launch_bounds__(kTileThreads) tile_kernel(const TileArgs a) {
  using T = typename std::conditional<DET, unsigned long long, double>::type;
  constexpr int kThreads = kTileThreads;
  __shared__ T acc[kPadVox];
  __shared__ int2 claimed;
  __shared__ int claimed_bin;
  const int tid = static_cast<int>(threadIdx.x);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const float ds = a.ds;
  double det_scale = 0.0;
  if constexpr (DET) det_scale = *a.det_scale;
  // claims run over (item, bin): the bins of one item are taken one after another, so
  // every bin's heavy items come first and a launch drains once, not once per bin
  const int n_bins = a.n_bins;
  const int n_claims = *a.item_total * n_bins;

  for (;;) {
    if (tid == 0) {
      const int item = atomicAdd(a.item_next, 1);
      claimed = item < n_claims ? a.item_map[item / n_bins] : make_int2(-1, 0);
      claimed_bin = item < n_claims ? item % n_bins : 0;
    }
    for (int i = tid; i < kPadVox; i += kThreads) acc[i] = T(0);
    __syncthreads();
    const int t = claimed.x;
    if (t < 0) {
      // the last work-group out rewinds the claim counter, so the same schedule serves
      // the next launch (every work-group has made its final claim by then)
      if (tid == 0 && atomicAdd(a.item_done, 1) == static_cast<int>(gridDim.x) - 1) {
        atomicExch(a.item_next, 0);
        atomicExch(a.item_done, 0);
      }
      break;
    }
    const int part = claimed.y & 0xffff, parts = claimed.y >> 16;
    const int bin = claimed_bin;
    const float* const V = a.V + bin * a.v_bin_stride;
    const TileGeom g = tile_geom(a, t);
    const int x0 = g.x0, y0 = g.y0, z0 = g.z0, ex = g.ex, ey = g.ey, ez = g.ez;
    const int faces = tile_faces(g, nx, ny, nz);

    // The item's share of the tile's chunk records; only records below the fill cursor
    // and inside the buffer were written.
    const long long rbegin = a.tile_begin[t], rcount = a.tile_count[t];
    long long rend = rbegin + rcount * (part + 1) / parts;
    rend = min(rend, min(a.tile_fill[t], a.rec_capacity));
    // Lanes take the item's records in blocks of kThreads, each wave 8 runs of 8 consecutive
    // records 64 apart (a run: one or two rays' consecutive chunks), not 64 consecutive ones:
    // neighbouring rays of a patch deposit into the same or nearby cells at the same
    // substep, and the LDS adds of one instruction then collide more often (uneven 256^3
    // tile pass 0.71 -> 0.67 ms, turbulent 128^3 0.14 -> 0.13 ms).
    const int lane_rec = (tid % 8) * (kThreads / 8) + tid / 8;
    for (long long i0 = rbegin + rcount * part / parts; i0 < rend; i0 += kThreads) {
      const long long i = i0 + lane_rec;
      if (i >= rend) continue;
      const uint2 rec = a.recs[i];
      const int s = static_cast<int>((rec.x >> kRecRayBits) | ((rec.y >> kRecChunkEnd) << 8));
      const int ray = static_cast<int>(rec.x & ((1u << kRecRayBits) - 1u));
      if (s >= a.n_src) continue;   // (not produced by the fill pass)
      const SrcRec* sr = a.src + s;
      const int nrays = sr->nrays;
      if (ray >= nrays) continue;
      const int kblk = static_cast<int>((rec.y >> 6) & ((1u << (kRecChunkEnd - 6)) - 1u)) * kChunk;
      const int kbeg = kblk + static_cast<int>((rec.y >> 3) & 7u), kend = kblk + static_cast<int>(rec.y & 7u);
      const float4 dd = sr->dirs[ray];
      const float4 src = make_float4(sr->sx, sr->sy, sr->sz, 0.0f);
      const float* vrow = V + row_slot(sr->vbase, nrays, ray, kblk);
      // the chunk's recorded values, fetched before any of them is needed
      float vv[kChunk];
#pragma unroll
      for (int q = 0; q < kChunk / 4; ++q) {
        const float4 f = reinterpret_cast<const float4*>(vrow)[q];
        vv[4 * q] = f.x;
        vv[4 * q + 1] = f.y;
        vv[4 * q + 2] = f.z;
        vv[4 * q + 3] = f.w;
      }
      // A lane sums the weighted corners of consecutive samples that share a lower corner
      // (the nearest voxel, for NEAREST) in registers: samples less than a voxel apart
      // often do. The sums reach the tile when the ray moves on to another cell and at the
      // end of the chunk, which takes a third or more of the LDS atomics away. Such a run
      // has at most kChunk terms, so it is summed in binary32 (error below kChunk units in
      // the last place of the sum of the terms' magnitudes; the terms share the sign of the
      // ray's I, which changes only where j does) and only the tile is binary64 (or fixed
      // point). The nearest-voxel deposits of the adjoint mix signs: their runs are binary64.
      // A run holds the samples of one chunk record in their order along the ray, whatever
      // the schedule, the source order or the launch split, so in the deterministic mode
      // its sum, converted to fixed point when it reaches the tile, is the same on every call.
      constexpr int kCorners = NEAREST ? 1 : 8;
      using R = typename std::conditional<NEAREST, double, float>::type;
      int cell = -1;   // padded slot of the current lower corner (nearest voxel)
      R run[kCorners];
      // SKIP_ZERO: sums that are exactly zero are not added. In a tile on a box face, a
      // sample clamped on an axis (beyond the face: four in ten samples of a march whose
      // rays run out of the box) carries no weight on its upper corners along that axis,
      // and the adds left out make the instruction cheaper (an LDS atomic costs about one
      // pass per lane that shares a bank with another active lane).
      auto flush = [&](auto skip_tag) {
        constexpr bool SKIP_ZERO = decltype(skip_tag)::value;
        if (cell < 0) return;
#pragma unroll
        for (int c = 0; c < kCorners; ++c)
          if (!SKIP_ZERO || run[c] != R(0))
            atomicAdd(&acc[cell + (c >> 2) * kPadPlane + ((c >> 1) & 1) * kPadRow + (c & 1)],
                      tile_value<T>(run[c], det_scale));
      };
      auto move_to = [&](int slot, auto skip_tag) {
        if (slot == cell) return;
        flush(skip_tag);
        cell = slot;
#pragma unroll
        for (int c = 0; c < kCorners; ++c) run[c] = R(0);
      };
      // FACES (uniform over the item): bit 4, 2, 1 set for the axes x, y, z on which the
      // tile touches a box face. On the other axes a sample whose stencil reaches the tile
      // is never clamped (a clamped lower corner is 0 or n - 1, outside the tile's reach
      // there), so their clamps and collapsed-axis weights drop out of the sample loop, and
      // unless the tile touches faces on all three axes so does the box-corner test.
      auto samples = [&](auto faces_tag) {
        constexpr int FACES = decltype(faces_tag)::value;
        constexpr bool INNER = FACES == 0;
        constexpr std::integral_constant<bool, !INNER> skip_zero{};
#pragma unroll
        for (int u = 0; u < kChunk; ++u) {
          const int k = kblk + u;
          const float dist = sample_distance(k, ds);
          const float x = sample_axis(src.x, dist, dd.x);
          const float y = sample_axis(src.y, dist, dd.y);
          const float z = sample_axis(src.z, dist, dd.z);
          if constexpr (FACES != 7) {
            if ((k < kbeg) | (k > kend)) continue;
          } else {
            // outside this ray's range for the tile, or collapsed onto one corner voxel of
            // the box (summed by the record phase)
            // (bitwise tests: one branch per sample, not a chain of short-circuit branches)
            const int clamped = static_cast<int>(axis_clamped(x, nx)) + static_cast<int>(axis_clamped(y, ny)) +
                                static_cast<int>(axis_clamped(z, nz));
            if ((k < kbeg) | (k > kend) | (clamped == 3)) continue;
          }
          if constexpr (NEAREST) {
            int lx, ly, lz;
            if constexpr (INNER) {   // (bounded before the conversion; the bound never passes the test)
              lx = static_cast<int>(fminf(fmaxf(rintf(x), -1.0f), static_cast<float>(nx))) - x0;
              ly = static_cast<int>(fminf(fmaxf(rintf(y), -1.0f), static_cast<float>(ny))) - y0;
              lz = static_cast<int>(fminf(fmaxf(rintf(z), -1.0f), static_cast<float>(nz))) - z0;
            } else {
              lx = axis_stencil(x, nx).nearest - x0;
              ly = axis_stencil(y, ny).nearest - y0;
              lz = axis_stencil(z, nz).nearest - z0;
            }
            if ((static_cast<unsigned>(lx) >= static_cast<unsigned>(ex)) |
                (static_cast<unsigned>(ly) >= static_cast<unsigned>(ey)) |
                (static_cast<unsigned>(lz) >= static_cast<unsigned>(ez)))
              continue;
            move_to(pad_slot(lx + 1, ly + 1, lz + 1), skip_zero);
            run[0] += static_cast<R>(vv[u]);
          } else {
            // some corner lies in the tile iff the lower corner is in [origin - 1, origin +
            // extent - 1] on every axis (a collapsed axis, lower = upper corner, only occurs
            // on the box faces, where the lower corner is never origin - 1)
            float wx[2], wy[2], wz[2];
            const int px = tile_axis<(FACES & 4) != 0>(x, nx, x0, wx);
            const int py = tile_axis<(FACES & 2) != 0>(y, ny, y0, wy);
            const int pz = tile_axis<(FACES & 1) != 0>(z, nz, z0, wz);
            if ((static_cast<unsigned>(px) > static_cast<unsigned>(ex)) |
                (static_cast<unsigned>(py) > static_cast<unsigned>(ey)) |
                (static_cast<unsigned>(pz) > static_cast<unsigned>(ez)))
              continue;
            move_to(pad_slot(px, py, pz), skip_zero);
            // v (wx wy) wz as (wx wy)(v wz): 14 products instead of 20
            const float vz[2] = {vv[u] * wz[0], vv[u] * wz[1]};
#pragma unroll
            for (int c = 0; c < 8; ++c) run[c] += (wx[c >> 2] * wy[(c >> 1) & 1]) * vz[c & 1];
          }
        }
        flush(skip_zero);
      };
      switch (faces) {
        case 0: samples(std::integral_constant<int, 0>{}); break;
        case 4: samples(std::integral_constant<int, 4>{}); break;
        case 2: samples(std::integral_constant<int, 2>{}); break;
        case 1: samples(std::integral_constant<int, 1>{}); break;
        default: samples(std::integral_constant<int, 7>{}); break;   // (edges and corners of the box)
      }
    }
    __syncthreads();

    // the corner voxels of the box also receive the record phase's per-corner sums
    for (int i = tid; i < kTileVox; i += kThreads) {
      const int lx = i / (kTile * kTile), ly = (i / kTile) % kTile, lz = i % kTile;
      if (lx >= ex || ly >= ey || lz >= ez) continue;
      const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
      const long long voxel = (static_cast<long long>(gx) * ny + gy) * nz + gz;
      const bool cx_any = (gx == 0 || gx == nx - 1), cy_any = (gy == 0 || gy == ny - 1),
                 cz_any = (gz == 0 || gz == nz - 1);
      T val = acc[pad_slot(lx + 1, ly + 1, lz + 1)];
      if (cx_any && cy_any && cz_any && part == 0) {
        for (int c = 0; c < 8; ++c) {
          const int vx = (c & 4) ? nx - 1 : 0, vy = (c & 2) ? ny - 1 : 0, vz = (c & 1) ? nz - 1 : 0;
          if (vx == gx && vy == gy && vz == gz) {
            if constexpr (DET) val += a.corner_q[bin * 8 + c];
            else val += a.corner[bin * 8 + c];
          }
        }
      }
      // The field was zeroed before the launch. A tile served by one item adds its sum
      // with a plain read-modify-write; items sharing a tile add atomically (consecutive
      // lanes hold consecutive z, so the adds of a wave coalesce).
      if constexpr (DET) {
        unsigned long long* o = a.out_q + bin * a.out_stride + voxel;
        if (val != 0ull) {
          if (parts > 1) atomicAdd(o, val);
          else *o += val;
        }
      } else {
        float* o = a.out + bin * a.out_stride + voxel;
        if (val != 0.0) {
          if (parts > 1) unsafeAtomicAdd(o, static_cast<float>(val));
          else *o = static_cast<float>(static_cast<double>(*o) + val);
        }
      }
    }
    __syncthreads();   // the tile is cleared for the next item
  }
}

// Gather pass: the samples of a launch gathered tile by tile instead of ray by ray. A work
// item stages its tile's j and kappa with a one-voxel upper halo (17^3 voxels, indices
// clamped to the box as the corners of the 64-byte gather table are) in LDS, then takes
// its share of the tile's chunk records: every sample whose lower stencil corner lies in
// the tile gets j (trilinear, as three rounds of linear interpolation; a collapsed axis
// weighs its lower corner 1 and its upper corner 0, as the gather table does) and kappa at
// its nearest voxel (always one of the staged corners), written to the sample's slot of
// rows shaped like bin 0's deposit
// rows. A sample's lower corner lies in one tile, whose records list it (they list every
// sample that can reach the tile), so each slot is written once; samples collapsed onto a
// box-corner voxel are left to the record pass. The record pass then reads one 64-byte
// piece per ray and 8 substeps instead of one random 64-byte table line per sample.
constexpr int kGEdge = kTile + 1;

// One axis of a sample in the gather pass's tile with origin o: the lower corner's index in
// the tile, the upper corner's weight and the nearest voxel's index. FACE as in tile_axis;
// otherwise the nearest voxel is the lower corner, or the upper one past the midpoint
// (rint's halfway cases round to even; no clamp reaches a sample that the tile owns).
template <bool FACE>
__device__ __forceinline__ int gather_axis(float x, int n, int o, float& w1, int& nearest) {
  if constexpr (FACE) {
    const Axis A = axis_stencil(x, n);
    w1 = A.lo == A.hi ? 0.0f : A.w1;
    nearest = A.nearest - o;
    return A.lo - o;
  } else {
    const float f = floorf(x);
    const int l = static_cast<int>(fminf(fmaxf(f, -1.0f), static_cast<float>(n))) - o;
    w1 = x - f;
    nearest = l + static_cast<int>(rintf(x) - f);
    return l;
  }
}
constexpr int kGatherMerge = 4;   // work items of one tile per staging
constexpr int kGPlane = kGEdge * kGEdge;
constexpr int kGVox = kGEdge * kGPlane;

__global__ void __launch_bounds__(kTileThreads) gather_pass_kernel(const TileArgs a) {
  constexpr int kThreads = kTileThreads;
  __shared__ float sj[kGVox], sk[kGVox];
  __shared__ int2 claimed;
  const int tid = static_cast<int>(threadIdx.x);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const float ds = a.ds;
  const int n_items = *a.item_total;
  const int merge = max(1, min(kGatherMerge, n_items / (4 * static_cast<int>(gridDim.x))));
  // The rows are written through a buffer resource: its stores take a 32-bit byte offset
  // (the launch's rows stay below 4 GiB), and whole 16-byte pairs go out as one store
  // (the compiler would otherwise split a pair into the two 8-byte stores of the partial
  // case). Stores past the rows' end would be dropped by the hardware.
  const __amdgpu_buffer_rsrc_t jk_rsrc =
      __builtin_amdgcn_make_buffer_rsrc(a.jk, 0, static_cast<int>(a.jk_bytes), 0x00020000);
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

  for (;;) {
    if (tid == 0) {
      const int item = atomicAdd(a.item_next, 1);
      claimed = item < n_items ? a.item_map[item] : make_int2(-1, 0);
    }
    __syncthreads();
    const int2 c = claimed;
    __syncthreads();   // (read by every lane before lane 0 claims again)
    const int t = c.x;
    if (t < 0) {
      // the last work-group out rewinds the claim counters for the tile passes
      if (tid == 0 && atomicAdd(a.item_done, 1) == static_cast<int>(gridDim.x) - 1) {
        atomicExch(a.item_next, 0);
        atomicExch(a.item_done, 0);
      }
      break;
    }
    // A tile's items are consecutive in the item map; with several items per work-group
    // this pass takes them `merge` at a time (one staging of the tile per `merge` shares of
    // its records) and lets the claims of the other parts go by.
    const int part = c.y & 0xffff, parts = c.y >> 16;
    if (part % merge != 0) continue;
    const int part_end = min(part + merge, parts);
    const TileGeom g = tile_geom(a, t);
    const int x0 = g.x0, y0 = g.y0, z0 = g.z0, ex = g.ex, ey = g.ey, ez = g.ez;
    const int faces = tile_faces(g, nx, ny, nz);
    {   // (each lane keeps one z of rows kRowsPerPass apart)
      constexpr int kRowsPerPass = kThreads / kGEdge;
      const int lz = tid % kGEdge;
      const int gz = min(z0 + lz, nz - 1);
      for (int r = tid / kGEdge; r < kGPlane && tid < kRowsPerPass * kGEdge; r += kRowsPerPass) {
        const int lx = r / kGEdge, ly = r - lx * kGEdge;
        const long long v = (static_cast<long long>(min(x0 + lx, nx - 1)) * ny + min(y0 + ly, ny - 1)) * nz + gz;
        sj[r * kGEdge + lz] = a.gj[v];
        sk[r * kGEdge + lz] = a.gk[v];
      }
    }
    __syncthreads();

    const long long rbegin = a.tile_begin[t], rcount = a.tile_count[t];
    long long rend = rbegin + rcount * part_end / parts;
    rend = min(rend, min(a.tile_fill[t], a.rec_capacity));
    // (the lane's next record is fetched while this one is processed: the pass waits on
    // the chain record -> source -> direction more than on anything else)
    const long long rfirst = rbegin + rcount * part / parts + tid;
    uint2 rec_next = rfirst < rend ? a.recs[rfirst] : make_uint2(0u, 0u);
    for (long long i = rfirst; i < rend; i += kThreads) {
      const uint2 rec = rec_next;
      if (i + kThreads < rend) rec_next = a.recs[i + kThreads];
      const int s = static_cast<int>((rec.x >> kRecRayBits) | ((rec.y >> kRecChunkEnd) << 8));
      const int ray = static_cast<int>(rec.x & ((1u << kRecRayBits) - 1u));
      if (s >= a.n_src) continue;   // (not produced by the fill pass)
      const SrcRec* sr = a.src + s;
      const int nrays = sr->nrays;
      if (ray >= nrays) continue;
      const int kblk = static_cast<int>((rec.y >> 6) & ((1u << (kRecChunkEnd - 6)) - 1u)) * kChunk;
      const int kbeg = kblk + static_cast<int>((rec.y >> 3) & 7u), kend = kblk + static_cast<int>(rec.y & 7u);
      const float4 dd = sr->dirs[ray];
      const float sx = sr->sx, sy = sr->sy, sz = sr->sz;
      // (byte offset below 4 GiB, carried as the 32-bit pattern the store takes)
      const unsigned row = static_cast<unsigned>(row_slot(sr->vbase, nrays, ray, kblk) * static_cast<long long>(sizeof(float2)));
      // (FACES: the axes on which the tile touches a box face, as in the tile kernel; a
      // sample this tile owns is clamped on no other axis)
      auto samples = [&](auto faces_tag) {
        constexpr int FACES = decltype(faces_tag)::value;
        // sample u of the chunk: false if this tile does not own it, else its (j, kappa)
        auto one = [&](int u, float2& res) -> bool {
          const int k = kblk + u;
          if (FACES != 7 && ((k < kbeg) | (k > kend))) return false;
          const float dist = sample_distance(k, ds);
          const float x = sample_axis(sx, dist, dd.x);
          const float y = sample_axis(sy, dist, dd.y);
          const float z = sample_axis(sz, dist, dd.z);
          if constexpr (FACES == 7) {
            const int clamped = static_cast<int>(axis_clamped(x, nx)) + static_cast<int>(axis_clamped(y, ny)) +
                                static_cast<int>(axis_clamped(z, nz));
            if ((k < kbeg) | (k > kend) | (clamped == 3)) return false;
          }
          float wx[2], wy[2], wz[2];   // (only the upper weights are used)
          int nxl, nyl, nzl;
          const int lx = gather_axis<(FACES & 4) != 0>(x, nx, x0, wx[1], nxl);
          const int ly = gather_axis<(FACES & 2) != 0>(y, ny, y0, wy[1], nyl);
          const int lz = gather_axis<(FACES & 1) != 0>(z, nz, z0, wz[1], nzl);
          if ((static_cast<unsigned>(lx) >= static_cast<unsigned>(ex)) |
              (static_cast<unsigned>(ly) >= static_cast<unsigned>(ey)) |
              (static_cast<unsigned>(lz) >= static_cast<unsigned>(ez)))
            return false;
          // trilinear j as three rounds of linear interpolation, z then y then x (a + w (b - a);
          // a collapsed axis has w = 0 and takes its lower corner)
          const int base = lx * kGPlane + ly * kGEdge + lz;
          float e[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int o = base + (q >> 1) * kGPlane + (q & 1) * kGEdge;
            const float a0 = sj[o], a1 = sj[o + 1];
            e[q] = a0 + wz[1] * (a1 - a0);
          }
          const float f0 = e[0] + wy[1] * (e[1] - e[0]), f1 = e[2] + wy[1] * (e[3] - e[2]);
          res = make_float2(f0 + wx[1] * (f1 - f0), sk[nxl * kGPlane + nyl * kGEdge + nzl]);
          return true;
        };
        // two samples per 16-byte store where this tile owns both (a whole chunk: four
        // stores filling its 64 bytes), else one 8-byte store per owned sample
#pragma unroll
        for (int h = 0; h < kChunk / 2; ++h) {
          float2 r0, r1;
          const bool m0 = one(2 * h, r0), m1 = one(2 * h + 1, r1);
          if (m0 & m1) {
            const u32x4 q = {__float_as_uint(r0.x), __float_as_uint(r0.y), __float_as_uint(r1.x), __float_as_uint(r1.y)};
            __builtin_amdgcn_raw_buffer_store_b128(q, jk_rsrc, static_cast<int>(row + 16u * h), 0, 0);
          } else {
            if (m0) __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(r0.x), __float_as_uint(r0.y)}, jk_rsrc,
                                                          static_cast<int>(row + 16u * h), 0, 0);
            if (m1) __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(r1.x), __float_as_uint(r1.y)}, jk_rsrc,
                                                          static_cast<int>(row + 16u * h + 8u), 0, 0);
          }
        }
      };
      switch (faces) {
        case 0: samples(std::integral_constant<int, 0>{}); break;
        case 4: samples(std::integral_constant<int, 4>{}); break;
        case 2: samples(std::integral_constant<int, 2>{}); break;
        case 1: samples(std::integral_constant<int, 1>{}); break;
        default: samples(std::integral_constant<int, 7>{}); break;
      }
    }
    __syncthreads();   // the staged tile is replaced by the next item's
  }
}

template <int NB>
hipError_t launch_record_nb(const RecordArgs& a, bool shared_j, bool det, int, hipStream_t s) {
  // kXcds work-groups per round, one per XCD group, as many rounds as the largest group has blocks
  int rounds = 0;
  for (int x = 0; x < kXcds; ++x) rounds = max(rounds, a.xcd_blocks[x]);
  if (rounds == 0) return hipSuccess;
  const dim3 grid(rounds * kXcds), block(kBlock);
  if (a.jk) {
    if (det) hipLaunchKernelGGL((record_kernel<NB, true, true, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((record_kernel<NB, true, false, 2>), grid, block, 0, s, a);
  } else if (a.med) {
    if (det) hipLaunchKernelGGL((record_kernel<NB, true, true, 1>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((record_kernel<NB, true, false, 1>), grid, block, 0, s, a);
  } else if (shared_j) {
    if (det) hipLaunchKernelGGL((record_kernel<NB, true, true, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((record_kernel<NB, true, false, 0>), grid, block, 0, s, a);
  } else {
    if (det) hipLaunchKernelGGL((record_kernel<NB, false, true, 0>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((record_kernel<NB, false, false, 0>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

// Work-groups of a persistent grid: as many as fit on the device at once (any surplus
// simply starts later and finds no work left).
template <typename K>
int resident_groups(K kernel, int threads, int* cache) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kCacheDevices) dev = 0;
  if (cache[dev] == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 1;
    cache[dev] = per_cu * cus;
  }
  return cache[dev];
}

template <bool DET, bool NEAREST>
hipError_t launch_tile_variant(const TileArgs& a, hipStream_t s) {
  static int cache[kCacheDevices] = {0};   // one per kernel variant and device
  static int cus[kCacheDevices] = {0};
  const auto kernel = tile_kernel<DET, NEAREST>;
  int groups = resident_groups(kernel, kTileThreads, cache);
  if (a.groups_per_cu > 0) {   // fewer resident work-groups than fit (a tuning knob)
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kCacheDevices) dev = 0;
    if (cus[dev] == 0 && (hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                          cus[dev] < 1))
      cus[dev] = 1;
    groups = min(groups, a.groups_per_cu * cus[dev]);
  }
  hipLaunchKernelGGL(kernel, dim3(groups), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tile_one_bin(const TileArgs& a, bool det, bool nearest, hipStream_t s) {
  if (nearest) return det ? launch_tile_variant<true, true>(a, s) : launch_tile_variant<false, true>(a, s);
  return det ? launch_tile_variant<true, false>(a, s) : launch_tile_variant<false, false>(a, s);
}

// One lane per source: copy the record, completing the distance of its last substep and
// the position margin of the tile geometry (binary32, as the kernels that read them).
__global__ void __launch_bounds__(64) write_sources_kernel(const SrcWrite w) {
  const int i = static_cast<int>(threadIdx.x);
  if (i >= w.count) return;
  SrcRec r = w.rec[i];
  r.tmax = sample_distance(r.nsub - 1, w.ds);
  r.marg = 5.0e-7f * (fmaxf(fabsf(r.sx), fmaxf(fabsf(r.sy), fabsf(r.sz))) + r.tmax + 2.0f) + 1.0e-6f;
  w.table[w.first + i] = r;
}

dim3 pairs_grid(const TileArgs& a, int tiles) {
  const int nblocks = (a.n_pairs + kPairBlock - 1) / kPairBlock;
  return dim3(tiles, nblocks < 65535 ? nblocks : 65535);
}

}  // namespace

template <int NB>
void launch_fixup_nb(const RecordArgs& a, bool det, dim3 grid, hipStream_t s) {
  if (det) hipLaunchKernelGGL((fixup_kernel<NB, true>), grid, dim3(kFixupThreads), 0, s, a);
  else hipLaunchKernelGGL((fixup_kernel<NB, false>), grid, dim3(kFixupThreads), 0, s, a);
}

hipError_t launch_fixup(const RecordArgs& a, int n_bins, bool det, int waves, hipStream_t s) {
  const dim3 grid((waves + kFixupThreads / 64 - 1) / (kFixupThreads / 64));
  switch (n_bins) {
    case 1: launch_fixup_nb<1>(a, det, grid, s); break;
    case 2: launch_fixup_nb<2>(a, det, grid, s); break;
    case 3: launch_fixup_nb<3>(a, det, grid, s); break;
    case 4: launch_fixup_nb<4>(a, det, grid, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_record(const RecordArgs& a, int n_bins, bool shared_j, bool det, int blocks,
                         hipStream_t s) {
  switch (n_bins) {
    case 1: return launch_record_nb<1>(a, shared_j, det, blocks, s);
    case 2: return launch_record_nb<2>(a, shared_j, det, blocks, s);
    case 3: return launch_record_nb<3>(a, shared_j, det, blocks, s);
    case 4: return launch_record_nb<4>(a, shared_j, det, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_write_sources(const SrcWrite& w, hipStream_t s) {
  if (w.count < 1 || w.count > kSrcPerWrite) return hipErrorInvalidValue;
  hipLaunchKernelGGL(write_sources_kernel, dim3(1), dim3(64), 0, s, w);
  return hipGetLastError();
}

hipError_t launch_cell_table(const float* j, const float* kap, float4* table, int nx, int ny, int nz,
                             hipStream_t s) {
  const long long cells = static_cast<long long>(nx) * ny * nz;
  long long blocks = (4 * cells + kBlock * 4 - 1) / (kBlock * 4);
  blocks = blocks < 1 ? 1 : (blocks > 16384 ? 16384 : blocks);
  hipLaunchKernelGGL(cell_table_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, j, kap, table,
                     nx, ny, nz);
  return hipGetLastError();
}

hipError_t launch_gather_pass(const TileArgs& a, hipStream_t s) {
  static int cache[kCacheDevices] = {0};
  const int groups = resident_groups(gather_pass_kernel, kTileThreads, cache);
  hipLaunchKernelGGL(gather_pass_kernel, dim3(groups), dim3(kTileThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tile_schedule(const TileArgs& a, int tiles, hipStream_t s) {
  hipError_t e = launch_fill_zero_u64(a.tile_cost, tiles, s);
  if (e != hipSuccess) return e;
  if (a.n_pairs > 0)   // (without rays every tile keeps a zero count)
    hipLaunchKernelGGL(tile_pairs_kernel<false>, pairs_grid(a, tiles), dim3(kCostThreads), 0, s, a);
  hipLaunchKernelGGL(tile_schedule_kernel, dim3(1), dim3(kScheduleThreads), 0, s, a, tiles);
  return hipGetLastError();
}

hipError_t launch_tile_fill(const TileArgs& a, int tiles, hipStream_t s) {
  if (a.n_pairs > 0 && a.rec_capacity > 0)
    hipLaunchKernelGGL(tile_pairs_kernel<true>, pairs_grid(a, tiles), dim3(kCostThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tile_bin(const TileArgs& a, int bin, bool det, bool nearest, hipStream_t s) {
  // One pass per bin over the same schedule (each pass leaves it rewound for the next).
  // A one-bin LDS tile with its halo (49 KB) lets three work-groups share a compute unit;
  // tiles of several bins would hold one, and measured slower than repeating the geometry.
  if (bin < 0 || bin >= kMaxBinsPerLaunch) return hipErrorInvalidValue;
  TileArgs b = a;
  b.V = a.V + bin * a.v_bin_stride;
  if (a.out) b.out = a.out + bin * a.out_stride;
  if (a.out_q) b.out_q = a.out_q + bin * a.out_stride;
  b.corner = a.corner + bin * 8;
  b.corner_q = a.corner_q + bin * 8;
  b.n_bins = 1;
  return launch_tile_one_bin(b, det, nearest, s);
}

hipError_t launch_tile_bins(const TileArgs& a, int n_bins, bool det, bool nearest, hipStream_t s) {
  if (n_bins < 1 || n_bins > kMaxBinsPerLaunch) return hipErrorInvalidValue;
  TileArgs b = a;
  b.n_bins = n_bins;
  return launch_tile_one_bin(b, det, nearest, s);
}

hipError_t launch_tile_run(const TileArgs& a, int n_bins, bool det, bool nearest, hipStream_t s) {
  if (n_bins < 1 || n_bins > kMaxBinsPerLaunch) return hipErrorInvalidValue;
  for (int b0 = 0; b0 < n_bins; ++b0) {
    const hipError_t e = launch_tile_bin(a, b0, det, nearest, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rtmi
