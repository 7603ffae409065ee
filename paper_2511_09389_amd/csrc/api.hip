// Host layer of librtmi: argument validation, substep count, direction tables, launches.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/rtmi.h"
#include "common.h"

namespace {

using rtmi::kBlock;
using rtmi::kMaxBinsPerLaunch;
using rtmi::kMaxSrcPerLaunch;

constexpr int64_t kMaxCount = int64_t(1) << 24;  // num_rays and N_s limit (k is exact in binary32)
constexpr double kFourPi = 4.0 * 3.14159265358979323846;

thread_local std::string g_error;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int32_t hip_fail(hipError_t e, const char* what) {
  return fail(RTMI_ERR_HIP, "%s failed: %s", what, hipGetErrorString(e));
}

// N_s = ceil(c dt / ds) in binary64 on the binary32 arguments, then min(cap) if cap > 0.
int64_t substeps(float ds, float c, float dt, int32_t cap) {
  const double q = (static_cast<double>(c) * static_cast<double>(dt)) / static_cast<double>(ds);
  double n = std::ceil(q);
  if (cap > 0 && n > static_cast<double>(cap)) n = static_cast<double>(cap);
  if (n > static_cast<double>(kMaxCount)) return -1;
  return static_cast<int64_t>(n);
}

int32_t check_scalars(float ds, float c, float dt) {
  if (!std::isfinite(ds) || !std::isfinite(c) || !std::isfinite(dt))
    return fail(RTMI_ERR_NONFINITE, "step_size, radiation_velocity and time_step must be finite");
  if (!(ds > 0.0f)) return fail(RTMI_ERR_INVALID_ARG, "step_size must be > 0 (got %g)", ds);
  if (c < 0.0f) return fail(RTMI_ERR_INVALID_ARG, "radiation_velocity must be >= 0 (got %g)", c);
  if (dt < 0.0f) return fail(RTMI_ERR_INVALID_ARG, "time_step must be >= 0 (got %g)", dt);
  return RTMI_OK;
}

int32_t check_shape(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1)
    return fail(RTMI_ERR_SHAPE, "grid dimensions must be >= 1 (got %d x %d x %d)", nx, ny, nz);
  const int64_t cells = int64_t(nx) * ny * nz;
  if (cells >= (int64_t(1) << 31))
    return fail(RTMI_ERR_SHAPE, "nx*ny*nz = %lld must be < 2^31", static_cast<long long>(cells));
  return RTMI_OK;
}

// The golden-angle lattice in binary64, rounded to binary32. Row i = lattice point i.
void fibonacci_host(int32_t n, std::vector<float>& xyz) {
  xyz.resize(static_cast<size_t>(n) * 3);
  const double g = (3.0 - std::sqrt(5.0)) / 2.0;
  const double two_pi = 2.0 * 3.14159265358979323846;
  for (int32_t i = 0; i < n; ++i) {
    const double z = 1.0 - (2.0 * i + 1.0) / n;
    const double r = std::sqrt(std::fmax(0.0, 1.0 - z * z));
    const double ig = i * g;
    const double phi = two_pi * (ig - std::floor(ig));
    xyz[3 * size_t(i) + 0] = static_cast<float>(r * std::cos(phi));
    xyz[3 * size_t(i) + 1] = static_cast<float>(r * std::sin(phi));
    xyz[3 * size_t(i) + 2] = static_cast<float>(z);
  }
}

// Device table: float4 (x, y, z, bits of the lattice index) per lane.
std::vector<float4> lane_table(const std::vector<float>& xyz) {
  const size_t n = xyz.size() / 3;
  std::vector<float4> t(n);
  for (size_t i = 0; i < n; ++i) {
    int32_t idx = static_cast<int32_t>(i);
    float w;
    std::memcpy(&w, &idx, sizeof w);
    t[i] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], w);
  }
  return t;
}

std::mutex g_mu;
std::map<std::pair<int, int32_t>, float4*> g_dirs;  // (device, N) -> table, kept for the process

int32_t current_device(int* dev) {
  const hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return RTMI_OK;
}

int32_t get_dirs(int32_t n, hipStream_t stream, const float4** out) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_dirs.find({dev, n});
  if (it != g_dirs.end()) {
    *out = it->second;
    return RTMI_OK;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (stream != nullptr && hipStreamIsCapturing(stream, &cap) == hipSuccess &&
      cap != hipStreamCaptureStatusNone)
    return fail(RTMI_ERR_UNSUPPORTED,
                "direction table for %d rays not prepared; call rtmi_prepare before capture", n);
  std::vector<float> xyz;
  fibonacci_host(n, xyz);
  const std::vector<float4> t = lane_table(xyz);
  float4* d = nullptr;
  hipError_t e = hipMalloc(&d, t.size() * sizeof(float4));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(direction table)");
  e = hipMemcpy(d, t.data(), t.size() * sizeof(float4), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy(direction table)");
  }
  g_dirs[{dev, n}] = d;
  *out = d;
  return RTMI_OK;
}

// ---- measurement hooks: event pairs around march launches ----
std::mutex g_tmu;
bool g_timing = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_pending;  // recorded, not yet read
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_free;

hipError_t timed_launch_begin(hipStream_t s, std::pair<hipEvent_t, hipEvent_t>* ev, bool* on) {
  std::lock_guard<std::mutex> lock(g_tmu);
  *on = g_timing;
  if (!g_timing) return hipSuccess;
  if (g_free.empty()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    g_free.push_back({a, b});
  }
  *ev = g_free.back();
  g_free.pop_back();
  return hipEventRecord(ev->first, s);
}

hipError_t timed_launch_end(hipStream_t s, const std::pair<hipEvent_t, hipEvent_t>& ev, bool on) {
  if (!on) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_tmu);
  const hipError_t e = hipEventRecord(ev.second, s);
  g_pending.push_back(ev);
  return e;
}

struct Problem {
  const float* j;
  int64_t j_stride;
  const float* kap;
  int64_t k_stride;
  const float* kscale;  // host, n_bins, or null
  int32_t n_bins;
  int32_t nx, ny, nz;
  int32_t n_src;
  const float* src;       // host [n_src][3]
  const int32_t* nrays;   // host [n_src]
  const int32_t* caps;    // host [n_src] or null
  float ds, c, dt;
  float* out;
  const rtmi_options* opts;
  hipStream_t stream;
};

int32_t run(const Problem& p) {
  // ---- validation: nothing is enqueued before all of it passes ----
  if (!p.j || !p.kap || !p.out || !p.src || !p.nrays)
    return fail(RTMI_ERR_INVALID_ARG, "null map, field, source_pos or num_rays pointer");
  if (int32_t st = check_shape(p.nx, p.ny, p.nz)) return st;
  if (int32_t st = check_scalars(p.ds, p.c, p.dt)) return st;
  if (p.n_src < 1) return fail(RTMI_ERR_INVALID_ARG, "n_src must be >= 1 (got %d)", p.n_src);
  if (p.n_bins < 1) return fail(RTMI_ERR_INVALID_ARG, "n_bins must be >= 1 (got %d)", p.n_bins);
  if (p.j_stride < 0 || p.k_stride < 0)
    return fail(RTMI_ERR_INVALID_ARG, "bin strides must be >= 0");
  const int64_t cells = int64_t(p.nx) * p.ny * p.nz;
  if (p.n_bins > 1 && ((p.j_stride != 0 && p.j_stride < cells) || (p.k_stride != 0 && p.k_stride < cells)))
    return fail(RTMI_ERR_INVALID_ARG, "a non-zero bin stride must be >= nx*ny*nz");
  if (p.kscale)
    for (int32_t b = 0; b < p.n_bins; ++b)
      if (!std::isfinite(p.kscale[b])) return fail(RTMI_ERR_NONFINITE, "kappa_scale[%d] is not finite", b);
  const bool det = p.opts && p.opts->accum_mode == RTMI_ACCUM_DETERMINISTIC;
  if (p.opts && p.opts->accum_mode != RTMI_ACCUM_ATOMIC && !det)
    return fail(RTMI_ERR_INVALID_ARG, "unknown accum_mode %d", p.opts->accum_mode);
  const bool explicit_dirs = p.opts && p.opts->directions;
  std::vector<int32_t> nsub(p.n_src);
  double bound_per_unit_j = 0.0;  // worst-case |J| per voxel per unit max|j| (deterministic mode)
  for (int32_t s = 0; s < p.n_src; ++s) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p.src[3 * s + a])) return fail(RTMI_ERR_NONFINITE, "source_pos[%d] is not finite", s);
    if (p.nrays[s] < 1 || p.nrays[s] > kMaxCount)
      return fail(p.nrays[s] < 1 ? RTMI_ERR_INVALID_ARG : RTMI_ERR_RANGE,
                  "num_rays[%d] = %d must be in [1, 2^24]", s, p.nrays[s]);
    if (explicit_dirs && p.nrays[s] != p.nrays[0])
      return fail(RTMI_ERR_INVALID_ARG, "explicit directions need one num_rays for all sources");
    const int64_t n = substeps(p.ds, p.c, p.dt, p.caps ? p.caps[s] : 0);
    if (n < 0) return fail(RTMI_ERR_RANGE, "N_s = ceil(c dt / ds) exceeds 2^24");
    nsub[s] = static_cast<int32_t>(n);
    // I <= N_s ds max|j| (exp factors <= 1 for kappa >= 0); each ray deposits at most
    // N_s times into one voxel with weight <= 1, times 4 pi / N_Omega, summed over N_Omega rays.
    bound_per_unit_j += kFourPi * double(n) * double(n) * double(p.ds);
  }
  if (explicit_dirs && p.opts->ray_weight > 0.0f && !std::isfinite(p.opts->ray_weight))
    return fail(RTMI_ERR_NONFINITE, "ray_weight is not finite");

  // ---- directions ----
  std::vector<const float4*> dirs(p.n_src);
  float4* explicit_table = nullptr;
  if (explicit_dirs) {
    const int32_t n = p.nrays[0];
    for (int64_t i = 0; i < int64_t(n) * 3; ++i)
      if (!std::isfinite(p.opts->directions[i])) return fail(RTMI_ERR_NONFINITE, "directions contain NaN/Inf");
    std::vector<float> xyz(p.opts->directions, p.opts->directions + size_t(n) * 3);
    const std::vector<float4> t = lane_table(xyz);
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&explicit_table), t.size() * sizeof(float4), p.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(directions)");
    e = hipMemcpyAsync(explicit_table, t.data(), t.size() * sizeof(float4), hipMemcpyHostToDevice, p.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(directions)");
    for (int32_t s = 0; s < p.n_src; ++s) dirs[s] = explicit_table;
  } else {
    for (int32_t s = 0; s < p.n_src; ++s)
      if (int32_t st = get_dirs(p.nrays[s], p.stream, &dirs[s])) return st;
  }

  // ---- output: zero, then accumulate ----
  const int64_t total = cells * p.n_bins;
  unsigned long long* acc = nullptr;
  double* det_scale = nullptr;
  hipError_t e;
  if (det) {
    e = hipMallocAsync(reinterpret_cast<void**>(&acc), size_t(total) * 8 + 16, p.stream);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(fixed-point field)");
    det_scale = reinterpret_cast<double*>(acc + total);
    if ((e = rtmi::launch_fill_zero_u64(acc, total, p.stream)) != hipSuccess) return hip_fail(e, "fill");
    const int64_t j_count = p.j_stride ? p.j_stride * (p.n_bins - 1) + cells : cells;
    if ((e = rtmi::launch_det_scale(p.j, j_count, bound_per_unit_j, det_scale, p.stream)) != hipSuccess)
      return hip_fail(e, "det_scale");
  } else {
    if ((e = rtmi::launch_fill_zero(p.out, total, p.stream)) != hipSuccess) return hip_fail(e, "fill");
  }

  for (int32_t b0 = 0; b0 < p.n_bins; b0 += kMaxBinsPerLaunch) {
    const int32_t nb = std::min<int32_t>(kMaxBinsPerLaunch, p.n_bins - b0);
    for (int32_t s0 = 0; s0 < p.n_src; s0 += kMaxSrcPerLaunch) {
      const int32_t ns = std::min<int32_t>(kMaxSrcPerLaunch, p.n_src - s0);
      rtmi::MarchArgs a;
      std::memset(&a, 0, sizeof a);
      a.j = p.j + b0 * p.j_stride;
      a.j_stride = p.j_stride;
      a.kap = p.kap + b0 * p.k_stride;
      a.k_stride = p.k_stride;
      for (int32_t b = 0; b < nb; ++b) a.kscale[b] = p.kscale ? p.kscale[b0 + b] : 1.0f;
      a.out = p.out + b0 * cells;
      a.acc = acc ? acc + b0 * cells : nullptr;
      a.det_scale = det_scale;
      a.out_stride = cells;
      a.nx = p.nx;
      a.ny = p.ny;
      a.nz = p.nz;
      a.ds = p.ds;
      a.n_src = ns;
      int blocks = 0;
      for (int32_t i = 0; i < ns; ++i) {
        const int32_t s = s0 + i;
        a.blk_begin[i] = blocks;
        a.sx[i] = p.src[3 * s];
        a.sy[i] = p.src[3 * s + 1];
        a.sz[i] = p.src[3 * s + 2];
        const double w = (explicit_dirs && p.opts->ray_weight > 0.0f) ? double(p.opts->ray_weight)
                                                                       : kFourPi / p.nrays[s];
        a.wray[i] = static_cast<float>(w);
        a.nrays[i] = nsub[s] > 0 ? p.nrays[s] : 0;
        a.nsub[i] = nsub[s];
        a.dirs[i] = dirs[s];
        blocks += (a.nrays[i] + kBlock - 1) / kBlock;
      }
      a.blk_begin[ns] = blocks;
      if (blocks == 0) continue;
      std::pair<hipEvent_t, hipEvent_t> ev{};
      bool timed = false;
      if ((e = timed_launch_begin(p.stream, &ev, &timed)) != hipSuccess) return hip_fail(e, "timing event");
      if ((e = rtmi::launch_march(a, nb, p.j_stride == 0, det, blocks, p.stream)) != hipSuccess)
        return hip_fail(e, "march launch");
      if ((e = timed_launch_end(p.stream, ev, timed)) != hipSuccess) return hip_fail(e, "timing event");
    }
  }

  if (det) {
    if ((e = rtmi::launch_det_convert(acc, det_scale, p.out, total, p.stream)) != hipSuccess)
      return hip_fail(e, "det_convert");
    if ((e = hipFreeAsync(acc, p.stream)) != hipSuccess) return hip_fail(e, "hipFreeAsync");
  }
  if (explicit_table && (e = hipFreeAsync(explicit_table, p.stream)) != hipSuccess)
    return hip_fail(e, "hipFreeAsync(directions)");
  g_error.clear();
  return RTMI_OK;
}

}  // namespace

extern "C" {

const char* rtmi_last_error(void) { return g_error.c_str(); }

int32_t rtmi_version(void) { return 100; }

int64_t rtmi_num_substeps(float step_size, float radiation_velocity, float time_step,
                          int32_t cap) {
  if (int32_t st = check_scalars(step_size, radiation_velocity, time_step)) return st;
  const int64_t n = substeps(step_size, radiation_velocity, time_step, cap);
  if (n < 0) return fail(RTMI_ERR_RANGE, "N_s = ceil(c dt / ds) exceeds 2^24");
  return n;
}

int32_t rtmi_fibonacci_directions(int32_t n, float* host_xyz) {
  if (!host_xyz) return fail(RTMI_ERR_INVALID_ARG, "null output pointer");
  if (n < 1 || n > kMaxCount) return fail(RTMI_ERR_INVALID_ARG, "n must be in [1, 2^24]");
  std::vector<float> xyz;
  fibonacci_host(n, xyz);
  std::memcpy(host_xyz, xyz.data(), xyz.size() * sizeof(float));
  return RTMI_OK;
}

int32_t rtmi_prepare(int32_t num_rays) {
  if (num_rays < 1 || num_rays > kMaxCount) return fail(RTMI_ERR_INVALID_ARG, "num_rays must be in [1, 2^24]");
  const float4* d = nullptr;
  return get_dirs(num_rays, nullptr, &d);
}

int32_t rtmi_trace_single(const float* j_map, const float* kappa_map, int32_t nx, int32_t ny,
                          int32_t nz, const float* source_pos, int32_t num_rays,
                          float step_size, float radiation_velocity, float time_step,
                          float* out_field, void* stream) {
  const Problem p{j_map, 0, kappa_map, 0, nullptr, 1, nx, ny, nz, 1, source_pos, &num_rays,
                  nullptr, step_size, radiation_velocity, time_step, out_field, nullptr,
                  static_cast<hipStream_t>(stream)};
  return run(p);
}

int32_t rtmi_trace_multi(const float* j_map, const float* kappa_map, int32_t nx, int32_t ny,
                         int32_t nz, int32_t n_src, const float* source_pos,
                         const int32_t* num_rays, const int32_t* substep_cap, float step_size,
                         float radiation_velocity, float time_step, float* out_field,
                         void* stream) {
  const Problem p{j_map, 0, kappa_map, 0, nullptr, 1, nx, ny, nz, n_src, source_pos, num_rays,
                  substep_cap, step_size, radiation_velocity, time_step, out_field, nullptr,
                  static_cast<hipStream_t>(stream)};
  return run(p);
}

int32_t rtmi_trace_bins(const float* j_maps, int64_t j_bin_stride, const float* kappa_maps,
                        int64_t kappa_bin_stride, const float* kappa_scale, int32_t n_bins,
                        int32_t nx, int32_t ny, int32_t nz, int32_t n_src,
                        const float* source_pos, const int32_t* num_rays,
                        const int32_t* substep_cap, float step_size, float radiation_velocity,
                        float time_step, float* out_fields, const rtmi_options* opts,
                        void* stream) {
  const Problem p{j_maps, j_bin_stride, kappa_maps, kappa_bin_stride,
                  kappa_bin_stride ? nullptr : kappa_scale, n_bins, nx, ny, nz, n_src,
                  source_pos, num_rays, substep_cap, step_size, radiation_velocity, time_step,
                  out_fields, opts, static_cast<hipStream_t>(stream)};
  return run(p);
}

int32_t rtmi_debug_rays(const float* j_map, const float* kappa_map, int32_t nx, int32_t ny,
                        int32_t nz, const float* source_pos, int32_t num_rays, float step_size,
                        float radiation_velocity, float time_step, int32_t cap, float* out_rays,
                        float* out_tau, void* stream) {
  if (!j_map || !kappa_map || !source_pos || !out_rays)
    return fail(RTMI_ERR_INVALID_ARG, "null map, source_pos or output pointer");
  if (int32_t st = check_shape(nx, ny, nz)) return st;
  if (int32_t st = check_scalars(step_size, radiation_velocity, time_step)) return st;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(source_pos[a])) return fail(RTMI_ERR_NONFINITE, "source_pos is not finite");
  if (num_rays < 1 || num_rays > kMaxCount) return fail(RTMI_ERR_INVALID_ARG, "num_rays must be in [1, 2^24]");
  const int64_t n = substeps(step_size, radiation_velocity, time_step, cap);
  if (n < 0) return fail(RTMI_ERR_RANGE, "N_s exceeds 2^24");
  if (n == 0) return RTMI_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  rtmi::DebugArgs a;
  std::memset(&a, 0, sizeof a);
  if (int32_t st = get_dirs(num_rays, s, &a.dirs)) return st;
  a.j = j_map;
  a.kap = kappa_map;
  a.out_rays = out_rays;
  a.out_tau = out_tau;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.ds = step_size;
  a.sx = source_pos[0];
  a.sy = source_pos[1];
  a.sz = source_pos[2];
  a.nrays = num_rays;
  a.nsub = static_cast<int>(n);
  const hipError_t e = rtmi::launch_debug(a, s);
  if (e != hipSuccess) return hip_fail(e, "debug launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lock(g_tmu);
  g_timing = on != 0;
  for (auto& ev : g_pending) g_free.push_back(ev);
  g_pending.clear();
  return RTMI_OK;
}

int32_t rtmi_timing_read(double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return fail(RTMI_ERR_INVALID_ARG, "null output pointer");
  std::lock_guard<std::mutex> lock(g_tmu);
  double sum = 0.0;
  for (auto& ev : g_pending) {
    hipError_t e = hipEventSynchronize(ev.second);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
    if (e != hipSuccess) return hip_fail(e, "reading timing events");
    sum += ms;
  }
  *total_ms = sum;
  *launches = static_cast<int64_t>(g_pending.size());
  for (auto& ev : g_pending) g_free.push_back(ev);
  g_pending.clear();
  return RTMI_OK;
}

}  // extern "C"
