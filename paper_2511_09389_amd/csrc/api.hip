// Host layer of librtmi: argument validation, substep count, direction tables, workspace,
// and the launch sequences of the two execution paths.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <memory>
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
using rtmi::kPatch;
using rtmi::kRowAlign;
using rtmi::kTile;

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

int32_t check_conv_shape(int32_t n, int32_t d, int32_t h, int32_t w) {
  if (n < 1 || d < 1 || h < 1 || w < 1) return fail(RTMI_ERR_SHAPE, "conv extents must be >= 1");
  if (int64_t(n) * d * h * w * rtmi::kConvChannels > (int64_t(1) << 40))
    return fail(RTMI_ERR_SHAPE, "conv tensor too large");
  return RTMI_OK;
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

// Distance along a Hilbert curve through a 2^k x 2^k grid (standard bit-twiddling form).
uint32_t hilbert_index(uint32_t side, uint32_t x, uint32_t y) {
  uint32_t d = 0;
  for (uint32_t s = side / 2; s > 0; s /= 2) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - x;
        y = s - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

// Lane order of the rays: sorted along a Hilbert curve drawn on the octahedral map of
// the sphere, so that each run of 64 lanes (one wavefront) holds a compact patch of
// directions. The sum over rays does not depend on this order.
std::vector<size_t> coherent_order(const std::vector<float>& xyz) {
  const size_t n = xyz.size() / 3;
  std::vector<uint32_t> key(n);
  for (size_t i = 0; i < n; ++i) {
    const double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    const double l1 = std::fabs(x) + std::fabs(y) + std::fabs(z);
    double u = l1 > 0 ? x / l1 : 0.0, v = l1 > 0 ? y / l1 : 0.0;
    if (z < 0) {
      const double uu = (1.0 - std::fabs(v)) * (u >= 0 ? 1.0 : -1.0);
      const double vv = (1.0 - std::fabs(u)) * (v >= 0 ? 1.0 : -1.0);
      u = uu;
      v = vv;
    }
    const uint32_t qx = std::min<uint32_t>(1023u, static_cast<uint32_t>((u + 1.0) * 512.0));
    const uint32_t qy = std::min<uint32_t>(1023u, static_cast<uint32_t>((v + 1.0) * 512.0));
    key[i] = hilbert_index(1024u, qx, qy);
  }
  std::vector<size_t> ord(n);
  for (size_t i = 0; i < n; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
  return ord;
}

// Device-side direction table: float4 (x, y, z, bits of the lattice index) per lane in
// coherent order, followed by per-patch direction bounds (8 floats per 64 lanes).
struct HostTable {
  std::vector<float4> dirs;
  std::vector<float> bounds;
};

HostTable build_table(const std::vector<float>& xyz) {
  const size_t n = xyz.size() / 3;
  const std::vector<size_t> ord = coherent_order(xyz);
  HostTable t;
  t.dirs.resize(n);
  for (size_t lane = 0; lane < n; ++lane) {
    const size_t i = ord[lane];
    int32_t idx = static_cast<int32_t>(i);
    float w;
    std::memcpy(&w, &idx, sizeof w);
    t.dirs[lane] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], w);
  }
  const size_t np = (n + kPatch - 1) / kPatch;
  t.bounds.assign(np * rtmi::kPatchRec, 0.0f);
  for (size_t p = 0; p < np; ++p) {
    float* rec = &t.bounds[p * rtmi::kPatchRec];
    const size_t l0 = p * kPatch, l1 = std::min(n, (p + 1) * kPatch);
    float lo[3] = {2.f, 2.f, 2.f}, hi[3] = {-2.f, -2.f, -2.f};
    double axis[3] = {0.0, 0.0, 0.0};
    for (size_t lane = l0; lane < l1; ++lane) {
      const float c[3] = {t.dirs[lane].x, t.dirs[lane].y, t.dirs[lane].z};
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], c[a]);
        hi[a] = std::max(hi[a], c[a]);
        axis[a] += c[a];
      }
    }
    // cone around the mean direction that holds every ray of the patch (a whole-sphere
    // cone when the patch's mean direction degenerates)
    const double len = std::sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
    double cos_b = -1.0;
    if (len > 1e-9) {
      for (int a = 0; a < 3; ++a) axis[a] /= len;
      cos_b = 1.0;
      for (size_t lane = l0; lane < l1; ++lane) {
        const double dn = std::sqrt(double(t.dirs[lane].x) * t.dirs[lane].x +
                                    double(t.dirs[lane].y) * t.dirs[lane].y +
                                    double(t.dirs[lane].z) * t.dirs[lane].z);
        const double c = (axis[0] * t.dirs[lane].x + axis[1] * t.dirs[lane].y + axis[2] * t.dirs[lane].z) / dn;
        cos_b = std::min(cos_b, c);
      }
      // widen by 2e-3 rad: the kernel compares binary32 cosines, whose rounding near 1
      // is worth a few 1e-4 rad of angle
      const double b = std::acos(std::max(-1.0, std::min(1.0, cos_b))) + 2e-3;
      cos_b = b >= 3.14159265358979323846 ? -1.0 : std::cos(b);
    } else {
      axis[0] = 1.0;
      axis[1] = axis[2] = 0.0;
    }
    for (int a = 0; a < 3; ++a) {
      rec[a] = lo[a];
      rec[3 + a] = hi[a];
      rec[8 + a] = static_cast<float>(axis[a]);
    }
    rec[11] = static_cast<float>(cos_b);
    rec[12] = static_cast<float>(std::sqrt(std::max(0.0, 1.0 - cos_b * cos_b)));
  }
  return t;
}

struct DevTable {
  float4* dirs = nullptr;
  float* bounds = nullptr;
};

size_t table_bytes(const HostTable& t) {
  return t.dirs.size() * sizeof(float4) + t.bounds.size() * sizeof(float);
}

std::mutex g_mu;
std::map<std::pair<int, int32_t>, DevTable> g_dirs;  // (device, N) -> table, kept for the process
std::map<int, hipMemPool_t> g_pools;                  // device -> workspace pool

int32_t current_device(int* dev) {
  const hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return RTMI_OK;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  return s != nullptr && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
}

int32_t get_dirs(int32_t n, hipStream_t stream, DevTable* out, bool may_alloc = true) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_dirs.find({dev, n});
  if (it != g_dirs.end()) {
    *out = it->second;
    return RTMI_OK;
  }
  if (!may_alloc)
    return fail(RTMI_ERR_UNSUPPORTED,
                "direction table for %d rays not prepared on this device; call rtmi_prepare(%d) first", n, n);
  if (capturing(stream))
    return fail(RTMI_ERR_UNSUPPORTED,
                "direction table for %d rays not prepared; call rtmi_prepare before capture", n);
  std::vector<float> xyz;
  fibonacci_host(n, xyz);
  const HostTable t = build_table(xyz);
  char* d = nullptr;
  hipError_t e = hipMalloc(&d, table_bytes(t));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(direction table)");
  const size_t db = t.dirs.size() * sizeof(float4);
  e = hipMemcpy(d, t.dirs.data(), db, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d + db, t.bounds.data(), t.bounds.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(e, "hipMemcpy(direction table)");
  }
  DevTable dt;
  dt.dirs = reinterpret_cast<float4*>(d);
  dt.bounds = reinterpret_cast<float*>(d + db);
  g_dirs[{dev, n}] = dt;
  *out = dt;
  return RTMI_OK;
}

// Workspace pool of the current device: a private stream-ordered pool that keeps what it
// has allocated, so that repeated calls reuse memory instead of going back to the system.
int32_t get_pool(hipMemPool_t* pool) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_pools.find(dev);
  if (it != g_pools.end()) {
    *pool = it->second;
    return RTMI_OK;
  }
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof props);
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t p = nullptr;
  hipError_t e = hipMemPoolCreate(&p, &props);
  if (e != hipSuccess) return hip_fail(e, "hipMemPoolCreate");
  uint64_t keep = UINT64_MAX;
  e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return hip_fail(e, "hipMemPoolSetAttribute");
  g_pools[dev] = p;
  *pool = p;
  return RTMI_OK;
}

int32_t pool_alloc(void** ptr, size_t bytes, hipStream_t s) {
  hipMemPool_t pool = nullptr;
  if (int32_t st = get_pool(&pool)) return st;
  const hipError_t e = hipMallocFromPoolAsync(ptr, std::max<size_t>(bytes, 256), pool, s);
  if (e != hipSuccess) return hip_fail(e, "workspace allocation");
  return RTMI_OK;
}

// Scratch of the stateless calls, kept per (device, stream, purpose) and reused by the
// next call on the same stream: stream order makes the reuse safe (the call before has
// finished with it by the time the next one's kernels run), and it spares a stream-ordered
// free per call, which costs a few hundred microseconds of host time on this runtime,
// more than a whole 128^3 march. A call that needs more grows it (the old block is freed
// in stream order). Under graph capture a call takes its own stream-ordered allocation,
// which the graph owns. The cached blocks are held until the process ends.
enum WorkspaceSlot { kSlotTiled = 0, kSlotFixedPoint = 1, kSlotAdjoint = 2, kSlotConv = 3 };

struct Scratch {
  char* ptr = nullptr;
  bool owned = false;   // freed by the caller (captured allocation)
  hipError_t release(hipStream_t s) { return owned ? hipFreeAsync(ptr, s) : hipSuccess; }
};

std::mutex g_scratch_mu;   // (not g_mu: the pool lookup below takes that one)
std::map<std::tuple<int, hipStream_t, int>, std::pair<char*, size_t>> g_scratch;

int32_t acquire_scratch(size_t bytes, hipStream_t s, WorkspaceSlot slot, Scratch* out) {
  bytes = std::max<size_t>(bytes, 256);
  if (capturing(s)) {
    out->owned = true;
    return pool_alloc(reinterpret_cast<void**>(&out->ptr), bytes, s);
  }
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto& held = g_scratch[std::make_tuple(dev, s, static_cast<int>(slot))];
  if (held.second < bytes) {
    if (held.first) {
      const hipError_t e = hipFreeAsync(held.first, s);
      held = {nullptr, 0};
      if (e != hipSuccess) return hip_fail(e, "workspace release");
    }
    void* p = nullptr;
    if (int32_t rc = pool_alloc(&p, bytes, s)) return rc;
    held = {static_cast<char*>(p), bytes};
  }
  out->ptr = held.first;
  out->owned = false;
  return RTMI_OK;
}

// ---- chunk records the stateless calls could not store (reported by rtmi_dropped_records) ----
// One counter per device: this file-scope device variable, whose per-device address is
// looked up once per device and passed to the schedule kernels.
__device__ unsigned long long g_dropped_records;

std::mutex g_dropped_mu;
std::map<int, unsigned long long*> g_dropped_ptr;

int32_t dropped_counter(unsigned long long** out) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_dropped_mu);
  auto it = g_dropped_ptr.find(dev);
  if (it == g_dropped_ptr.end()) {
    unsigned long long* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(g_dropped_records));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(dropped-record counter)");
    it = g_dropped_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return RTMI_OK;
}

// ---- the scratch of rtmi_trace_bins_static: a fixed device array, nothing allocated ----
// Each device that runs the library holds its own copy of this array for the life of the
// process. Host code never passes the array's name to a kernel or a copy (on the host it
// only names the symbol): it looks up the array's address on each device once, with that
// device current, and uses that address.
constexpr size_t kStaticScratchBytes = size_t(384) << 20;
static __device__ __align__(256) unsigned char g_static_scratch[kStaticScratchBytes];

std::mutex g_static_mu;
std::map<int, char*> g_static_ptr;   // device -> address of its copy of g_static_scratch

int32_t static_scratch(char** out) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  std::lock_guard<std::mutex> lock(g_static_mu);
  auto it = g_static_ptr.find(dev);
  if (it == g_static_ptr.end()) {
    char* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(g_static_scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(static scratch)");
    if (!ptr) return fail(RTMI_ERR_HIP, "hipGetSymbolAddress(static scratch) returned a null address");
    it = g_static_ptr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return RTMI_OK;
}

// ---- measurement hooks: event pairs around kernel launches, per kernel kind ----
std::mutex g_tmu;
bool g_timing = false;
using EventPair = std::pair<hipEvent_t, hipEvent_t>;
std::vector<EventPair> g_pending[5];  // recorded, not yet read
std::vector<EventPair> g_free;

struct TimedLaunch {
  EventPair ev{};
  bool on = false;
  int kind = 0;
};

// (allowed = false: a call that may not allocate, so it creates no events either)
hipError_t timed_begin(hipStream_t s, int kind, TimedLaunch* t, bool allowed = true) {
  std::lock_guard<std::mutex> lock(g_tmu);
  t->on = g_timing && allowed;
  t->kind = kind;
  if (!g_timing) return hipSuccess;
  if (g_free.empty()) {
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    g_free.push_back({a, b});
  }
  t->ev = g_free.back();
  g_free.pop_back();
  return hipEventRecord(t->ev.first, s);
}

hipError_t timed_end(hipStream_t s, const TimedLaunch& t) {
  if (!t.on) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_tmu);
  const hipError_t e = hipEventRecord(t.ev.second, s);
  g_pending[t.kind].push_back(t.ev);
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

// Everything a validated call needs to enqueue work.
struct Plan {
  bool det = false;
  bool tiled = true;
  bool explicit_dirs = false;
  int32_t item_chunks = 0;  // tile work-item size; 0: kItemChunks
  int64_t record_capacity = 0;  // > 0: stateless chunk-record buffers capped (test hook)
  bool no_alloc = false;        // the call may not allocate (static scratch, no events)
  int32_t gather_table = 0;     // 0 auto, 1 gather j and kappa from the 64-byte table, 2 from the maps
  int32_t sources_per_launch = 0;   // > 0: at most this many sources per record launch
  int32_t tile_groups_per_cu = 0;   // > 0: cap on the persistent tile grid per compute unit
  std::vector<int32_t> nsub;
  std::vector<DevTable> tables;
  double bound_per_unit_j = 0.0;
  double det_growth = 0.0;   // N_s ds, largest over sources
  double kscale_max = 1.0;   // largest |kappa_scale| (1 without scales)
  int64_t cells = 0;
};

// maps_given: the call carries its maps and field (false when a plan is made without them)
int32_t validate(const Problem& p, Plan* plan, bool maps_given = true) {
  if (maps_given && (!p.j || !p.kap || !p.out))
    return fail(RTMI_ERR_INVALID_ARG, "null map or field pointer");
  if (!p.src || !p.nrays) return fail(RTMI_ERR_INVALID_ARG, "null source_pos or num_rays pointer");
  if (int32_t st = check_shape(p.nx, p.ny, p.nz)) return st;
  if (int32_t st = check_scalars(p.ds, p.c, p.dt)) return st;
  if (p.n_src < 1) return fail(RTMI_ERR_INVALID_ARG, "n_src must be >= 1 (got %d)", p.n_src);
  if (p.n_bins < 1) return fail(RTMI_ERR_INVALID_ARG, "n_bins must be >= 1 (got %d)", p.n_bins);
  if (p.j_stride < 0 || p.k_stride < 0) return fail(RTMI_ERR_INVALID_ARG, "bin strides must be >= 0");
  plan->cells = int64_t(p.nx) * p.ny * p.nz;
  if (p.n_bins > 1 && ((p.j_stride != 0 && p.j_stride < plan->cells) ||
                       (p.k_stride != 0 && p.k_stride < plan->cells)))
    return fail(RTMI_ERR_INVALID_ARG, "a non-zero bin stride must be >= nx*ny*nz");
  if (p.kscale)
    for (int32_t b = 0; b < p.n_bins; ++b) {
      if (!std::isfinite(p.kscale[b])) return fail(RTMI_ERR_NONFINITE, "kappa_scale[%d] is not finite", b);
      plan->kscale_max = std::max(plan->kscale_max, std::fabs(double(p.kscale[b])));
    }
  if (p.opts) {
    if (p.opts->accum_mode != RTMI_ACCUM_ATOMIC && p.opts->accum_mode != RTMI_ACCUM_DETERMINISTIC)
      return fail(RTMI_ERR_INVALID_ARG, "unknown accum_mode %d", p.opts->accum_mode);
    if (p.opts->path != RTMI_PATH_TILED && p.opts->path != RTMI_PATH_DIRECT)
      return fail(RTMI_ERR_INVALID_ARG, "unknown path %d", p.opts->path);
    plan->det = p.opts->accum_mode == RTMI_ACCUM_DETERMINISTIC;
    if (plan->det && p.kscale)
      for (int32_t b = 0; b < p.n_bins; ++b)
        if (p.kscale[b] < 0.0f)
          return fail(RTMI_ERR_INVALID_ARG, "the deterministic mode needs kappa_scale >= 0 (bin %d: %g)", b,
                      double(p.kscale[b]));
    plan->tiled = p.opts->path == RTMI_PATH_TILED;
    plan->explicit_dirs = p.opts->directions != nullptr;
    if (p.opts->tile_item_chunks < 0 || p.opts->tile_item_chunks > (1 << 20))
      return fail(RTMI_ERR_INVALID_ARG, "tile_item_chunks must be in [0, 2^20] (got %d)",
                  p.opts->tile_item_chunks);
    plan->item_chunks = p.opts->tile_item_chunks;
    if (p.opts->record_capacity < 0)
      return fail(RTMI_ERR_INVALID_ARG, "record_capacity must be >= 0");
    plan->record_capacity = p.opts->record_capacity;
    if (p.opts->gather_table < 0 || p.opts->gather_table > 3)
      return fail(RTMI_ERR_INVALID_ARG, "gather_table must be 0, 1, 2 or 3 (got %d)", p.opts->gather_table);
    plan->gather_table = p.opts->gather_table;
    if (p.opts->sources_per_launch < 0)
      return fail(RTMI_ERR_INVALID_ARG, "sources_per_launch must be >= 0 (got %d)", p.opts->sources_per_launch);
    plan->sources_per_launch = p.opts->sources_per_launch;
    if (p.opts->tile_groups_per_cu < 0)
      return fail(RTMI_ERR_INVALID_ARG, "tile_groups_per_cu must be >= 0 (got %d)", p.opts->tile_groups_per_cu);
    plan->tile_groups_per_cu = p.opts->tile_groups_per_cu;
    if (plan->explicit_dirs && p.opts->ray_weight > 0.0f && !std::isfinite(p.opts->ray_weight))
      return fail(RTMI_ERR_NONFINITE, "ray_weight is not finite");
  }
  plan->nsub.resize(p.n_src);
  for (int32_t s = 0; s < p.n_src; ++s) {
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p.src[3 * s + a])) return fail(RTMI_ERR_NONFINITE, "source_pos[%d] is not finite", s);
    if (p.nrays[s] < 1 || p.nrays[s] > kMaxCount)
      return fail(p.nrays[s] < 1 ? RTMI_ERR_INVALID_ARG : RTMI_ERR_RANGE,
                  "num_rays[%d] = %d must be in [1, 2^24]", s, p.nrays[s]);
    if (plan->explicit_dirs && p.nrays[s] != p.nrays[0])
      return fail(RTMI_ERR_INVALID_ARG, "explicit directions need one num_rays for all sources");
    const int64_t n = substeps(p.ds, p.c, p.dt, p.caps ? p.caps[s] : 0);
    if (n < 0) return fail(RTMI_ERR_RANGE, "N_s = ceil(c dt / ds) exceeds 2^24");
    plan->nsub[s] = static_cast<int32_t>(n);
    // I <= N_s ds max|j| (exp factors <= 1 for kappa >= 0); each ray deposits at most
    // N_s times into one voxel with weight <= 1, times its ray weight, over N_Omega rays.
    // (A negative kappa multiplies this by at most exp(N_s ds max(-kappa)): det_growth.)
    const double wray = (plan->explicit_dirs && p.opts->ray_weight > 0.0f) ? double(p.opts->ray_weight)
                                                                           : kFourPi / p.nrays[s];
    plan->bound_per_unit_j += wray * double(p.nrays[s]) * double(n) * double(n) * double(p.ds);
    plan->det_growth = std::max(plan->det_growth, double(n) * double(p.ds));
  }
  if (plan->explicit_dirs)
    for (int64_t i = 0; i < int64_t(p.nrays[0]) * 3; ++i)
      if (!std::isfinite(p.opts->directions[i])) return fail(RTMI_ERR_NONFINITE, "directions contain NaN/Inf");
  return RTMI_OK;
}

float ray_weight(const Problem& p, const Plan& plan, int32_t s) {
  const double w = (plan.explicit_dirs && p.opts->ray_weight > 0.0f) ? double(p.opts->ray_weight)
                                                                     : kFourPi / p.nrays[s];
  return static_cast<float>(w);
}

// Fixed-point scale of the deterministic mode, on the device: from max|j| over the bins'
// j and max(0, -kappa) over their kappa (which widens the bound by exp(N_s ds |kappa|)).
hipError_t det_scale_launch(const Problem& p, const Plan& plan, double* det_scale) {
  const int64_t j_count = p.j_stride ? p.j_stride * (p.n_bins - 1) + plan.cells : plan.cells;
  const int64_t k_count = p.k_stride ? p.k_stride * (p.n_bins - 1) + plan.cells : plan.cells;
  return rtmi::launch_det_scale(p.j, j_count, p.kap, k_count, plan.kscale_max * plan.det_growth,
                                plan.bound_per_unit_j, det_scale, p.stream);
}

size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Target chunks (ray segments of up to kChunk substeps inside one tile) per tile work
// item when the caller does not choose: two rounds of the work-group's lanes.
constexpr int kItemChunks = 2 * rtmi::kTileThreads;

// Schedule buffers of the tile launches, carved from the workspace.
struct TileSchedule {
  unsigned long long* cost = nullptr;
  long long *begin = nullptr, *count = nullptr, *fill = nullptr;
  unsigned* mask = nullptr;   // per (tile, block of kPairBlock pairs): pairs with chunks
  int2* map = nullptr;
  int* counters = nullptr;   // item total, next, done; the record total at byte 16
  static size_t mask_bytes(int tiles, int pair_blocks) {
    return align256(size_t(tiles) * std::max(pair_blocks, 1) * (rtmi::kPairBlock / 32) * sizeof(unsigned));
  }
  static size_t bytes(int tiles, int pair_blocks) {
    return 4 * align256(size_t(tiles) * 8) + mask_bytes(tiles, pair_blocks) +
           align256(size_t(tiles) * rtmi::kMaxParts * sizeof(int2)) + 256;
  }
  void carve(char* base, int tiles, int pair_blocks) {
    const size_t per = align256(size_t(tiles) * 8);
    cost = reinterpret_cast<unsigned long long*>(base);
    begin = reinterpret_cast<long long*>(base + per);
    count = reinterpret_cast<long long*>(base + 2 * per);
    fill = reinterpret_cast<long long*>(base + 3 * per);
    mask = reinterpret_cast<unsigned*>(base + 4 * per);
    base += 4 * per + mask_bytes(tiles, pair_blocks);
    map = reinterpret_cast<int2*>(base);
    counters = reinterpret_cast<int*>(base + align256(size_t(tiles) * rtmi::kMaxParts * sizeof(int2)));
  }
  long long* rec_total() const { return reinterpret_cast<long long*>(counters + 4); }
  void apply(rtmi::TileArgs& t, int item_chunks, uint2* recs, int64_t capacity,
             unsigned long long* dropped = nullptr) const {
    t.dropped = dropped;
    t.tile_cost = cost;
    t.tile_begin = begin;
    t.tile_count = count;
    t.tile_fill = fill;
    t.pair_mask = mask;
    t.rec_total = rec_total();
    t.recs = recs;
    t.rec_capacity = capacity;
    t.item_map = map;
    t.item_total = counters;
    t.item_next = counters + 1;
    t.item_done = counters + 2;
    t.item_chunks = item_chunks > 0 ? item_chunks : kItemChunks;
  }
};

// Blocks of kPairBlock (source, patch) pairs in a launch of sources [s0, s0 + ns).
int pair_blocks(const Problem& p, const Plan& plan, int32_t s0, int32_t ns) {
  int64_t patches = 0;
  for (int32_t s = s0; s < s0 + ns; ++s)
    if (plan.nsub[s] > 0) patches += (p.nrays[s] + kPatch - 1) / kPatch;
  return static_cast<int>((patches + rtmi::kPairBlock - 1) / rtmi::kPairBlock);
}

// Upper bound on the chunk records that sources [s0, s0 + ns) can produce. A tile lists a
// chunk (kChunk substeps from 8c) when its substep range [ka, kb] meets the chunk, and
// that range lies within two substeps (plus division rounding) of the ray's parameter
// interval inside the tile widened by the stencil and the margin m. So the ray, over
// t in [(8c - 2) ds, (8c + 9) ds] (widened for rounding to 13 ds), meets that tile's
// widened box, whose extent along an axis is at most 17 + 4m with a stride of 16 between
// tiles: at most floor((13 ds + 17 + 4m) / 16) + 1 tiles per axis, which for m <= 1/2 is
// floor((13 ds + 19) / 16) + 1. (The fill kernel also never writes past the buffer.)
int64_t record_bound(const Problem& p, const Plan& plan, int32_t s0, int32_t ns, int tiles_x, int tiles_y,
                     int tiles_z) {
  int64_t total = 0;
  for (int32_t s = s0; s < s0 + ns; ++s) {
    if (plan.nsub[s] <= 0) continue;
    const double tmax = double(plan.nsub[s] - 1) * p.ds;
    const double amax = std::max(std::fabs(double(p.src[3 * s])),
                                 std::max(std::fabs(double(p.src[3 * s + 1])), std::fabs(double(p.src[3 * s + 2]))));
    const double m = 5.0e-7 * (amax + tmax + 2.0) + 1.0e-6;
    const int64_t per_axis = m <= 0.5 ? int64_t(std::floor((13.0 * p.ds + 19.0) / 16.0)) + 1 : int64_t(1) << 30;
    const int64_t f = std::min<int64_t>(per_axis, tiles_x) * std::min<int64_t>(per_axis, tiles_y) *
                      std::min<int64_t>(per_axis, tiles_z);
    total += int64_t(p.nrays[s]) * ((plan.nsub[s] + rtmi::kChunk - 1) / rtmi::kChunk) * f;
  }
  return total;
}

// A plan's chunk records: one slice per launch, sized exactly at plan creation.
struct RecordSlices {
  uint2* base = nullptr;
  std::vector<int64_t> off, count;
};

int64_t row_stride(int32_t nsub) { return (int64_t(nsub) + kRowAlign - 1) / kRowAlign * kRowAlign; }

// ---- tiled path: record + tile per (bin chunk, source chunk) ----

// Source groups of the tiled path: runs of consecutive sources that one record launch
// and one tile pass per bin cover. A group ends where its deposit rows would pass
// kGroupRowBytes (so the workspace stays bounded for thousands of sources), where the
// gather pass's (j, kappa) rows would pass kGroupJkBytes (the reach of its stores' 32-bit
// byte offsets), or at kMaxSrcPerTiledLaunch sources (or the caller's sources_per_launch).
constexpr int64_t kGroupRowBytes = int64_t(4) << 30;
constexpr int64_t kGroupJkBytes = (int64_t(4) << 30) - 256;
bool use_gather_pass(const Plan& plan);

struct SourceGroup {
  int32_t s0 = 0, ns = 0;
};

std::vector<SourceGroup> source_groups(const Problem& p, const Plan& plan) {
  const int64_t nb = std::min(kMaxBinsPerLaunch, p.n_bins);
  const bool jk = p.j_stride == 0 && p.k_stride == 0 && use_gather_pass(plan);
  std::vector<SourceGroup> g;
  int64_t bytes = 0, jk_bytes = 0;
  for (int32_t s = 0; s < p.n_src; ++s) {
    const int64_t e = plan.nsub[s] > 0 ? int64_t(p.nrays[s]) * row_stride(plan.nsub[s]) : 0;
    const int64_t b = e * nb * 4, bj = jk ? e * 8 : 0;
    const int32_t cap = plan.sources_per_launch > 0 ? std::min(plan.sources_per_launch, rtmi::kMaxSrcPerTiledLaunch)
                                                    : rtmi::kMaxSrcPerTiledLaunch;
    if (g.empty() || (g.back().ns > 0 && (bytes + b > kGroupRowBytes || jk_bytes + bj > kGroupJkBytes)) ||
        g.back().ns >= cap) {
      g.push_back({s, 0});
      bytes = 0;
      jk_bytes = 0;
    }
    g.back().ns += 1;
    bytes += b;
    jk_bytes += bj;
  }
  return g;
}

// Workspace of a tiled execution: corner sums, the device source table, tile schedules
// (one shared by all launches, or one per launch when a plan keeps them), the
// interleaved (j, kappa) copy and the recorded rows of the largest launch.
struct TiledLayout {
  int tiles_x = 0, tiles_y = 0, tiles_z = 0, tiles = 0;
  int n_launch = 0;
  bool interleaved = false;   // the 64-byte gather table
  bool jk_rows = false;       // or the gather pass's (j, kappa) rows
  size_t corner = 0, srcs = 0, sched = 0, med = 0, v = 0, p = 0, segtot = 0, recs = 0, total = 0;   // byte offsets / size
  size_t sched_bytes = 0;
  int pair_blocks = 0;        // most pair blocks of any launch
  int64_t rec_capacity = 0;   // chunk records of each shared buffer (0: a plan's own slices)
  int rec_buffers = 1;        // shared buffers: two when several launches alternate
  std::vector<SourceGroup> groups;
  std::vector<int> seg_len;   // per source group: substeps per record run (0: whole rays)
};

// Substeps per record run for a launch of `rays` rays of at most max_nsub substeps: the
// rays are cut into runs when they alone would give the device less than one wave per
// SIMD, keeping runs at least two gather chunks long. (With a wave per SIMD already, more
// runs measured slower: the gathers, not the latency of one ray's chain, bound the
// kernel, and the fixup pass costs extra traffic.)
int record_run_length(int64_t rays, int32_t max_nsub) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    cus = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) ? v : 256;
  }
  if (rays < 1 || max_nsub < 1) return 0;
  const int64_t target = int64_t(cus) * 4 * 64;
  int runs = static_cast<int>(std::min<int64_t>(8, (target + rays - 1) / rays));
  while (runs > 1 && (max_nsub + runs - 1) / runs < 2 * kRowAlign) --runs;
  if (runs <= 1) return 0;
  const int len = (max_nsub + runs - 1) / runs;
  return (len + kRowAlign - 1) / kRowAlign * kRowAlign;
}

constexpr size_t kCornerBytes = 256;   // [4][8] floats, then (next 256 B) [4][8] u64

// The 64-byte-per-voxel gather table measured faster than gathering from the maps at
// every grid size tried (128^3: record pass 0.13 vs 0.43 ms; 256^3, where the table no
// longer fits the Infinity Cache: 1.06 vs 2.05 ms).
bool use_gather_table(const Plan& plan) {
  if (plan.gather_table != 0) return plan.gather_table == 1;
  return true;
}

// The gather pass (option 3): j and kappa of every sample gathered tile by tile into rows
// that the record pass reads in whole 64-byte pieces. By default it replaces the 64-byte
// table once the table outgrows the 256 MB Infinity Cache (the record pass then reads
// the table from HBM several times over: 256^3, 4.94 -> 4.24 ms per uneven step), and
// not below (128^3: the table, 0.33 ms per step, beats the pass, 0.35 ms).
bool use_gather_pass(const Plan& plan) {
  if (plan.gather_table != 0) return plan.gather_table == 3;
  return plan.cells * 64 > (int64_t(256) << 20);
}

TiledLayout tiled_layout(const Problem& p, const Plan& plan, bool sched_per_launch, bool shared_records) {
  TiledLayout L;
  L.tiles_x = (p.nx + kTile - 1) / kTile;
  L.tiles_y = (p.ny + kTile - 1) / kTile;
  L.tiles_z = (p.nz + kTile - 1) / kTile;
  L.tiles = L.tiles_x * L.tiles_y * L.tiles_z;
  L.groups = source_groups(p, plan);
  int64_t v_elems_max = 0, p_elems_max = 0, t_elems_max = 0;
  for (const SourceGroup& g : L.groups) {
    int64_t e = 0, rays = 0;
    int32_t max_nsub = 0;
    for (int32_t s = g.s0; s < g.s0 + g.ns; ++s)
      if (plan.nsub[s] > 0) {
        e += int64_t(p.nrays[s]) * row_stride(plan.nsub[s]);
        rays += p.nrays[s];
        max_nsub = std::max(max_nsub, plan.nsub[s]);
      }
    // (the deterministic mode marches whole rays: runs chained by the fix-up round their
    // values differently, and their length depends on the launch, so its bits would too)
    const int len = plan.det ? 0 : record_run_length(rays, max_nsub);
    L.seg_len.push_back(len);
    if (shared_records)
      L.rec_capacity = std::max(L.rec_capacity, record_bound(p, plan, g.s0, g.ns, L.tiles_x, L.tiles_y, L.tiles_z));
    L.pair_blocks = std::max(L.pair_blocks, pair_blocks(p, plan, g.s0, g.ns));
    int64_t t = 0;
    if (len > 0)
      for (int32_t s = g.s0; s < g.s0 + g.ns; ++s)
        if (plan.nsub[s] > 0) t += int64_t(p.nrays[s]) * ((plan.nsub[s] + len - 1) / len);
    v_elems_max = std::max(v_elems_max, e);
    p_elems_max = std::max(p_elems_max, len > 0 ? e : int64_t(0));
    t_elems_max = std::max(t_elems_max, t);
  }
  if (shared_records && plan.record_capacity > 0) L.rec_capacity = std::min(L.rec_capacity, plan.record_capacity);
  L.n_launch = static_cast<int>(L.groups.size()) * ((p.n_bins + kMaxBinsPerLaunch - 1) / kMaxBinsPerLaunch);
  const int32_t nb_max = std::min(kMaxBinsPerLaunch, p.n_bins);
  // a shared j and a shared (scaled) kappa are gathered from one interleaved copy
  L.jk_rows = p.j_stride == 0 && p.k_stride == 0 && use_gather_pass(plan);
  L.interleaved = p.j_stride == 0 && p.k_stride == 0 && !L.jk_rows && use_gather_table(plan);
  L.sched_bytes = TileSchedule::bytes(L.tiles, L.pair_blocks);
  L.corner = 0;
  L.srcs = 2 * kCornerBytes;
  L.sched = L.srcs + align256(size_t(p.n_src) * sizeof(rtmi::SrcRec));
  L.med = L.sched + L.sched_bytes * (sched_per_launch ? L.n_launch : 1);
  L.v = L.med + (L.interleaved ? align256(size_t(plan.cells) * 4 * sizeof(float4))
                                : L.jk_rows ? align256(size_t(v_elems_max) * sizeof(float2)) : 0);
  L.p = L.v + align256(size_t(v_elems_max) * nb_max * sizeof(float));
  L.segtot = L.p + align256(size_t(p_elems_max) * nb_max * sizeof(float));
  L.recs = L.segtot + align256(size_t(t_elems_max) * nb_max * sizeof(float2));
  L.rec_buffers = L.n_launch > 1 ? 2 : 1;
  L.total = L.recs + size_t(L.rec_buffers) * align256(size_t(L.rec_capacity) * sizeof(uint2));
  return L;
}

// A source group's device table in record-block order: sources are given to the XCDs
// greedily by cost (longest processing time first: blocks x substeps per block), and each
// XCD's sources run most costly first. Fills the table entries (without tmax and marg,
// which the device completes), the XCD group bounds of the record launch, and the pairs
// and fix-up totals of the group.
struct GroupTable {
  std::vector<rtmi::SrcRec> rec;
  int xcd_src[rtmi::kXcds + 1] = {0};
  int xcd_blocks[rtmi::kXcds] = {0};
  int n_pairs = 0, fix_waves = 0;
  int64_t v_elems = 0, t_elems = 0;
};

GroupTable group_table(const Problem& p, const Plan& plan, const SourceGroup& g, int seg_len) {
  constexpr int X = rtmi::kXcds;
  struct Item {
    int32_t s;
    int blocks;
    int64_t cost;
  };
  std::vector<Item> items;
  for (int32_t s = g.s0; s < g.s0 + g.ns; ++s) {
    const int32_t nr = plan.nsub[s] > 0 ? p.nrays[s] : 0;
    const int nseg = (seg_len > 0 && nr > 0) ? (plan.nsub[s] + seg_len - 1) / seg_len : 1;
    const int blocks = nseg * ((nr + kBlock - 1) / kBlock);
    const int per_block = seg_len > 0 ? std::min(seg_len, plan.nsub[s]) : plan.nsub[s];
    items.push_back({s, blocks, int64_t(blocks) * per_block});
  }
  std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.cost > b.cost; });
  std::vector<std::vector<Item>> per_xcd(X);
  int64_t load[X] = {0};
  for (const Item& it : items) {
    const int x = static_cast<int>(std::min_element(load, load + X) - load);
    per_xcd[x].push_back(it);
    load[x] += it.cost;
  }
  GroupTable T;
  int pairs = 0, fix = 0;
  for (int x = 0; x < X; ++x) {
    T.xcd_src[x] = static_cast<int>(T.rec.size());
    // each XCD's blocks most costly first: sort by the cost of one block
    std::stable_sort(per_xcd[x].begin(), per_xcd[x].end(), [&](const Item& a, const Item& b) {
      return plan.nsub[a.s] > plan.nsub[b.s];
    });
    int blk = 0;
    for (const Item& it : per_xcd[x]) {
      const int32_t s = it.s;
      const int32_t nr = plan.nsub[s] > 0 ? p.nrays[s] : 0;
      const int nseg = (seg_len > 0 && nr > 0) ? (plan.nsub[s] + seg_len - 1) / seg_len : 1;
      rtmi::SrcRec r;
      std::memset(&r, 0, sizeof r);
      r.sx = p.src[3 * s];
      r.sy = p.src[3 * s + 1];
      r.sz = p.src[3 * s + 2];
      r.wray = ray_weight(p, plan, s);
      r.nrays = nr;
      r.nsub = plan.nsub[s];
      r.vbase = T.v_elems;
      r.sbase = T.t_elems;
      r.dirs = plan.tables[s].dirs;
      r.pbounds = plan.tables[s].bounds;
      r.blk_begin = blk;
      r.pbegin = pairs;
      r.nseg = nseg;
      r.fbegin = fix;
      T.rec.push_back(r);
      blk += it.blocks;
      pairs += (nr + kPatch - 1) / kPatch;
      fix += nr * (nseg - 1);
      T.v_elems += int64_t(nr) * row_stride(plan.nsub[s]);
      T.t_elems += int64_t(nr) * nseg;
    }
    T.xcd_blocks[x] = blk;
  }
  T.xcd_src[X] = static_cast<int>(T.rec.size());
  T.n_pairs = pairs;
  T.fix_waves = fix;
  return T;
}

// Writes a group's table at table[first ..] in launches of kSrcPerWrite entries.
hipError_t write_group_table(const GroupTable& T, rtmi::SrcRec* table, float ds, hipStream_t st) {
  for (size_t i0 = 0; i0 < T.rec.size(); i0 += rtmi::kSrcPerWrite) {
    rtmi::SrcWrite w;
    std::memset(&w, 0, sizeof w);
    w.count = static_cast<int>(std::min<size_t>(rtmi::kSrcPerWrite, T.rec.size() - i0));
    for (int i = 0; i < w.count; ++i) w.rec[i] = T.rec[i0 + i];
    w.table = table;
    w.first = static_cast<int>(i0);
    w.ds = ds;
    const hipError_t e = rtmi::launch_write_sources(w, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// What the tiled path enqueues: kFull (schedules and records computed in line, the
// stateless calls), kSchedule and kFill (only the schedules, each into its own buffer,
// then only the records: plan creation, which sizes the records in between) and kReplay
// (everything but the schedules and records, which a plan keeps).
enum class TiledMode { kFull, kSchedule, kFill, kReplay };

// One (bin chunk, source chunk) launch of the tiled path.
struct LaunchArgs {
  rtmi::RecordArgs r;
  rtmi::TileArgs t;
  int32_t nb;
  int blocks;
  int fix_waves;
};

// A second stream of the device (default priority), forked from and joined to the
// caller's stream with events, for work that only depends on the geometry.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, done = nullptr;
  hipError_t open(hipStream_t from) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
      static std::mutex mu;
      static std::map<int, hipStream_t> streams;
      std::lock_guard<std::mutex> lock(mu);
      auto it = streams.find(dev);
      if (it == streams.end()) {
        hipStream_t s = nullptr;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return e;
        it = streams.emplace(dev, s).first;
      }
      stream = it->second;
    }
    if ((e = hipEventCreateWithFlags(&fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&done, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventRecord(fork, from)) != hipSuccess) return e;
    return hipStreamWaitEvent(stream, fork, 0);
  }
  // marks the end of the side work; the caller's stream waits on `done` where needed
  hipError_t join(hipStream_t) { return hipEventRecord(done, stream); }
  ~SideStream() {
    if (fork) (void)hipEventDestroy(fork);
    if (done) (void)hipEventDestroy(done);
  }
};

// Events that order the two streams launch by launch (destroyed with the list; HIP
// releases an event whose recorded work is still pending once that work completes).
struct EventList {
  std::vector<hipEvent_t> ev;
  hipError_t create(size_t n) {
    for (size_t i = 0; i < n; ++i) {
      hipEvent_t x = nullptr;
      const hipError_t e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
      if (e != hipSuccess) return e;
      ev.push_back(x);
    }
    return hipSuccess;
  }
  hipEvent_t operator[](size_t i) const { return ev[i]; }
  ~EventList() {
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
  }
};

int32_t run_tiled(const Problem& p, const Plan& plan, unsigned long long* out_q,
                  const double* det_scale, TiledMode mode = TiledMode::kFull,
                  char* given_ws = nullptr, const RecordSlices* slices = nullptr, bool use_side = true) {
  const hipStream_t st = p.stream;
  // a stateless call keeps its records in the workspace; a plan, in slices of its own
  const TiledLayout L = tiled_layout(p, plan, true, mode == TiledMode::kFull);
  if ((mode == TiledMode::kFill || mode == TiledMode::kReplay) && !slices)
    return fail(RTMI_ERR_INVALID_ARG, "a plan's chunk records are missing");
  unsigned long long* dropped = nullptr;
  if (mode == TiledMode::kFull)
    if (int32_t rc = dropped_counter(&dropped)) return rc;
  char* ws = given_ws;
  Scratch scratch;
  if (!ws) {
    if (mode != TiledMode::kFull) return fail(RTMI_ERR_INVALID_ARG, "a plan's workspace is missing");
    if (int32_t rc = acquire_scratch(L.total, st, kSlotTiled, &scratch)) return rc;
    ws = scratch.ptr;
  }
  float* corner = reinterpret_cast<float*>(ws + L.corner);
  unsigned long long* corner_q = reinterpret_cast<unsigned long long*>(ws + L.corner + kCornerBytes);
  float4* med = L.interleaved ? reinterpret_cast<float4*>(ws + L.med) : nullptr;
  float2* jk = L.jk_rows ? reinterpret_cast<float2*>(ws + L.med) : nullptr;
  float* V = reinterpret_cast<float*>(ws + L.v);
  float* Prow = reinterpret_cast<float*>(ws + L.p);
  float2* segtot = reinterpret_cast<float2*>(ws + L.segtot);
  hipError_t e;

  // the device source tables: one per source group, written in every mode that computes
  // schedules (a plan's replays reuse the ones written at its creation)
  rtmi::SrcRec* srcs = reinterpret_cast<rtmi::SrcRec*>(ws + L.srcs);
  std::vector<GroupTable> tables;
  for (size_t gi = 0; gi < L.groups.size(); ++gi) tables.push_back(group_table(p, plan, L.groups[gi], L.seg_len[gi]));
  if (mode == TiledMode::kFull || mode == TiledMode::kSchedule)
    for (size_t gi = 0; gi < L.groups.size(); ++gi)
      if ((e = write_group_table(tables[gi], srcs + L.groups[gi].s0, p.ds, st)) != hipSuccess)
        return hip_fail(e, "source table");

  std::vector<LaunchArgs> launches;
  int launch = 0;
  for (int32_t b0 = 0; b0 < p.n_bins; b0 += kMaxBinsPerLaunch) {
    const int32_t nb = std::min(kMaxBinsPerLaunch, p.n_bins - b0);
    for (size_t gi = 0; gi < L.groups.size(); ++gi, ++launch) {
      const GroupTable& T = tables[gi];
      const rtmi::SrcRec* gsrc = srcs + L.groups[gi].s0;
      rtmi::RecordArgs r;
      rtmi::TileArgs t;
      std::memset(&r, 0, sizeof r);
      std::memset(&t, 0, sizeof t);
      int blocks = 0;
      for (int x = 0; x < rtmi::kXcds; ++x) {
        r.xcd_src[x] = T.xcd_src[x];
        r.xcd_blocks[x] = T.xcd_blocks[x];
        blocks += T.xcd_blocks[x];
      }
      r.xcd_src[rtmi::kXcds] = T.xcd_src[rtmi::kXcds];
      r.src = t.src = gsrc;
      r.n_src = t.n_src = L.groups[gi].ns;
      t.n_pairs = T.n_pairs;
      const int seg_len = L.seg_len[gi];
      r.seg_len = seg_len;
      r.fix_waves = T.fix_waves;
      r.P = seg_len > 0 ? Prow : nullptr;
      r.segtot = seg_len > 0 ? segtot : nullptr;
      r.med = med;
      r.jk = jk;
      t.gj = p.j;
      t.gk = p.kap;
      t.jk = jk;
      t.jk_bytes = jk ? T.v_elems * int64_t(sizeof(float2)) : 0;
      r.j = p.j ? p.j + b0 * p.j_stride : nullptr;
      r.j_stride = p.j_stride;
      r.kap = p.kap ? p.kap + b0 * p.k_stride : nullptr;
      r.k_stride = p.k_stride;
      for (int32_t b = 0; b < nb; ++b) r.kscale[b] = p.kscale ? p.kscale[b0 + b] : 1.0f;
      r.V = V;
      t.V = V;
      r.v_bin_stride = t.v_bin_stride = T.v_elems;
      r.corner = corner;
      r.corner_q = corner_q;
      t.corner = corner;
      t.corner_q = corner_q;
      r.det_scale = t.det_scale = det_scale;
      r.nx = t.nx = p.nx;
      r.ny = t.ny = p.ny;
      r.nz = t.nz = p.nz;
      r.ds = t.ds = p.ds;
      t.out = p.out ? p.out + b0 * plan.cells : nullptr;
      t.out_q = out_q ? out_q + b0 * plan.cells : nullptr;
      t.out_stride = plan.cells;
      t.tiles_x = L.tiles_x;
      t.tiles_y = L.tiles_y;
      t.tiles_z = L.tiles_z;
      t.groups_per_cu = plan.tile_groups_per_cu;
      TileSchedule sched;
      sched.carve(ws + L.sched + launch * L.sched_bytes, L.tiles, L.pair_blocks);
      if (slices && launch < static_cast<int>(slices->off.size()))
        sched.apply(t, plan.item_chunks, slices->base + slices->off[launch], slices->count[launch]);
      else   // launches alternate between the shared buffers, sized by a bound
        sched.apply(t, plan.item_chunks,
                    reinterpret_cast<uint2*>(ws + L.recs + (launch % L.rec_buffers) *
                                                               align256(size_t(L.rec_capacity) * sizeof(uint2))),
                    L.rec_capacity, dropped);
      launches.push_back({r, t, nb, blocks, T.fix_waves});
    }
  }

  // The schedules and records depend on the geometry only. A stateless call computes them
  // on a side stream, overlapped with the gather table and the record passes. With one
  // launch, the first tile pass waits for all of it. Several launches alternate between
  // two record buffers: the side stream fills launch i + 2 once the tile pass of launch i
  // has read its buffer, while launches i + 1 and i + 2 record (per-launch events order
  // the two streams). Without a side stream, each fill runs just before its tile pass.
  hipStream_t sched_st = st;
  SideStream side;
  if (mode == TiledMode::kFull && use_side && side.open(st) == hipSuccess) sched_st = side.stream;
  if (mode == TiledMode::kFull || mode == TiledMode::kSchedule)
    for (const LaunchArgs& l : launches)
      if ((e = rtmi::launch_tile_schedule(l.t, L.tiles, sched_st)) != hipSuccess)
        return hip_fail(e, "tile schedule");
  const bool fill_each = mode == TiledMode::kFull && launches.size() > 1;
  const bool fill_ahead = fill_each && sched_st != st;
  if (mode == TiledMode::kFill || (mode == TiledMode::kFull && !fill_each))
    for (const LaunchArgs& l : launches)
      if ((e = rtmi::launch_tile_fill(l.t, L.tiles, sched_st)) != hipSuccess)
        return hip_fail(e, "tile records");
  if (mode == TiledMode::kSchedule || mode == TiledMode::kFill) return RTMI_OK;
  EventList filled, read;   // per launch: its records written / its tile pass done
  if (fill_ahead) {
    if ((e = filled.create(launches.size())) != hipSuccess || (e = read.create(launches.size())) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
    for (size_t i = 0; i < std::min<size_t>(2, launches.size()); ++i)
      if ((e = rtmi::launch_tile_fill(launches[i].t, L.tiles, sched_st)) != hipSuccess ||
          (e = hipEventRecord(filled[i], sched_st)) != hipSuccess)
        return hip_fail(e, "tile records");
  } else if (sched_st != st && (e = side.join(st)) != hipSuccess) {
    return hip_fail(e, "side stream");
  }

  if (L.interleaved) {
    TimedLaunch tl;
    if ((e = timed_begin(st, RTMI_KERNEL_TABLE, &tl, !plan.no_alloc)) != hipSuccess) return hip_fail(e, "timing");
    if ((e = rtmi::launch_cell_table(p.j, p.kap, med, p.nx, p.ny, p.nz, st)) != hipSuccess)
      return hip_fail(e, "gather table");
    if ((e = timed_end(st, tl)) != hipSuccess) return hip_fail(e, "timing");
  }
  {   // every tile launch adds into the zeroed field
    const int64_t total = plan.cells * p.n_bins;
    if (plan.det) e = rtmi::launch_fill_zero_u64(out_q, total, st);
    else e = rtmi::launch_fill_zero(p.out, total, st);
    if (e != hipSuccess) return hip_fail(e, "fill");
  }
  bool joined = sched_st == st || fill_ahead;
  // this launch's chunk records, written before its tile passes (and, with the gather
  // pass, before its record pass)
  auto records_ready = [&](size_t li) -> hipError_t {
    hipError_t err = hipSuccess;
    if (!joined) {
      if ((err = hipStreamWaitEvent(st, side.done, 0)) != hipSuccess) return err;
      joined = true;
    }
    if (fill_ahead) return hipStreamWaitEvent(st, filled[li], 0);
    if (fill_each) return rtmi::launch_tile_fill(launches[li].t, L.tiles, st);
    return err;
  };
  for (size_t li = 0; li < launches.size(); ++li) {
    const LaunchArgs& l = launches[li];
    if ((e = rtmi::launch_fill_zero(corner, 2 * kCornerBytes / sizeof(float), st)) != hipSuccess)
      return hip_fail(e, "fill");
    if (L.jk_rows) {
      if ((e = records_ready(li)) != hipSuccess) return hip_fail(e, "tile records");
      TimedLaunch tl;
      if ((e = timed_begin(st, RTMI_KERNEL_GATHER, &tl, !plan.no_alloc)) != hipSuccess) return hip_fail(e, "timing");
      if ((e = rtmi::launch_gather_pass(l.t, st)) != hipSuccess) return hip_fail(e, "gather pass");
      if ((e = timed_end(st, tl)) != hipSuccess) return hip_fail(e, "timing");
    }
    if (l.blocks > 0) {
      TimedLaunch tl;
      if ((e = timed_begin(st, RTMI_KERNEL_RECORD, &tl, !plan.no_alloc)) != hipSuccess) return hip_fail(e, "timing");
      if ((e = rtmi::launch_record(l.r, l.nb, p.j_stride == 0, plan.det, l.blocks, st)) != hipSuccess)
        return hip_fail(e, "record launch");
      if (l.fix_waves > 0 && (e = rtmi::launch_fixup(l.r, l.nb, plan.det, l.fix_waves, st)) != hipSuccess)
        return hip_fail(e, "record fixup launch");
      if ((e = timed_end(st, tl)) != hipSuccess) return hip_fail(e, "timing");
    }
    if (!L.jk_rows && (e = records_ready(li)) != hipSuccess) return hip_fail(e, "tile records");
    if (l.nb > 0) {   // one tile pass over every bin of the launch
      TimedLaunch tl;
      if ((e = timed_begin(st, RTMI_KERNEL_TILE, &tl, !plan.no_alloc)) != hipSuccess) return hip_fail(e, "timing");
      if ((e = rtmi::launch_tile_bins(l.t, l.nb, plan.det, false, st)) != hipSuccess) return hip_fail(e, "tile launch");
      if ((e = timed_end(st, tl)) != hipSuccess) return hip_fail(e, "timing");
    }
    if (fill_ahead && li + 2 < launches.size()) {   // launch li + 2 reuses this launch's buffer
      if ((e = hipEventRecord(read[li], st)) != hipSuccess ||
          (e = hipStreamWaitEvent(sched_st, read[li], 0)) != hipSuccess ||
          (e = rtmi::launch_tile_fill(launches[li + 2].t, L.tiles, sched_st)) != hipSuccess ||
          (e = hipEventRecord(filled[li + 2], sched_st)) != hipSuccess)
        return hip_fail(e, "tile records");
    }
  }
  if ((e = scratch.release(st)) != hipSuccess) return hip_fail(e, "workspace release");
  return RTMI_OK;
}

// ---- direct path: one kernel, register windows and global atomics ----
int32_t run_direct(const Problem& p, const Plan& plan, unsigned long long* out_q,
                   const double* det_scale) {
  const hipStream_t st = p.stream;
  hipError_t e;
  const int64_t total = plan.cells * p.n_bins;
  if (!plan.det && (e = rtmi::launch_fill_zero(p.out, total, st)) != hipSuccess) return hip_fail(e, "fill");
  for (int32_t b0 = 0; b0 < p.n_bins; b0 += kMaxBinsPerLaunch) {
    const int32_t nb = std::min(kMaxBinsPerLaunch, p.n_bins - b0);
    for (int32_t s0 = 0; s0 < p.n_src; s0 += kMaxSrcPerLaunch) {
      const int32_t ns = std::min(kMaxSrcPerLaunch, p.n_src - s0);
      rtmi::MarchArgs a;
      std::memset(&a, 0, sizeof a);
      a.j = p.j + b0 * p.j_stride;
      a.j_stride = p.j_stride;
      a.kap = p.kap + b0 * p.k_stride;
      a.k_stride = p.k_stride;
      for (int32_t b = 0; b < nb; ++b) a.kscale[b] = p.kscale ? p.kscale[b0 + b] : 1.0f;
      a.out = p.out + b0 * plan.cells;
      a.acc = out_q ? out_q + b0 * plan.cells : nullptr;
      a.det_scale = det_scale;
      a.out_stride = plan.cells;
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
        a.wray[i] = ray_weight(p, plan, s);
        a.nrays[i] = plan.nsub[s] > 0 ? p.nrays[s] : 0;
        a.nsub[i] = plan.nsub[s];
        a.dirs[i] = plan.tables[s].dirs;
        blocks += (a.nrays[i] + kBlock - 1) / kBlock;
      }
      a.blk_begin[ns] = blocks;
      if (blocks == 0) continue;
      TimedLaunch tl;
      if ((e = timed_begin(st, RTMI_KERNEL_DIRECT, &tl, !plan.no_alloc)) != hipSuccess) return hip_fail(e, "timing");
      if ((e = rtmi::launch_march(a, nb, p.j_stride == 0, plan.det, blocks, st)) != hipSuccess)
        return hip_fail(e, "march launch");
      if ((e = timed_end(st, tl)) != hipSuccess) return hip_fail(e, "timing");
    }
  }
  return RTMI_OK;
}

// no_alloc: the call takes every buffer from the static scratch (or fails before it
// enqueues anything), uses only direction tables prepared beforehand, and runs the tile
// geometry passes on the caller's stream (no side stream, no events).
int32_t run(const Problem& p, bool no_alloc = false) {
  Plan plan;
  if (int32_t st = validate(p, &plan)) return st;
  plan.no_alloc = no_alloc;
  const hipStream_t st = p.stream;
  hipError_t e;

  const int64_t total = plan.cells * p.n_bins;
  char* fixed_ws = nullptr;   // no_alloc: the tiled workspace, then the fixed-point field
  size_t fixed_off = 0;
  if (no_alloc) {
    if (plan.explicit_dirs)
      return fail(RTMI_ERR_UNSUPPORTED, "explicit directions are uploaded per call, which allocates; "
                  "this entry point takes the prepared Fibonacci tables only");
    if (plan.tiled) fixed_off = align256(tiled_layout(p, plan, true, true).total);
    const size_t need = fixed_off + (plan.det ? align256(size_t(total) * 8 + 16) : 0);
    if (need > kStaticScratchBytes)
      return fail(RTMI_ERR_RANGE, "the call needs %zu bytes of scratch, more than the %zu bytes of the "
                  "static scratch", need, kStaticScratchBytes);
    if (int32_t rc = static_scratch(&fixed_ws)) return rc;
  }

  // directions: cached Fibonacci tables, or this call's explicit table
  plan.tables.resize(p.n_src);
  char* explicit_table = nullptr;
  if (plan.explicit_dirs) {
    const int32_t n = p.nrays[0];
    std::vector<float> xyz(p.opts->directions, p.opts->directions + size_t(n) * 3);
    const HostTable t = build_table(xyz);
    if (int32_t rc = pool_alloc(reinterpret_cast<void**>(&explicit_table), table_bytes(t), st)) return rc;
    const size_t db = t.dirs.size() * sizeof(float4);
    e = hipMemcpyAsync(explicit_table, t.dirs.data(), db, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(explicit_table + db, t.bounds.data(), t.bounds.size() * sizeof(float),
                         hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(directions)");
    DevTable dt;
    dt.dirs = reinterpret_cast<float4*>(explicit_table);
    dt.bounds = reinterpret_cast<float*>(explicit_table + db);
    for (int32_t s = 0; s < p.n_src; ++s) plan.tables[s] = dt;
  } else {
    for (int32_t s = 0; s < p.n_src; ++s)
      if (int32_t rc = get_dirs(p.nrays[s], st, &plan.tables[s], !no_alloc)) return rc;
  }

  // deterministic mode: fixed-point field and its scale
  unsigned long long* out_q = nullptr;
  double* det_scale = nullptr;
  Scratch fixed;
  if (plan.det) {
    if (no_alloc) fixed.ptr = fixed_ws + fixed_off;
    else if (int32_t rc = acquire_scratch(size_t(total) * 8 + 16, st, kSlotFixedPoint, &fixed)) return rc;
    out_q = reinterpret_cast<unsigned long long*>(fixed.ptr);
    det_scale = reinterpret_cast<double*>(out_q + total);
    if (!plan.tiled && (e = rtmi::launch_fill_zero_u64(out_q, total, st)) != hipSuccess)
      return hip_fail(e, "fill");
    if ((e = det_scale_launch(p, plan, det_scale)) != hipSuccess) return hip_fail(e, "det_scale");
  }

  const int32_t rc = !plan.tiled ? run_direct(p, plan, out_q, det_scale)
                   : no_alloc ? run_tiled(p, plan, out_q, det_scale, TiledMode::kFull, fixed_ws, nullptr, false)
                              : run_tiled(p, plan, out_q, det_scale);
  if (rc != RTMI_OK) return rc;

  if (plan.det) {
    if ((e = rtmi::launch_det_convert(out_q, det_scale, p.out, total, st)) != hipSuccess)
      return hip_fail(e, "det_convert");
    if ((e = fixed.release(st)) != hipSuccess) return hip_fail(e, "workspace release");
  }
  if (explicit_table && (e = hipFreeAsync(explicit_table, st)) != hipSuccess)
    return hip_fail(e, "workspace release");
  g_error.clear();
  return RTMI_OK;
}

// ---- adjoint: checkpointed reverse sweep + tile deposits of dL/dj and dL/dkappa ----
// Bins are independent problems (Sec. 2, "Frequency-bin agnosticism"), so each bin's
// adjoint is the one-bin adjoint at (j_b, kappa_b), run bin after bin. A j or kappa shared
// by the bins collects every bin's gradient in one output (the tile passes add into it);
// with kappa_b = s_b kappa, a bin's dL/dkappa deposits are multiplied by s_b, and
// dL/ds_b = sum over samples of kappa(nearest voxel) x the sample's dL/dkappa_b.
int32_t run_vjp(const Problem& p, const float* grad, float* grad_j, float* grad_k, float* grad_scale) {
  Plan plan;
  if (int32_t st = validate(p, &plan)) return st;
  if (!grad || !grad_j || !grad_k) return fail(RTMI_ERR_INVALID_ARG, "null gradient pointer");
  if (grad_scale && p.k_stride != 0)
    return fail(RTMI_ERR_INVALID_ARG, "grad_kappa_scale needs a kappa shared by the bins (kappa_bin_stride 0)");
  if (plan.det || !plan.tiled || plan.explicit_dirs)
    return fail(RTMI_ERR_UNSUPPORTED, "the adjoint runs the float tiled path with the Fibonacci directions");
  const hipStream_t st = p.stream;
  plan.tables.resize(p.n_src);
  for (int32_t s = 0; s < p.n_src; ++s)
    if (int32_t rc = get_dirs(p.nrays[s], st, &plan.tables[s])) return rc;

  int64_t v_elems_max = 0, c_elems_max = 0;
  for (int32_t s0 = 0; s0 < p.n_src; s0 += kMaxSrcPerLaunch) {
    int64_t e = 0, c = 0;
    for (int32_t s = s0; s < std::min(p.n_src, s0 + kMaxSrcPerLaunch); ++s) {
      if (plan.nsub[s] == 0) continue;
      e += int64_t(p.nrays[s]) * row_stride(plan.nsub[s]);
      c += int64_t(p.nrays[s]) * ((plan.nsub[s] + rtmi::kSeg - 1) / rtmi::kSeg);
    }
    v_elems_max = std::max(v_elems_max, e);
    c_elems_max = std::max(c_elems_max, c);
  }
  const size_t corner_bytes = 256;
  const size_t med_bytes = align256(size_t(plan.cells) * 4 * sizeof(float4));
  const size_t v_bytes = (size_t(v_elems_max) * sizeof(float) + 255) / 256 * 256;
  const size_t c_bytes = size_t(c_elems_max) * sizeof(float2);
  const int tiles_x = (p.nx + kTile - 1) / kTile, tiles_y = (p.ny + kTile - 1) / kTile,
            tiles_z = (p.nz + kTile - 1) / kTile;
  const int tiles = tiles_x * tiles_y * tiles_z;
  int64_t rec_capacity = 0;
  int max_blocks = 0;
  for (int32_t s0 = 0; s0 < p.n_src; s0 += kMaxSrcPerLaunch) {
    rec_capacity = std::max(rec_capacity, record_bound(p, plan, s0, std::min(kMaxSrcPerLaunch, p.n_src - s0),
                                                       tiles_x, tiles_y, tiles_z));
    max_blocks = std::max(max_blocks, pair_blocks(p, plan, s0, std::min(kMaxSrcPerLaunch, p.n_src - s0)));
  }
  const size_t sched_bytes = TileSchedule::bytes(tiles, max_blocks);
  const size_t srcs_bytes = align256(size_t(kMaxSrcPerLaunch) * sizeof(rtmi::SrcRec));
  const size_t dscale_bytes = align256(size_t(p.n_bins) * sizeof(double));
  const size_t rec_off = corner_bytes + med_bytes + 2 * v_bytes + align256(c_bytes) + sched_bytes + srcs_bytes +
                         dscale_bytes;
  unsigned long long* dropped = nullptr;
  if (int32_t rc = dropped_counter(&dropped)) return rc;
  Scratch scratch;
  if (int32_t rc = acquire_scratch(rec_off + size_t(rec_capacity) * sizeof(uint2), st, kSlotAdjoint, &scratch))
    return rc;
  char* ws = scratch.ptr;
  TileSchedule sched;
  sched.carve(ws + corner_bytes + med_bytes + 2 * v_bytes + align256(c_bytes), tiles, max_blocks);
  uint2* recs = reinterpret_cast<uint2*>(ws + rec_off);
  rtmi::SrcRec* srcs = reinterpret_cast<rtmi::SrcRec*>(ws + rec_off - dscale_bytes - srcs_bytes);
  double* dscale = reinterpret_cast<double*>(ws + rec_off - dscale_bytes);
  float* corner = reinterpret_cast<float*>(ws);  // [0..7] for dL/dj, [8..15] for dL/dkappa
  float4* med = reinterpret_cast<float4*>(ws + corner_bytes);
  float* Vj = reinterpret_cast<float*>(ws + corner_bytes + med_bytes);
  float* Vk = reinterpret_cast<float*>(ws + corner_bytes + med_bytes + v_bytes);
  float2* ckpt = reinterpret_cast<float2*>(ws + corner_bytes + med_bytes + 2 * v_bytes);
  hipError_t e;
  // every bin's deposits add into these, zeroed once
  if ((e = rtmi::launch_fill_zero(grad_j, plan.cells * (p.j_stride ? p.n_bins : 1), st)) != hipSuccess ||
      (e = rtmi::launch_fill_zero(grad_k, plan.cells * (p.k_stride ? p.n_bins : 1), st)) != hipSuccess ||
      (grad_scale && (e = rtmi::launch_fill_zero_u64(reinterpret_cast<unsigned long long*>(dscale), p.n_bins, st)) !=
                         hipSuccess))
    return hip_fail(e, "fill");

  for (int32_t b = 0; b < p.n_bins; ++b) {
    const float s_b = (p.k_stride == 0 && p.kscale) ? p.kscale[b] : 1.0f;
    if ((e = rtmi::launch_cell_table(p.j + b * p.j_stride, p.kap + b * p.k_stride, med, p.nx, p.ny, p.nz, st)) !=
        hipSuccess)
      return hip_fail(e, "gather table");
    for (int32_t s0 = 0; s0 < p.n_src; s0 += kMaxSrcPerLaunch) {
      const int32_t ns = std::min(kMaxSrcPerLaunch, p.n_src - s0);
      rtmi::AdjointArgs r;
      rtmi::TileArgs t;
      std::memset(&r, 0, sizeof r);
      std::memset(&t, 0, sizeof t);
      int64_t v_elems = 0, c_elems = 0;
      int blocks = 0, patches = 0;
      GroupTable T;   // the tile passes' source table, in launch order
      for (int32_t i = 0; i < ns; ++i) {
        const int32_t s = s0 + i;
        const int32_t nr = plan.nsub[s] > 0 ? p.nrays[s] : 0;
        r.blk_begin[i] = blocks;
        r.sx[i] = p.src[3 * s];
        r.sy[i] = p.src[3 * s + 1];
        r.sz[i] = p.src[3 * s + 2];
        r.wray[i] = ray_weight(p, plan, s);
        r.nrays[i] = nr;
        r.nsub[i] = plan.nsub[s];
        r.vbase[i] = v_elems;
        r.cstride[i] = (plan.nsub[s] + rtmi::kSeg - 1) / rtmi::kSeg;
        r.cbase[i] = c_elems;
        r.dirs[i] = plan.tables[s].dirs;
        rtmi::SrcRec q;
        std::memset(&q, 0, sizeof q);
        q.sx = r.sx[i];
        q.sy = r.sy[i];
        q.sz = r.sz[i];
        q.wray = r.wray[i];
        q.nrays = nr;
        q.nsub = plan.nsub[s];
        q.vbase = v_elems;
        q.dirs = plan.tables[s].dirs;
        q.pbounds = plan.tables[s].bounds;
        q.pbegin = patches;
        q.nseg = 1;
        T.rec.push_back(q);
        v_elems += int64_t(nr) * row_stride(plan.nsub[s]);
        c_elems += int64_t(nr) * r.cstride[i];
        blocks += (nr + kBlock - 1) / kBlock;
        patches += (nr + kPatch - 1) / kPatch;
      }
      r.blk_begin[ns] = blocks;
      if ((e = write_group_table(T, srcs, p.ds, st)) != hipSuccess) return hip_fail(e, "source table");
      t.src = srcs;
      t.n_pairs = patches;
      r.med = med;
      r.grad = grad + b * plan.cells;
      r.Vj = Vj;
      r.Vk = Vk;
      r.ckpt = ckpt;
      r.corner_j = corner;
      r.corner_k = corner + 8;
      r.kscale = s_b;
      r.kgrad_scale = s_b;
      r.dscale = grad_scale ? dscale + b : nullptr;
      r.nx = t.nx = p.nx;
      r.ny = t.ny = p.ny;
      r.nz = t.nz = p.nz;
      r.ds = t.ds = p.ds;
      r.n_src = t.n_src = ns;
      t.v_bin_stride = v_elems;
      t.out_stride = plan.cells;
      t.tiles_x = tiles_x;
      t.tiles_y = tiles_y;
      t.tiles_z = tiles_z;
      sched.apply(t, 0, recs, rec_capacity, dropped);
      if ((e = rtmi::launch_fill_zero(corner, 64, st)) != hipSuccess) return hip_fail(e, "fill");
      if (blocks > 0 && (e = rtmi::launch_adjoint_record(r, blocks, st)) != hipSuccess)
        return hip_fail(e, "adjoint launch");
      t.V = Vj;
      t.corner = corner;
      t.out = grad_j + b * (p.j_stride ? plan.cells : 0);
      // one schedule and one set of records serve both deposits (same rays, same tiles)
      if ((e = rtmi::launch_tile_schedule(t, tiles, st)) != hipSuccess ||
          (e = rtmi::launch_tile_fill(t, tiles, st)) != hipSuccess ||
          (e = rtmi::launch_tile_run(t, 1, false, false, st)) != hipSuccess)
        return hip_fail(e, "tile launch");
      t.V = Vk;
      t.corner = corner + 8;
      t.out = grad_k + b * (p.k_stride ? plan.cells : 0);
      if ((e = rtmi::launch_tile_run(t, 1, false, true, st)) != hipSuccess) return hip_fail(e, "tile launch");
    }
  }
  if (grad_scale && (e = rtmi::launch_f64_to_f32(dscale, grad_scale, p.n_bins, st)) != hipSuccess)
    return hip_fail(e, "scale gradient");
  if ((e = scratch.release(st)) != hipSuccess) return hip_fail(e, "workspace release");
  g_error.clear();
  return RTMI_OK;
}

// ---- plans ----

}  // namespace

// A validated problem with its direction tables, workspace and tile schedules, executed
// any number of times on new maps. Owns everything it points to except the maps and field.
struct rtmi_plan {
  int device = 0;
  std::vector<float> src, kscale;
  std::vector<int32_t> nrays, caps;
  rtmi_options opts{};
  Problem p{};
  Plan plan;
  char* ws = nullptr;          // hipMalloc'd
  size_t ws_bytes = 0;
  RecordSlices recs;          // chunk records of every launch; recs.base hipMalloc'd
  char* table = nullptr;       // explicit direction table, hipMalloc'd
  unsigned long long* out_q = nullptr;
  double* det_scale = nullptr;
};

namespace {

void plan_release(rtmi_plan* P) {
  if (!P) return;
  int cur = 0;
  const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != P->device;
  if (switch_dev) (void)hipSetDevice(P->device);
  if (P->ws) (void)hipFree(P->ws);
  if (P->recs.base) (void)hipFree(P->recs.base);
  if (P->table) (void)hipFree(P->table);
  if (switch_dev) (void)hipSetDevice(cur);
  delete P;
}

int32_t plan_create(const Problem& given, rtmi_plan** out) {
  std::unique_ptr<rtmi_plan, void (*)(rtmi_plan*)> P(new rtmi_plan, plan_release);
  if (hipGetDevice(&P->device) != hipSuccess) return fail(RTMI_ERR_HIP, "no current HIP device");
  Problem p = given;
  if (int32_t st = validate(p, &P->plan, false)) return st;
  if (!P->plan.tiled) return fail(RTMI_ERR_UNSUPPORTED, "plans run the tiled path only");
  // own copies of the host arrays
  P->src.assign(p.src, p.src + size_t(p.n_src) * 3);
  P->nrays.assign(p.nrays, p.nrays + p.n_src);
  if (p.caps) P->caps.assign(p.caps, p.caps + p.n_src);
  if (p.kscale) P->kscale.assign(p.kscale, p.kscale + p.n_bins);
  if (p.opts) {
    P->opts = *p.opts;
    P->opts.directions = nullptr;   // uploaded below; the caller's array is not kept
  }
  p.src = P->src.data();
  p.nrays = P->nrays.data();
  p.caps = p.caps ? P->caps.data() : nullptr;
  p.kscale = p.kscale ? P->kscale.data() : nullptr;
  const rtmi_options* user_opts = p.opts;
  p.opts = p.opts ? &P->opts : nullptr;
  p.j = nullptr;
  p.kap = nullptr;
  p.out = nullptr;

  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{st};
  p.stream = st;

  // direction tables
  P->plan.tables.resize(p.n_src);
  if (P->plan.explicit_dirs) {
    const int32_t n = p.nrays[0];
    std::vector<float> xyz(user_opts->directions, user_opts->directions + size_t(n) * 3);
    const HostTable t = build_table(xyz);
    if ((e = hipMalloc(reinterpret_cast<void**>(&P->table), table_bytes(t))) != hipSuccess)
      return hip_fail(e, "hipMalloc(directions)");
    const size_t db = t.dirs.size() * sizeof(float4);
    if ((e = hipMemcpy(P->table, t.dirs.data(), db, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(P->table + db, t.bounds.data(), t.bounds.size() * sizeof(float),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "hipMemcpy(directions)");
    DevTable dt;
    dt.dirs = reinterpret_cast<float4*>(P->table);
    dt.bounds = reinterpret_cast<float*>(P->table + db);
    for (int32_t s = 0; s < p.n_src; ++s) P->plan.tables[s] = dt;
  } else {
    for (int32_t s = 0; s < p.n_src; ++s)
      if (int32_t rc = get_dirs(p.nrays[s], st, &P->plan.tables[s])) return rc;
  }

  // workspace: the tiled layout with one schedule per launch, then the fixed-point field;
  // the chunk records get their own allocation once the schedules have counted them
  const TiledLayout L = tiled_layout(p, P->plan, true, false);
  const int64_t total = P->plan.cells * p.n_bins;
  const size_t det_off = align256(L.total);
  P->ws_bytes = P->plan.det ? det_off + size_t(total) * 8 + 16 : L.total;
  if ((e = hipMalloc(reinterpret_cast<void**>(&P->ws), P->ws_bytes)) != hipSuccess)
    return hip_fail(e, "hipMalloc(plan workspace)");
  if (P->plan.det) {
    P->out_q = reinterpret_cast<unsigned long long*>(P->ws + det_off);
    P->det_scale = reinterpret_cast<double*>(P->out_q + total);
  }
  if (int32_t rc = run_tiled(p, P->plan, P->out_q, P->det_scale, TiledMode::kSchedule, P->ws)) return rc;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "plan schedule");
  int64_t rec_sum = 0;
  for (int i = 0; i < L.n_launch; ++i) {
    TileSchedule sched;
    sched.carve(P->ws + L.sched + size_t(i) * L.sched_bytes, L.tiles, L.pair_blocks);
    long long n = 0;
    if ((e = hipMemcpy(&n, sched.rec_total(), sizeof n, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "plan record count");
    P->recs.off.push_back(rec_sum);
    P->recs.count.push_back(n);
    rec_sum += n;
  }
  if ((e = hipMalloc(reinterpret_cast<void**>(&P->recs.base), std::max<size_t>(size_t(rec_sum) * sizeof(uint2), 256))) !=
      hipSuccess)
    return hip_fail(e, "hipMalloc(plan records)");
  P->ws_bytes += size_t(rec_sum) * sizeof(uint2);
  if (int32_t rc = run_tiled(p, P->plan, P->out_q, P->det_scale, TiledMode::kFill, P->ws, &P->recs)) return rc;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "plan records");
  p.stream = nullptr;
  P->p = p;
  *out = P.release();
  g_error.clear();
  return RTMI_OK;
}

int32_t plan_execute(const rtmi_plan* P, const float* j, const float* kap, float* out, hipStream_t st) {
  if (!P) return fail(RTMI_ERR_INVALID_ARG, "null plan");
  if (!j || !kap || !out) return fail(RTMI_ERR_INVALID_ARG, "null map or field pointer");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != P->device)
    return fail(RTMI_ERR_INVALID_ARG, "the plan belongs to device %d, the current device is %d", P->device, cur);
  Problem p = P->p;
  p.j = j;
  p.kap = kap;
  p.out = out;
  p.stream = st;
  hipError_t e;
  const int64_t total = P->plan.cells * p.n_bins;
  if (P->plan.det) {
    if ((e = det_scale_launch(p, P->plan, P->det_scale)) != hipSuccess) return hip_fail(e, "det_scale");
  }
  if (int32_t rc = run_tiled(p, P->plan, P->out_q, P->det_scale, TiledMode::kReplay, P->ws, &P->recs)) return rc;
  if (P->plan.det && (e = rtmi::launch_det_convert(P->out_q, P->det_scale, p.out, total, st)) != hipSuccess)
    return hip_fail(e, "det_convert");
  g_error.clear();
  return RTMI_OK;
}

}  // namespace

extern "C" {

const char* rtmi_last_error(void) { return g_error.c_str(); }

int32_t rtmi_version(void) { return 320; }

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
  DevTable d;
  return get_dirs(num_rays, nullptr, &d);
}

int32_t rtmi_reserve(int64_t bytes) {
  if (bytes < 0) return fail(RTMI_ERR_INVALID_ARG, "bytes must be >= 0");
  void* p = nullptr;
  if (int32_t rc = pool_alloc(&p, static_cast<size_t>(bytes), nullptr)) return rc;
  hipError_t e = hipFreeAsync(p, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return hip_fail(e, "rtmi_reserve");
  return RTMI_OK;
}

int32_t rtmi_dropped_records(int64_t* count) {
  if (!count) return fail(RTMI_ERR_INVALID_ARG, "null count pointer");
  unsigned long long* d = nullptr;
  if (int32_t rc = dropped_counter(&d)) return rc;
  hipError_t e = hipDeviceSynchronize();
  unsigned long long n = 0;
  if (e == hipSuccess) e = hipMemcpy(&n, d, sizeof n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n != 0) e = hipMemset(d, 0, sizeof n);
  if (e != hipSuccess) return hip_fail(e, "rtmi_dropped_records");
  *count = static_cast<int64_t>(n);
  if (n != 0)
    return fail(RTMI_ERR_RANGE, "%llu chunk records did not fit their buffers: those deposits are missing "
                "from the fields of the calls since the last query", n);
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_release_workspaces(void) {
  int dev = 0;
  if (int32_t st = current_device(&dev)) return st;
  hipError_t e = hipDeviceSynchronize();   // every call that used the blocks has finished
  if (e != hipSuccess) return hip_fail(e, "rtmi_release_workspaces");
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    for (auto it = g_scratch.begin(); it != g_scratch.end();) {
      if (std::get<0>(it->first) != dev) {
        ++it;
        continue;
      }
      // (the caller's stream may no longer exist: free on the null stream, now idle)
      if (it->second.first && (e = hipFreeAsync(it->second.first, nullptr)) != hipSuccess)
        return hip_fail(e, "rtmi_release_workspaces");
      it = g_scratch.erase(it);
    }
  }
  if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e, "rtmi_release_workspaces");
  g_error.clear();
  return RTMI_OK;
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

int32_t rtmi_trace_bins_static(const float* j_maps, int64_t j_bin_stride, const float* kappa_maps,
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
  return run(p, true);
}

int64_t rtmi_static_scratch_bytes(void) { return static_cast<int64_t>(kStaticScratchBytes); }

int32_t rtmi_trace_vjp(const float* j_map, const float* kappa_map, int32_t nx, int32_t ny,
                       int32_t nz, int32_t n_src, const float* source_pos,
                       const int32_t* num_rays, const int32_t* substep_cap, float step_size,
                       float radiation_velocity, float time_step, const float* grad_field,
                       float* grad_j, float* grad_kappa, void* stream) {
  const Problem p{j_map, 0, kappa_map, 0, nullptr, 1, nx, ny, nz, n_src, source_pos, num_rays,
                  substep_cap, step_size, radiation_velocity, time_step, grad_j, nullptr,
                  static_cast<hipStream_t>(stream)};
  return run_vjp(p, grad_field, grad_j, grad_kappa, nullptr);
}

int32_t rtmi_trace_bins_vjp(const float* j_maps, int64_t j_bin_stride, const float* kappa_maps,
                            int64_t kappa_bin_stride, const float* kappa_scale, int32_t n_bins, int32_t nx,
                            int32_t ny, int32_t nz, int32_t n_src, const float* source_pos,
                            const int32_t* num_rays, const int32_t* substep_cap, float step_size,
                            float radiation_velocity, float time_step, const float* grad_fields,
                            float* grad_j, float* grad_kappa, float* grad_kappa_scale, void* stream) {
  const Problem p{j_maps, j_bin_stride, kappa_maps, kappa_bin_stride,
                  kappa_bin_stride ? nullptr : kappa_scale, n_bins, nx, ny, nz, n_src,
                  source_pos, num_rays, substep_cap, step_size, radiation_velocity, time_step,
                  grad_j, nullptr, static_cast<hipStream_t>(stream)};
  return run_vjp(p, grad_fields, grad_j, grad_kappa, grad_kappa_scale);
}

int32_t rtmi_dot(const float* a, const float* b, int64_t count, float* out, void* stream) {
  if (!a || !b || !out) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (count < 1) return fail(RTMI_ERR_INVALID_ARG, "count must be >= 1");
  const hipError_t e = rtmi::launch_dot(a, b, count, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rtmi_dot");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_scaled_copy(const float* in, const float* scale, float* out, int64_t count, void* stream) {
  if (!in || !scale || !out) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (count < 1) return fail(RTMI_ERR_INVALID_ARG, "count must be >= 1");
  const hipError_t e = rtmi::launch_scaled_copy(in, scale, out, count, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rtmi_scaled_copy");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_field_mse(const float* field, const float* target, int64_t count, float scale,
                       float* grad, float* loss, void* stream) {
  if (!field || !target || !grad || !loss) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (count < 1) return fail(RTMI_ERR_INVALID_ARG, "count must be >= 1");
  if (!std::isfinite(scale)) return fail(RTMI_ERR_NONFINITE, "scale is not finite");
  const hipError_t e = rtmi::launch_field_mse(field, target, count, scale, grad, loss,
                                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "field_mse launch");
  g_error.clear();
  return RTMI_OK;
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
  DevTable t;
  if (int32_t st = get_dirs(num_rays, s, &t)) return st;
  a.dirs = t.dirs;
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

int32_t rtmi_plan_create(int32_t nx, int32_t ny, int32_t nz, int32_t n_src, const float* source_pos,
                         const int32_t* num_rays, const int32_t* substep_cap, int32_t n_bins,
                         int64_t j_bin_stride, int64_t kappa_bin_stride, const float* kappa_scale,
                         float step_size, float radiation_velocity, float time_step,
                         const rtmi_options* opts, rtmi_plan** plan) {
  if (!plan) return fail(RTMI_ERR_INVALID_ARG, "null plan pointer");
  *plan = nullptr;
  const Problem p{nullptr, j_bin_stride, nullptr, kappa_bin_stride,
                  kappa_bin_stride ? nullptr : kappa_scale, n_bins, nx, ny, nz, n_src, source_pos,
                  num_rays, substep_cap, step_size, radiation_velocity, time_step, nullptr, opts,
                  nullptr};
  return plan_create(p, plan);
}

int32_t rtmi_plan_execute(const rtmi_plan* plan, const float* j_maps, const float* kappa_maps,
                          float* out_fields, void* stream) {
  return plan_execute(plan, j_maps, kappa_maps, out_fields, static_cast<hipStream_t>(stream));
}

int64_t rtmi_plan_workspace_bytes(const rtmi_plan* plan) {
  if (!plan) return fail(RTMI_ERR_INVALID_ARG, "null plan");
  return static_cast<int64_t>(plan->ws_bytes);
}

int32_t rtmi_plan_destroy(rtmi_plan* plan) {
  plan_release(plan);
  return RTMI_OK;
}

// ---- surrogate network ----

int32_t rtmi_conv3d_forward(const void* x, const void* w, const float* bias, const void* residual,
                            int32_t gelu, int32_t n, int32_t d, int32_t h, int32_t w_dim, void* y,
                            float* z, void* stream) {
  if (!x || !w || !y) return fail(RTMI_ERR_INVALID_ARG, "null x, w or y pointer");
  if (int32_t st = check_conv_shape(n, d, h, w_dim)) return st;
  rtmi::ConvArgs a;
  std::memset(&a, 0, sizeof a);
  a.x = x;
  a.w = w;
  a.bias = bias;
  a.residual = residual;
  a.gelu = gelu != 0;
  a.z = z;
  a.y = y;
  a.n = n;
  a.d = d;
  a.h = h;
  a.w_dim = w_dim;
  const hipError_t e = rtmi::launch_conv(a, false, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "conv forward launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_conv3d_backward_data(const void* dz, const void* w, const float* residual,
                                  const float* zprev, int32_t n, int32_t d, int32_t h,
                                  int32_t w_dim, float* dh, void* dz_prev, void* stream) {
  if (!dz || !w) return fail(RTMI_ERR_INVALID_ARG, "null dz or w pointer");
  if (!dh && !dz_prev) return fail(RTMI_ERR_INVALID_ARG, "neither dh nor dz_prev requested");
  if (int32_t st = check_conv_shape(n, d, h, w_dim)) return st;
  rtmi::ConvArgs a;
  std::memset(&a, 0, sizeof a);
  a.x = dz;
  a.w = w;
  a.residual_f32 = residual;
  a.zprev = zprev;
  a.dh = dh;
  a.y = dz_prev;
  a.n = n;
  a.d = d;
  a.h = h;
  a.w_dim = w_dim;
  const hipError_t e = rtmi::launch_conv(a, true, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "conv backward-data launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_conv3d_backward_weight(const void* x, const void* dz, int32_t n, int32_t d, int32_t h,
                                    int32_t w_dim, float* dw, float* db, void* stream) {
  if (!x || !dz || !dw || !db) return fail(RTMI_ERR_INVALID_ARG, "null x, dz, dw or db pointer");
  if (int32_t st = check_conv_shape(n, d, h, w_dim)) return st;
  if (w_dim % 16 != 0)
    return fail(RTMI_ERR_UNSUPPORTED, "backward-weight needs an x extent that is a multiple of 16 (got %d)", w_dim);
  rtmi::ConvArgs a;
  std::memset(&a, 0, sizeof a);
  a.x = x;
  a.dz = dz;
  a.dw = dw;
  a.db = db;
  a.n = n;
  a.d = d;
  a.h = h;
  a.w_dim = w_dim;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch held;   // the work-groups' partial sums
  if (int32_t rc = acquire_scratch(rtmi::wgrad_scratch_bytes(a), st, kSlotConv, &held)) return rc;
  hipError_t e = rtmi::launch_wgrad(a, reinterpret_cast<float*>(held.ptr), st);
  if (e != hipSuccess) return hip_fail(e, "conv backward-weight launch");
  if ((e = held.release(st)) != hipSuccess) return hip_fail(e, "workspace release");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_mse_loss(const void* y, const float* target, int64_t n_voxels, float scale, void* dz,
                      float* loss, void* stream) {
  if (!y || !target || !dz || !loss) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (n_voxels < 1) return fail(RTMI_ERR_INVALID_ARG, "n_voxels must be >= 1");
  if (!std::isfinite(scale)) return fail(RTMI_ERR_NONFINITE, "scale is not finite");
  const hipError_t e = rtmi::launch_mse(static_cast<const unsigned short*>(y), target, n_voxels, scale,
                                        static_cast<unsigned short*>(dz), loss, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "mse launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_surrogate_features(const float* j, const float* kappa, const float* cheap,
                                int64_t cells, const float* stats, float* scale_sums, void* x,
                                void* stream) {
  if (!j || !kappa || !cheap || !stats || !scale_sums || !x) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (cells < 1) return fail(RTMI_ERR_INVALID_ARG, "cells must be >= 1");
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(stats[i])) return fail(RTMI_ERR_NONFINITE, "stats[%d] is not finite", i);
  if (!(stats[5] > 0.0f)) return fail(RTMI_ERR_INVALID_ARG, "stats[5] (floor) must be > 0");
  const rtmi::SurrogateStats st{stats[0], stats[1], stats[2], stats[3], stats[4], stats[5]};
  const hipError_t e = rtmi::launch_features(j, kappa, cheap, cells, st, scale_sums,
                                             static_cast<unsigned short*>(x), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "features launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_surrogate_output(const void* y, const float* cheap, int64_t cells, const float* scale_sums,
                              float* field, float* check_sums, void* stream) {
  if (!y || !cheap || !scale_sums || !field || !check_sums) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (cells < 1) return fail(RTMI_ERR_INVALID_ARG, "cells must be >= 1");
  const hipError_t e = rtmi::launch_surrogate_output(static_cast<const unsigned short*>(y), cheap, cells,
                                                     scale_sums, field, check_sums,
                                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "surrogate output launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_adam_step(float* w, float* m, float* v, const float* g, void* w_bf16, int64_t count,
                       float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!w || !m || !v || !g) return fail(RTMI_ERR_INVALID_ARG, "null pointer");
  if (count < 1 || step < 1) return fail(RTMI_ERR_INVALID_ARG, "count and step must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f && std::isfinite(lr)))
    return fail(RTMI_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  const float c1 = static_cast<float>(1.0 - std::pow(double(beta1), step));
  const float c2 = static_cast<float>(1.0 - std::pow(double(beta2), step));
  const hipError_t e = rtmi::launch_adam(w, m, v, g, static_cast<unsigned short*>(w_bf16), count, lr, beta1,
                                         beta2, eps, c1, c2, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  g_error.clear();
  return RTMI_OK;
}

int32_t rtmi_timing_enable(int32_t on) {
  std::lock_guard<std::mutex> lock(g_tmu);
  g_timing = on != 0;
  for (auto& v : g_pending) {
    for (auto& ev : v) g_free.push_back(ev);
    v.clear();
  }
  return RTMI_OK;
}

int32_t rtmi_timing_read(int32_t kind, double* total_ms, int64_t* launches) {
  if (!total_ms || !launches) return fail(RTMI_ERR_INVALID_ARG, "null output pointer");
  if (kind < 0 || kind > 4) return fail(RTMI_ERR_INVALID_ARG, "unknown kernel kind %d", kind);
  std::lock_guard<std::mutex> lock(g_tmu);
  double sum = 0.0;
  for (auto& ev : g_pending[kind]) {
    hipError_t e = hipEventSynchronize(ev.second);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
    if (e != hipSuccess) return hip_fail(e, "reading timing events");
    sum += ms;
  }
  *total_ms = sum;
  *launches = static_cast<int64_t>(g_pending[kind].size());
  for (auto& ev : g_pending[kind]) g_free.push_back(ev);
  g_pending[kind].clear();
  return RTMI_OK;
}

}  // extern "C"
