// C ABI of the Wallace normal generator: validation, device memory, work
// lists and launches.  Declared in include/wn.h.
//
// Nothing here computes normals: every step of generation runs in the kernels
// of wn_device.hpp.  The host computes only the per-pool-size chi-square
// constants (Section 5.5) with plain IEEE arithmetic, once per generator.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstddef>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wn.h"
#include "wn_internal.hpp"

namespace {

// the calling thread's last message (a fixed buffer: reporting an error
// allocates nothing)
thread_local char g_last_error[512];

wn_status fail(wn_status st, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

// A failed runtime call is reported through the status; hipGetLastError is
// read here so that the failure is not reported again by a later launch.
wn_status hip_fail(hipError_t e, const char *what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? WN_ENOMEM : WN_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

wn_status hip_fail(hipError_t e, const char *who, const char *what) {
  (void)hipGetLastError();
  return fail(e == hipErrorOutOfMemory ? WN_ENOMEM : WN_EDEVICE, "%s: %s: %s", who, what,
              hipGetErrorString(e));
}

bool is_pow2(uint32_t v) { return v && !(v & (v - 1)); }

uint32_t ilog2(uint32_t v) {
  uint32_t r = 0;
  while ((1u << r) < v) ++r;
  return r;
}

// Chi-square constants for nu = n (Section 5.5).  A is the small root of
// A^3 - 3 nu A + 2 nu = 0, by eight Newton steps from 2/3 in the order
// A <- A - (((A*A)*A - (3 nu)*A) + 2 nu) / (3*(A*A) - 3 nu); b = sqrt(2(nu - A*A)).
wn::Chi2Consts chi2_consts(uint32_t n) {
  wn::Chi2Consts c;
  c.nu = double(n);
  double A = 2.0 / 3.0;
  for (int it = 0; it < 8; ++it) {
    const double num = ((A * A) * A - (3.0 * c.nu) * A) + 2.0 * c.nu;
    const double den = 3.0 * (A * A) - 3.0 * c.nu;
    A = A - num / den;
  }
  c.A = A;
  c.b = std::sqrt(2.0 * (c.nu - c.A * c.A));
  c.fisher_root = std::sqrt(2.0 * c.nu - 1.0);
  const double w = 2.0 / (9.0 * c.nu);
  c.wh_c = std::sqrt(w);
  c.wh_shift = 1.0 - w;
  return c;
}

// Extreme-value threshold of the fused statistics for pools of n values
// (Section 5.7: a value expected about once in ten pools): the smallest
// multiple of 2^-8 at which the two-sided normal tail erfc(c / sqrt 2) falls
// to 0.1 / n or below.
double extreme_threshold(uint32_t n) {
  const double target = 0.1 / double(n);
  uint32_t j = 0;
  while (std::erfc(double(j) / (256.0 * std::sqrt(2.0))) > target) ++j;
  return double(j) / 256.0;
}

// A pinned staging buffer and its device twin for one work list.  A slot is
// reused only after the event recorded behind its last use has completed.
struct ListSlot {
  wn::WorkItem *host = nullptr;
  wn::WorkItem *dev = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

// Staging buffer, device work list and cached graph of one persistent launch.
// The graph copies the staging buffer to the device list, resets the item
// counter and runs the persistent kernel; it is replayed while the launch
// shape (key) stays the same.
struct PersistentSlot {
  wn::WorkItem *host = nullptr;
  wn::WorkItem *dev = nullptr;
  uint32_t *counter = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipGraphExec_t exec = nullptr;
  // key of the cached graph
  uint32_t k_nitems = 0, k_dtype = 0, k_variant = 0, k_grid = 0, k_max_n = 0, k_prio = 0;
  uint32_t k_defer = 0, k_entries = 0;
  void *k_out = nullptr;
};

}  // namespace

struct wn_gen {
  int device = 0;
  uint32_t num_streams = 0;
  uint32_t R = 1, K = 0, chi2 = 0;
  uint32_t x_current = 0, transform = 0, stride = 1;
  uint32_t variate = 0;  // 0 normal, 1 exponential
  double mean = 0.0, stddev = 1.0;
  bool pool_f64 = false;
  std::vector<uint32_t> pool_n;     // per stream
  std::vector<uint64_t> pool_off;   // per stream, bytes
  std::vector<uint32_t> sizes;      // distinct pool sizes, ascending
  std::vector<std::vector<uint32_t>> streams_of_size;
  std::vector<uint32_t *> d_seed_lists;  // per distinct size: device list of its streams
  unsigned char *d_arena = nullptr;
  wn::StreamHdr *d_hdr = nullptr;
  uint32_t *d_err = nullptr;
  size_t arena_bytes = 0;
  bool seeded = false;
  hipEvent_t last = nullptr;
  bool has_last = false;
  ListSlot slots[4];
  unsigned next_slot = 0;
  std::vector<uint8_t> seen;  // duplicate check scratch
  wn::Chi2Consts cc[wn::kNumSizes];  // per pool size 2^4 .. 2^14
  double xthr[wn::kNumSizes];        // extreme-value thresholds, same sizes
  // launch choices (wn_tuning); defaults: one LDS pool buffer (faster in steady
  // state on every workload measured), graph replay
  uint32_t variant = 0;
  uint32_t wgs_per_cu = 0;
  uint32_t long_priority_pct = 25;
  uint32_t streams_per_wg = 1;
  uint32_t defer_emission = 1;  // bit 0: one-size launches of few streams, bit 1: persistent
  uint32_t group_items = 0;     // persistent launches: 1 = pairs of 1024-value items
  bool use_graph = true;
  uint32_t cus = 256;        // compute units of the device
  // persistent launches: two staging/work-list slots, each with a cached graph
  PersistentSlot pslots[2];
  unsigned next_pslot = 0;
  hipStream_t capture_stream = nullptr;
  wn::StatsPartial *d_partials = nullptr;  // fused statistics, one per request
  size_t partials_cap = 0;
  wn::StatsPartial *d_static_partials = nullptr;  // wn_fill_stats_noalloc: the static array
};

namespace {

// values a pool of n gives: n - 1 normals, or n/2 - 1 exponentials
uint32_t positions_per_pool(const wn_gen *g, uint32_t n) {
  return g->variate ? n / 2 - 1 : n - 1;
}

wn::KernelCommon common(const wn_gen *g, uint32_t n) {
  wn::KernelCommon c;
  c.hdr = g->d_hdr;
  c.arena = g->d_arena;
  c.err = g->d_err;
  c.n = n;
  c.R = g->R;
  c.K = g->K;
  c.chi2 = g->chi2;
  c.x_current = g->x_current;
  c.has_mu = g->mean != 0.0;
  c.transform = g->transform;
  c.unit_sigma = g->stddev == 1.0 ? 1u : 0u;
  c.stride = g->stride;
  c.expo = g->variate;
  c.sigma = g->stddev;
  c.mu = g->mean;
  for (int i = 0; i < wn::kNumSizes; ++i) {
    c.cc[i] = g->cc[i];
    c.xthr[i] = g->xthr[i];
  }
  return c;
}

void release(wn_gen *g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  for (auto &s : g->slots) {
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  for (auto &s : g->pslots) {
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.counter) (void)hipFree(s.counter);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
  if (g->d_partials) (void)hipFree(g->d_partials);
  for (auto *p : g->d_seed_lists)
    if (p) (void)hipFree(p);
  if (g->d_arena) (void)hipFree(g->d_arena);
  if (g->d_hdr) (void)hipFree(g->d_hdr);
  if (g->d_err) (void)hipFree(g->d_err);
  if (g->last) (void)hipEventDestroy(g->last);
  delete g;
}

// Order this call after the generator's previous one, whatever its stream.
hipError_t order_after_last(wn_gen *g, hipStream_t st) {
  if (!g->has_last) return hipSuccess;
  return hipStreamWaitEvent(st, g->last, 0);
}

hipError_t record_last(wn_gen *g, hipStream_t st) {
  hipError_t e = hipEventRecord(g->last, st);
  if (e == hipSuccess) g->has_last = true;
  return e;
}

}  // namespace

namespace {
struct StateBlobHeader {  // prefix of a saved state
  uint64_t magic;         // "WNSTATE1"
  uint32_t num_streams, pool_f64, R, K, chi2, x_current, transform, stride, variate, pad;
  double mean, stddev;
  uint64_t arena_bytes, hdr_bytes;
};
constexpr uint64_t kStateMagic = 0x3145544154534e57ull;  // "WNSTATE1" little-endian

StateBlobHeader blob_header(const wn_gen *g) {
  StateBlobHeader h{};
  h.magic = kStateMagic;
  h.num_streams = g->num_streams;
  h.pool_f64 = g->pool_f64;
  h.R = g->R;
  h.K = g->K;
  h.chi2 = g->chi2;
  h.x_current = g->x_current;
  h.transform = g->transform;
  h.stride = g->stride;
  h.variate = g->variate;
  h.mean = g->mean;
  h.stddev = g->stddev;
  h.arena_bytes = g->arena_bytes;
  h.hdr_bytes = sizeof(wn::StreamHdr) * g->num_streams;
  return h;
}
}  // namespace

extern "C" {

uint32_t wn_version(void) { return 10000u; }

double wn_extreme_threshold(uint32_t n) {
  if (n < 16 || n > 16384 || !is_pow2(n)) return std::nan("");
  return extreme_threshold(n);
}

wn_status wn_chi2_constants(uint32_t n, double *out) {
  if (!out) return fail(WN_EINVAL, "wn_chi2_constants: out is NULL");
  if (n < 16 || n > 16384 || !is_pow2(n))
    return fail(WN_EINVAL, "wn_chi2_constants: pool size %u is not a power of two in [16, 16384]",
                n);
  const wn::Chi2Consts c = chi2_consts(n);
  out[0] = c.nu;
  out[1] = c.A;
  out[2] = c.b;
  out[3] = c.fisher_root;
  out[4] = c.wh_c;
  out[5] = c.wh_shift;
  return WN_OK;
}

const char *wn_last_error(void) { return g_last_error; }

wn_status wn_create(const wn_config *cfg, wn_gen **out_gen) {
  if (!out_gen) return fail(WN_EINVAL, "wn_create: out_gen is NULL");
  *out_gen = nullptr;
  if (!cfg) return fail(WN_EINVAL, "wn_create: cfg is NULL");
  if (cfg->struct_size != sizeof(wn_config) && cfg->struct_size != WN_CONFIG_V1_SIZE &&
      cfg->struct_size != WN_CONFIG_V2_SIZE)
    return fail(WN_EINVAL, "wn_create: struct_size %u, expected %zu, %u or %u", cfg->struct_size,
                sizeof(wn_config), WN_CONFIG_V2_SIZE, WN_CONFIG_V1_SIZE);
  static_assert(offsetof(wn_config, chi2_source) == WN_CONFIG_V1_SIZE, "v1 prefix");
  static_assert(offsetof(wn_config, emit_stride) == WN_CONFIG_V2_SIZE, "v2 prefix");
  const bool v2 = cfg->struct_size >= WN_CONFIG_V2_SIZE;
  const bool v3 = cfg->struct_size == sizeof(wn_config);
  const uint32_t stride = v3 && cfg->emit_stride ? cfg->emit_stride : 1u;
  if (stride > 16) return fail(WN_EINVAL, "wn_create: emit_stride %u, at most 16", stride);
  const uint32_t variate = v3 ? wn::enum_bits(cfg->variate) : 0u;
  if (variate > 1) return fail(WN_EINVAL, "wn_create: unknown variate %u", variate);
  const uint32_t x_src = v2 ? wn::enum_bits(cfg->chi2_source) : 0u;
  const uint32_t transform = v2 ? wn::enum_bits(cfg->transform) : 0u;
  const double mean = v2 ? cfg->mean : 0.0;
  const double stddev = v2 ? cfg->stddev : 1.0;
  if (x_src > 1) return fail(WN_EINVAL, "wn_create: unknown chi2_source %u", x_src);
  if (transform > 1) return fail(WN_EINVAL, "wn_create: unknown transform %u", transform);
  if (!(std::isfinite(mean)) || !(stddev > 0.0) || !std::isfinite(stddev))
    return fail(WN_EINVAL, "wn_create: mean must be finite and stddev finite and positive");
  if (variate == 1 && (mean != 0.0 || stddev != 1.0 || stride != 1))
    return fail(WN_EINVAL, "wn_create: exponential variates take mean 0, stddev 1 and "
                           "emit_stride 1");
  // one-size launches run one workgroup of up to 256 threads per stream: 2^24
  // streams keep a grid within the 2^32 work-items of one dimension
  if (cfg->num_streams == 0 || cfg->num_streams > (1u << 24))
    return fail(WN_EINVAL, "wn_create: num_streams must be in [1, 2^24]");
  if (cfg->passes_per_output == 0 || cfg->passes_per_output > 64)
    return fail(WN_EINVAL, "wn_create: passes_per_output must be in [1, 64]");
  const uint32_t pool_dtype = wn::enum_bits(cfg->pool_dtype);
  const uint32_t chi2 = wn::enum_bits(cfg->chi2);
  if (pool_dtype != WN_F32 && pool_dtype != WN_F64)
    return fail(WN_EINVAL, "wn_create: pool_dtype must be WN_F32 or WN_F64");
  if (chi2 > WN_CHI2_WH) return fail(WN_EINVAL, "wn_create: unknown chi2 mode %u", chi2);
  auto bad_n = [](uint32_t n) { return n < 16 || n > 16384 || !is_pow2(n); };
  if (!cfg->pool_n && bad_n(cfg->default_pool_n))
    return fail(WN_EINVAL, "wn_create: pool size %u is not a power of two in [16, 16384]",
                cfg->default_pool_n);
  if (cfg->pool_n)
    for (uint32_t s = 0; s < cfg->num_streams; ++s)
      if (bad_n(cfg->pool_n[s]))
        return fail(WN_EINVAL, "wn_create: pool_n[%u] = %u is not a power of two in [16, 16384]",
                    s, cfg->pool_n[s]);

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(WN_EDEVICE, "wn_create: no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev)
    return fail(WN_EDEVICE, "wn_create: device %d out of range (%d devices)", cfg->device, ndev);
  if (hipSetDevice(cfg->device) != hipSuccess)
    return fail(WN_EDEVICE, "wn_create: hipSetDevice(%d) failed", cfg->device);

  wn_gen *g = new (std::nothrow) wn_gen();
  if (!g) return fail(WN_ENOMEM, "wn_create: host allocation failed");
  g->device = cfg->device;
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device) ==
            hipSuccess &&
        cus > 0)
      g->cus = uint32_t(cus);
  }
  g->num_streams = cfg->num_streams;
  g->R = cfg->passes_per_output;
  g->K = cfg->renorm_period;
  g->chi2 = chi2;
  g->x_current = x_src;
  g->transform = transform;
  g->stride = stride;
  g->variate = variate;
  g->mean = mean;
  g->stddev = stddev;
  g->pool_f64 = pool_dtype == WN_F64;
  const size_t esz = g->pool_f64 ? 8 : 4;
  try {
    g->pool_n.resize(cfg->num_streams);
    g->pool_off.resize(cfg->num_streams);
    g->seen.assign(cfg->num_streams, 0);
  } catch (...) {
    delete g;
    return fail(WN_ENOMEM, "wn_create: host allocation failed");
  }
  uint64_t off = 0;
  for (uint32_t s = 0; s < cfg->num_streams; ++s) {
    const uint32_t n = cfg->pool_n ? cfg->pool_n[s] : cfg->default_pool_n;
    g->pool_n[s] = n;
    g->pool_off[s] = off;
    off += (uint64_t(n) * esz + 255) & ~uint64_t(255);
  }
  g->arena_bytes = off;
  for (uint32_t s = 0; s < cfg->num_streams; ++s) {
    auto it = std::lower_bound(g->sizes.begin(), g->sizes.end(), g->pool_n[s]);
    if (it == g->sizes.end() || *it != g->pool_n[s]) {
      const size_t at = size_t(it - g->sizes.begin());
      g->sizes.insert(it, g->pool_n[s]);
      g->streams_of_size.insert(g->streams_of_size.begin() + at, std::vector<uint32_t>());
    }
  }
  for (uint32_t s = 0; s < cfg->num_streams; ++s) {
    const size_t at = size_t(std::lower_bound(g->sizes.begin(), g->sizes.end(), g->pool_n[s]) -
                             g->sizes.begin());
    g->streams_of_size[at].push_back(s);
  }

  hipError_t e = hipSuccess;
  if ((e = hipMalloc(&g->d_arena, g->arena_bytes)) != hipSuccess ||
      (e = hipMalloc(&g->d_hdr, sizeof(wn::StreamHdr) * g->num_streams)) != hipSuccess ||
      (e = hipMalloc(&g->d_err, sizeof(uint32_t))) != hipSuccess) {
    release(g);
    return hip_fail(e, "wn_create: device allocation");
  }
  g->d_seed_lists.assign(g->sizes.size(), nullptr);
  for (size_t i = 0; i < g->sizes.size(); ++i) {
    const auto &v = g->streams_of_size[i];
    if ((e = hipMalloc(&g->d_seed_lists[i], v.size() * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMemcpy(g->d_seed_lists[i], v.data(), v.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice)) != hipSuccess) {
      release(g);
      return hip_fail(e, "wn_create: stream lists");
    }
  }
  // headers: pool offsets and sizes are fixed for the generator's lifetime
  std::vector<wn::StreamHdr> hdr(g->num_streams);
  for (uint32_t s = 0; s < g->num_streams; ++s) {
    std::memset(&hdr[s], 0, sizeof(wn::StreamHdr));
    hdr[s].pool_off = g->pool_off[s];
    hdr[s].n = g->pool_n[s];
    hdr[s].cursor = positions_per_pool(g, g->pool_n[s]);  // no pool ready
  }
  if ((e = hipMemcpy(g->d_hdr, hdr.data(), hdr.size() * sizeof(wn::StreamHdr),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(g->d_err, 0, sizeof(uint32_t))) != hipSuccess ||
      (e = hipEventCreateWithFlags(&g->last, hipEventDisableTiming)) != hipSuccess) {
    release(g);
    return hip_fail(e, "wn_create: initialisation");
  }
  for (auto &s : g->slots)
    if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) {
      release(g);
      return hip_fail(e, "wn_create: events");
    }
  for (auto &s : g->pslots)
    if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipMalloc(&s.counter, sizeof(uint32_t))) != hipSuccess) {
      release(g);
      return hip_fail(e, "wn_create: persistent slots");
    }
  if ((e = hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking)) != hipSuccess) {
    release(g);
    return hip_fail(e, "wn_create: capture stream");
  }
  if ((e = wn::noalloc_partials(g->device, &g->d_static_partials)) != hipSuccess) {
    release(g);
    return hip_fail(e, "wn_create: static partials");
  }
  for (int i = 0; i < wn::kNumSizes; ++i) {
    g->cc[i] = chi2_consts(16u << i);
    g->xthr[i] = extreme_threshold(16u << i);
  }
  *out_gen = g;
  return WN_OK;
}

wn_status wn_seed(wn_gen *g, uint64_t seed, void *hip_stream) {
  if (!g) return fail(WN_EINVAL, "wn_seed: generator is NULL");
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_seed: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess) return hip_fail(e, "wn_seed: ordering");
  for (size_t i = 0; i < g->sizes.size(); ++i) {
    wn::SeedArgs a;
    a.c = common(g, g->sizes[i]);
    a.streams = g->d_seed_lists[i];
    a.nstreams = uint32_t(g->streams_of_size[i].size());
    // a rotation joins two values where the 4x4 transform joins four, so its
    // dependency sets grow half as fast: twice the passes
    a.warmup = (g->transform ? 2 : 1) * ilog2(g->sizes[i]) + 4;
    a.seed = seed;
    if ((e = wn::launch_seed(a, g->pool_f64, st)) != hipSuccess)
      return hip_fail(e, "wn_seed: launch");
  }
  if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_seed: event");
  g->seeded = true;
  return WN_OK;
}

}  // extern "C"

namespace {

// Validation shared by wn_fill and wn_autotune; sets *total.
wn_status validate_fill(wn_gen *g, const char *who, uint32_t nreq, const uint32_t *streams,
                        const uint64_t *counts, void *out, wn_dtype out_dtype, uint64_t *total) {
  if (!g) return fail(WN_EINVAL, "%s: generator is NULL", who);
  if (nreq > 0 && (!streams || !counts))
    return fail(WN_EINVAL, "%s: streams/counts are NULL with nreq = %u", who, nreq);
  const uint32_t od = wn::enum_bits(out_dtype);
  if (od > WN_F16) return fail(WN_EINVAL, "%s: unknown output dtype %u", who, od);
  if (!g->pool_f64 && od == WN_F64)
    return fail(WN_ENOTSUP, "%s: binary64 output needs a binary64 pool", who);
  uint64_t sum = 0;
  enum { kOk, kBadId, kTwice, kTooMany } why = kOk;
  uint32_t bad = 0;
  constexpr uint64_t kMaxTotal = uint64_t(1) << 56;  // values per call (no offset overflows)
  for (uint32_t j = 0; j < nreq; ++j) {
    const uint32_t s = streams[j];
    why = s >= g->num_streams ? kBadId
          : g->seen[s]        ? kTwice
          : counts[j] > kMaxTotal - sum ? kTooMany
                                        : kOk;
    if (why != kOk) {
      bad = j;
      break;
    }
    g->seen[s] = 1;
    sum += counts[j];
  }
  for (uint32_t j = 0; j < nreq; ++j)
    if (streams[j] < g->num_streams) g->seen[streams[j]] = 0;
  switch (why) {
    case kBadId:
      return fail(WN_EINVAL, "%s: request %u names stream %u of %u", who, bad, streams[bad],
                  g->num_streams);
    case kTwice: return fail(WN_EINVAL, "%s: stream %u listed twice", who, streams[bad]);
    case kTooMany:
      return fail(WN_EINVAL, "%s: request %u takes the total past 2^56 values", who, bad);
    default: break;
  }
  if (sum > 0 && !out)
    return fail(WN_EINVAL, "%s: out is NULL with %llu values requested", who,
                (unsigned long long)sum);
  if (!g->seeded) return fail(WN_ESTATE, "%s: generator not seeded", who);
  *total = sum;
  return WN_OK;
}

hipError_t reserve(wn::WorkItem **host, wn::WorkItem **dev, size_t *cap, size_t need) {
  if (*cap >= need) return hipSuccess;
  if (*host) (void)hipHostFree(*host);
  if (*dev) (void)hipFree(*dev);
  *host = nullptr;
  *dev = nullptr;
  *cap = 0;
  const size_t c = std::max<size_t>(need, 1024);
  hipError_t e = hipHostMalloc(reinterpret_cast<void **>(host), c * sizeof(wn::WorkItem),
                               hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(dev), c * sizeof(wn::WorkItem));
  if (e == hipSuccess) *cap = c;
  return e;
}

// Persistent launch of the items (pool sizes >= 1024) already written, longest
// first, to slot.host[0 .. nitems): replays the slot's graph when the launch
// shape is unchanged, captures a new one otherwise (or launches directly when
// graphs are off).
// With nentries > 0 the list is slot.host[0 .. nitems) followed by nentries
// entry words (pairs of items, kEntry*), and the launch runs the entries.
hipError_t launch_persistent(wn_gen *g, PersistentSlot &slot, uint32_t nitems, uint32_t nentries,
                             uint32_t prio_items, uint32_t max_n, void *out, uint32_t dtype,
                             wn::StatsOut *stats, wn::StatsPartial *partials, hipStream_t st) {
  wn::FillArgs a;
  a.c = common(g, 0);
  a.items = slot.dev;
  a.nitems = nentries ? nentries : nitems;
  a.entries = nentries ? reinterpret_cast<const uint32_t *>(slot.dev + nitems) : nullptr;
  a.affine_s0 = 0;
  a.count_each = 0;
  a.out = out;
  a.variant = g->variant;
  a.counter = slot.counter;
  a.prio_items = prio_items;
  a.defer = (g->defer_emission >> 1) & 1u;
  a.partials = partials;
  a.stats = stats;
  int dev = 0, cus = 256;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const uint32_t grid = g->wgs_per_cu ? uint32_t(cus) * g->wgs_per_cu : 0;
  const size_t bytes = size_t(nitems) * sizeof(wn::WorkItem) + size_t(nentries) * sizeof(uint32_t);
  if (!g->use_graph || stats) {
    if ((e = hipMemcpyAsync(slot.dev, slot.host, bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
      return e;
    return wn::launch_fill_persistent(a, g->pool_f64, dtype, max_n, grid, st);
  }
  const bool hit = slot.exec && slot.k_nitems == nitems && slot.k_dtype == dtype &&
                   slot.k_variant == g->variant && slot.k_grid == grid && slot.k_max_n == max_n &&
                   slot.k_out == out && slot.k_prio == prio_items && slot.k_defer == a.defer &&
                   slot.k_entries == nentries;
  if (!hit) {
    if (slot.exec) {
      (void)hipGraphExecDestroy(slot.exec);
      slot.exec = nullptr;
    }
    hipStream_t cs = g->capture_stream;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t e1 = hipMemcpyAsync(slot.dev, slot.host, bytes, hipMemcpyHostToDevice, cs);
    if (e1 == hipSuccess) e1 = wn::launch_fill_persistent(a, g->pool_f64, dtype, max_n, grid, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (e1 != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return e1 != hipSuccess ? e1 : e;
    }
    e = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      slot.exec = nullptr;
      return e;
    }
    slot.k_nitems = nitems;
    slot.k_dtype = dtype;
    slot.k_variant = g->variant;
    slot.k_grid = grid;
    slot.k_max_n = max_n;
    slot.k_out = out;
    slot.k_prio = prio_items;
    slot.k_defer = a.defer;
    slot.k_entries = nentries;
  }
  return hipGraphLaunch(slot.exec, st);
}

// Enqueue a validated request.  Three forms:
//  * affine (streams s0, s0+1, ... with equal counts and one pool size): one
//    workgroup per stream, no work list;
//  * otherwise, streams with pools >= 1024 go to one persistent launch over a
//    work list sorted longest first (estimated pools times (pool size + 4096));
//  * streams with smaller pools go to one launch per pool size.
// The affine form: streams s0, s0+1, ... with equal counts and one pool size.
bool is_affine(const wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts) {
  bool affine = nreq > 0;
  for (uint32_t j = 1; j < nreq && affine; ++j)
    affine = streams[j] == streams[0] + j && counts[j] == counts[0];
  if (affine)
    for (uint32_t j = 0; j < nreq && affine; ++j)
      affine = g->pool_n[streams[j]] == g->pool_n[streams[0]];
  return affine;
}

// With statistics, `partials` holds one partial per request (zeroed).
wn_status enqueue_fill(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                       void *out, wn_dtype out_dtype, hipStream_t st,
                       wn::StatsOut *stats = nullptr, wn::StatsPartial *partials = nullptr) {
  hipError_t e;
  if (is_affine(g, nreq, streams, counts)) {
    wn::FillArgs a;
    a.c = common(g, g->pool_n[streams[0]]);
    a.items = nullptr;
    a.nitems = nreq;
    a.affine_s0 = streams[0];
    a.count_each = counts[0];
    a.items_per_wg = g->streams_per_wg;
    a.out = out;
    a.variant = g->variant;
    // few streams: each has a compute unit to itself and its chain of pools is
    // the critical path
    a.defer = (g->defer_emission & 1u) && nreq <= g->cus;
    a.counter = nullptr;
    a.partials = partials;
    a.stats = stats;
    if ((e = wn::launch_fill(a, g->pool_f64, uint32_t(out_dtype), st)) != hipSuccess)
      return hip_fail(e, "wn_fill: launch");
    return WN_OK;
  }

  std::vector<uint64_t> off(nreq);
  uint64_t acc = 0;
  for (uint32_t j = 0; j < nreq; ++j) {
    off[j] = acc;
    acc += counts[j];
  }
  // Pools of 1024 values or more go to the persistent launch, smaller ones to
  // one-size launches per pool size: a persistent work list never holds a pool
  // below 1024 (its 128-thread form relies on that for lists up to 2048).
  uint32_t nbig = 0, nsmall = 0, max_n = 1024;
  for (uint32_t j = 0; j < nreq; ++j) {
    if (counts[j] == 0) continue;
    const uint32_t n = g->pool_n[streams[j]];
    if (n >= 1024) {
      ++nbig;
      max_n = std::max(max_n, n);
    } else {
      ++nsmall;
    }
  }

  if (nbig > 0) {
    PersistentSlot &slot = g->pslots[g->next_pslot];
    g->next_pslot = (g->next_pslot + 1) % 2;
    if (slot.pending) {
      if ((e = hipEventSynchronize(slot.done)) != hipSuccess)
        return hip_fail(e, "wn_fill: staging wait");
      slot.pending = false;
    }
    // Items of 1024 values may share a workgroup in pairs, one per half of 128
    // threads, in the plain loop (no statistics, thinning or rotations; pools
    // of at most 4096 values).  With the deferred form on, the items that run
    // alone take it.
    const uint32_t group = (!stats && g->stride == 1 && g->transform == 0 && !g->variate &&
                            max_n <= 4096)
                               ? g->group_items
                               : 0u;
    const size_t entry_slots = group ? (size_t(nbig) * sizeof(uint32_t) + sizeof(wn::WorkItem) - 1) /
                                           sizeof(wn::WorkItem)
                                     : 0;
    wn::WorkItem *old_dev = slot.dev;
    if ((e = reserve(&slot.host, &slot.dev, &slot.cap, nbig + entry_slots)) != hipSuccess)
      return hip_fail(e, "wn_fill: work list allocation");
    if (slot.dev != old_dev && slot.exec) {  // the cached graph points at the old list
      (void)hipGraphExecDestroy(slot.exec);
      slot.exec = nullptr;
    }
    std::vector<std::pair<uint64_t, uint32_t>> order;
    order.reserve(nbig);
    for (uint32_t j = 0; j < nreq; ++j) {
      const uint32_t n = g->pool_n[streams[j]];
      if (counts[j] == 0 || n < 1024) continue;
      // a pool's time alone grows with n from a fixed part about as large as a
      // 4096-value pool's n-proportional part (2.8, 3.4 and 4.1 thousand cycles
      // for n = 1024, 2048, 4096), so small pools cost more per value
      const uint64_t pools = counts[j] * g->stride / positions_per_pool(g, n) + 1;
      order.emplace_back(pools * (n + 4096), j);
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const auto &x, const auto &y) { return x.first > y.first; });
    uint32_t prio_items = 0, nentries = 0;
    if (!group) {
      for (uint32_t i = 0; i < nbig; ++i) {
        const uint32_t j = order[i].second;
        slot.host[i] = wn::WorkItem{streams[j], j, counts[j], off[j]};
      }
      if (g->long_priority_pct > 0) {
        const uint64_t cut = order[0].first * g->long_priority_pct / 100;
        while (prio_items < nbig && order[prio_items].first >= cut) ++prio_items;
      }
    } else {
      // Pairs of 1024-value items, neighbours in length (the list is longest
      // first).  The long items (estimated work at least long_priority_pct of
      // the longest, 25 when that is 0) run alone, as the critical path; a
      // pair's half has twice the values per thread, so its step costs about
      // what a pool of twice the size costs alone.  Entries are ordered
      // longest first; the long ones run at raised priority.
      const uint32_t pct = g->long_priority_pct ? g->long_priority_pct : 25u;
      const uint64_t cut = order[0].first * pct / 100;
      const uint32_t per = 2u;
      struct Entry {
        uint64_t est;
        uint32_t first, k;  // k requests from members[first]
      };
      std::vector<Entry> ent;
      std::vector<uint32_t> members;
      ent.reserve(nbig);
      members.reserve(nbig);
      std::vector<std::pair<uint64_t, uint32_t>> small;  // (pools, request), longest first
      for (uint32_t i = 0; i < nbig; ++i) {
        const uint32_t j = order[i].second;
        const uint32_t n = g->pool_n[streams[j]];
        if (n != 1024 || order[i].first >= cut) {
          ent.push_back(Entry{order[i].first, uint32_t(members.size()), 1});
          members.push_back(j);
        } else {
          small.emplace_back(order[i].first / (n + 4096), j);
        }
      }
      for (size_t i = 0; i < small.size(); i += per) {
        const uint32_t k = uint32_t(std::min<size_t>(per, small.size() - i));
        const uint64_t cost = k == 1 ? 1024 + 4096 : per * 1024 + 4096;
        ent.push_back(Entry{small[i].first * cost, uint32_t(members.size()), k});
        for (uint32_t m = 0; m < k; ++m) members.push_back(small[i + m].second);
      }
      std::stable_sort(ent.begin(), ent.end(),
                       [](const Entry &x, const Entry &y) { return x.est > y.est; });
      auto *words = reinterpret_cast<uint32_t *>(slot.host + nbig);
      uint32_t k = 0;
      for (const Entry &en : ent) {
        const uint32_t kind = en.k == 2 ? wn::kEntryPair : wn::kEntrySolo;
        words[nentries++] = k | (kind << wn::kEntryKindShift);
        for (uint32_t m = 0; m < en.k; ++m) {
          const uint32_t j = members[en.first + m];
          slot.host[k++] = wn::WorkItem{streams[j], j, counts[j], off[j]};
        }
        if (en.est >= cut) ++prio_items;
      }
    }
    if ((e = launch_persistent(g, slot, nbig, nentries, prio_items, max_n, out,
                               uint32_t(out_dtype), stats, partials, st)) != hipSuccess)
      return hip_fail(e, "wn_fill: persistent launch");
    if ((e = hipEventRecord(slot.done, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
    slot.pending = true;
  }

  if (nsmall > 0) {
    ListSlot &slot = g->slots[g->next_slot];
    g->next_slot = (g->next_slot + 1) % 4;
    if (slot.pending) {
      if ((e = hipEventSynchronize(slot.done)) != hipSuccess)
        return hip_fail(e, "wn_fill: staging wait");
      slot.pending = false;
    }
    if ((e = reserve(&slot.host, &slot.dev, &slot.cap, nsmall)) != hipSuccess)
      return hip_fail(e, "wn_fill: work list allocation");
    // bucket by pool size, request order inside a bucket
    auto size_index = [&](uint32_t n) {
      return uint32_t(std::lower_bound(g->sizes.begin(), g->sizes.end(), n) - g->sizes.begin());
    };
    std::vector<uint32_t> start(g->sizes.size() + 1, 0);
    for (uint32_t j = 0; j < nreq; ++j) {
      const uint32_t n = g->pool_n[streams[j]];
      if (counts[j] > 0 && n < 1024) start[size_index(n) + 1]++;
    }
    for (size_t b = 0; b < g->sizes.size(); ++b) start[b + 1] += start[b];
    std::vector<uint32_t> pos(start.begin(), start.end() - 1);
    for (uint32_t j = 0; j < nreq; ++j) {
      const uint32_t n = g->pool_n[streams[j]];
      if (counts[j] == 0 || n >= 1024) continue;
      slot.host[pos[size_index(n)]++] = wn::WorkItem{streams[j], j, counts[j], off[j]};
    }
    if ((e = hipMemcpyAsync(slot.dev, slot.host, nsmall * sizeof(wn::WorkItem),
                            hipMemcpyHostToDevice, st)) != hipSuccess)
      return hip_fail(e, "wn_fill: work list upload");
    for (size_t b = 0; b < g->sizes.size(); ++b) {
      const uint32_t cnt = start[b + 1] - start[b];
      if (cnt == 0) continue;
      wn::FillArgs a;
      a.c = common(g, g->sizes[b]);
      a.items = slot.dev + start[b];
      a.nitems = cnt;
      a.affine_s0 = 0;
      a.count_each = 0;
      a.out = out;
      a.variant = g->variant;
      a.counter = nullptr;
      a.partials = partials;
      a.stats = stats;
      if ((e = wn::launch_fill(a, g->pool_f64, uint32_t(out_dtype), st)) != hipSuccess)
        return hip_fail(e, "wn_fill: launch");
    }
    if ((e = hipEventRecord(slot.done, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
    slot.pending = true;
  }
  return WN_OK;
}

wn_status validate_stats(const char *who, uint32_t nreq, const uint64_t *counts,
                         const wn_stats *stats) {
  if (!stats || reinterpret_cast<uintptr_t>(stats) % 8 != 0)
    return fail(WN_EINVAL, "%s: stats is NULL or not 8-byte aligned", who);
  for (uint32_t j = 0; j < nreq; ++j)
    if (counts[j] >= (uint64_t(1) << 32))
      return fail(WN_EINVAL, "%s: request %u counts 2^32 values or more", who, j);
  return WN_OK;
}

// The statistics call after validation and ordering: zero the result and
// max(nreq, 1) partials (kernels, not memsets), fill, reduce, record.
wn_status enqueue_fill_stats(wn_gen *g, const char *who, uint32_t nreq, const uint32_t *streams,
                             const uint64_t *counts, void *out, wn_dtype out_dtype,
                             wn_stats *stats, wn::StatsPartial *partials, uint64_t total,
                             hipStream_t st) {
  hipError_t e;
  const size_t need = std::max<size_t>(nreq, 1);
  auto *so = reinterpret_cast<wn::StatsOut *>(stats);
  if ((e = wn::stats_zero(so, st)) != hipSuccess ||
      (e = wn::zero_words(partials, uint32_t(need * sizeof(wn::StatsPartial) / 8), st)) !=
          hipSuccess)
    return hip_fail(e, who, "zero");
  if (total > 0) {
    wn_status v = enqueue_fill(g, nreq, streams, counts, out, out_dtype, st, so, partials);
    if (v != WN_OK) return v;
  }
  if ((e = wn::stats_reduce(partials, nreq, so, st)) != hipSuccess)
    return hip_fail(e, who, "reduce");
  if ((e = record_last(g, st)) != hipSuccess)
    return hip_fail(e, who, "event");
  return WN_OK;
}

}  // namespace

extern "C" {

wn_status wn_fill(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                  void *out, wn_dtype out_dtype, void *hip_stream) {
  uint64_t total = 0;
  wn_status v = validate_fill(g, "wn_fill", nreq, streams, counts, out, out_dtype, &total);
  if (v != WN_OK) return v;
  if (total == 0) return WN_OK;
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_fill: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill: ordering");
  v = enqueue_fill(g, nreq, streams, counts, out, out_dtype, st);
  if (v != WN_OK) return v;
  if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
  return WN_OK;
}

wn_status wn_fill_stats(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                        void *out, wn_dtype out_dtype, wn_stats *stats, void *hip_stream) {
  static_assert(sizeof(wn_stats) == sizeof(wn::StatsOut), "wn_stats layout");
  uint64_t total = 0;
  wn_status v = validate_fill(g, "wn_fill_stats", nreq, streams, counts, out, out_dtype, &total);
  if (v != WN_OK) return v;
  if ((v = validate_stats("wn_fill_stats", nreq, counts, stats)) != WN_OK) return v;
  if (g->variate)
    return fail(WN_ENOTSUP, "wn_fill_stats: the statistics are those of normal values");
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_fill_stats: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill_stats: ordering");
  const size_t need = std::max<size_t>(nreq, 1);
  if (g->partials_cap < need) {
    // the previous buffer may still be read by queued work: wait before freeing
    if (g->d_partials) {
      if (g->has_last && (e = hipEventSynchronize(g->last)) != hipSuccess)
        return hip_fail(e, "wn_fill_stats: wait");
      (void)hipFree(g->d_partials);
      g->d_partials = nullptr;
      g->partials_cap = 0;
    }
    if ((e = hipMalloc(&g->d_partials, need * sizeof(wn::StatsPartial))) != hipSuccess)
      return hip_fail(e, "wn_fill_stats: partials");
    g->partials_cap = need;
  }
  return enqueue_fill_stats(g, "wn_fill_stats", nreq, streams, counts, out, out_dtype, stats,
                            g->d_partials, total, st);
}

static_assert(wn::kNoAllocRequests == WN_NOALLOC_MAX_REQUESTS, "static partials of wn.h");

wn_status wn_fill_stats_noalloc(wn_gen *g, uint32_t nreq, const uint32_t *streams,
                                const uint64_t *counts, void *out, wn_dtype out_dtype,
                                wn_stats *stats, void *hip_stream) {
  uint64_t total = 0;
  const char *who = "wn_fill_stats_noalloc";
  wn_status v = validate_fill(g, who, nreq, streams, counts, out, out_dtype, &total);
  if (v != WN_OK) return v;
  if ((v = validate_stats(who, nreq, counts, stats)) != WN_OK) return v;
  if (g->variate) return fail(WN_ENOTSUP, "%s: the statistics are those of normal values", who);
  if (nreq > wn::kNoAllocRequests)
    return fail(WN_EINVAL, "%s: %u requests, at most %u (the statically allocated partials)", who,
                nreq, wn::kNoAllocRequests);
  if (nreq > 1 && !is_affine(g, nreq, streams, counts))
    return fail(WN_ENOTSUP,
                "%s: the requests must name consecutive streams with one count and one pool "
                "size (other request lists need a work list, which is allocated)",
                who);
  if (!g->d_static_partials)
    return fail(WN_EDEVICE, "%s: the static partials were not found at wn_create", who);
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_fill_stats_noalloc: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess)
    return hip_fail(e, "wn_fill_stats_noalloc: ordering");
  return enqueue_fill_stats(g, who, nreq, streams, counts, out, out_dtype, stats,
                            g->d_static_partials, total, st);
}

wn_status wn_sync(wn_gen *g) {
  if (!g) return fail(WN_EINVAL, "wn_sync: generator is NULL");
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess && g->has_last) e = hipEventSynchronize(g->last);
  if (e != hipSuccess) return hip_fail(e, "wn_sync");
  uint32_t err = 0;
  if ((e = hipMemcpy(&err, g->d_err, sizeof(err), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "wn_sync: fault word");
  if (err) {
    (void)hipMemset(g->d_err, 0, sizeof(uint32_t));
    return fail(WN_EDEVICE, "wn_sync: a kernel met a non-finite or zero sum of squares");
  }
  return WN_OK;
}

wn_status wn_get_stream(wn_gen *g, uint32_t s, wn_stream_info *info, void *pool_out) {
  if (!g || !info) return fail(WN_EINVAL, "wn_get_stream: NULL argument");
  if (s >= g->num_streams)
    return fail(WN_EINVAL, "wn_get_stream: stream %u of %u", s, g->num_streams);
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess && g->has_last) e = hipEventSynchronize(g->last);
  if (e != hipSuccess) return hip_fail(e, "wn_get_stream");
  wn::StreamHdr h;
  if ((e = hipMemcpy(&h, g->d_hdr + s, sizeof(h), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "wn_get_stream: header");
  info->xs = h.xs;
  info->k = h.k;
  info->n = h.n;
  info->cursor = h.cursor;
  info->f = h.f;
  info->xnext = h.xnext;
  info->qlast = h.qlast;
  if (pool_out &&
      (e = hipMemcpy(pool_out, g->d_arena + g->pool_off[s],
                     size_t(g->pool_n[s]) * (g->pool_f64 ? 8 : 4), hipMemcpyDeviceToHost)) !=
          hipSuccess)
    return hip_fail(e, "wn_get_stream: pool");
  return WN_OK;
}

wn_status wn_set_tuning(wn_gen *g, const wn_tuning *t) {
  if (!g || !t) return fail(WN_EINVAL, "wn_set_tuning: NULL argument");
  if (t->struct_size != sizeof(wn_tuning))
    return fail(WN_EINVAL, "wn_set_tuning: struct_size %u, expected %zu", t->struct_size,
                sizeof(wn_tuning));
  const uint32_t w = t->waves_per_simd;
  const uint32_t wcode = w == 0 ? 0u : w == 8 ? 1u : w == 6 ? 2u : w == 5 ? 3u : 4u;
  if (t->lds_double_buffer > 1 || t->nontemporal_stores > 1 || wcode > 3 || t->use_graph > 1 ||
      (wcode && t->nontemporal_stores) || t->wgs_per_cu > 16 || t->long_priority_pct > 100 ||
      t->streams_per_wg < 1 || t->streams_per_wg > 16 || t->defer_emission > 3 ||
      t->group_items > 1 ||
      (t->threads_per_stream != 0 && t->threads_per_stream != 128 && t->threads_per_stream != 256))
    return fail(WN_EINVAL, "wn_set_tuning: flags must be 0 or 1, waves_per_simd 0/5/6/8 and "
                           "not with nontemporal_stores, wgs_per_cu <= 16, "
                           "long_priority_pct <= 100, streams_per_wg in [1, 16], "
                           "defer_emission <= 3, threads_per_stream 0, 128 or 256");
  g->variant = t->lds_double_buffer | (t->nontemporal_stores << 1) | (wcode << 2) |
               (t->threads_per_stream == 128 ? wn::kVariantThreads128 : 0u);
  g->wgs_per_cu = t->wgs_per_cu;
  g->use_graph = t->use_graph != 0;
  g->long_priority_pct = t->long_priority_pct;
  g->streams_per_wg = t->streams_per_wg;
  g->defer_emission = t->defer_emission;
  g->group_items = t->group_items;
  return WN_OK;
}

wn_status wn_get_tuning(wn_gen *g, wn_tuning *t) {
  if (!g || !t) return fail(WN_EINVAL, "wn_get_tuning: NULL argument");
  t->struct_size = sizeof(wn_tuning);
  t->lds_double_buffer = g->variant & 1u;
  t->nontemporal_stores = (g->variant >> 1) & 1u;
  static const uint32_t kWaves[4] = {0u, 8u, 6u, 5u};
  t->waves_per_simd = kWaves[(g->variant >> 2) & 3u];
  t->wgs_per_cu = g->wgs_per_cu;
  t->use_graph = g->use_graph ? 1u : 0u;
  t->long_priority_pct = g->long_priority_pct;
  t->streams_per_wg = g->streams_per_wg;
  t->defer_emission = g->defer_emission;
  t->group_items = g->group_items;
  t->threads_per_stream = (g->variant & wn::kVariantThreads128) ? 128u : 256u;
  return WN_OK;
}

wn_status wn_autotune(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                      void *out, wn_dtype out_dtype, void *hip_stream, wn_tuning *best) {
  uint64_t total = 0;
  wn_status v = validate_fill(g, "wn_autotune", nreq, streams, counts, out, out_dtype, &total);
  if (v != WN_OK) return v;
  wn_tuning cur;
  wn_get_tuning(g, &cur);
  if (total == 0) {
    if (best) *best = cur;
    return WN_OK;
  }
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_autotune: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess) return hip_fail(e, "wn_autotune: ordering");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "wn_autotune: sync");

  // which form will the request take?
  bool affine = nreq > 0;
  for (uint32_t j = 1; j < nreq && affine; ++j)
    affine = streams[j] == streams[0] + j && counts[j] == counts[0] &&
             g->pool_n[streams[j]] == g->pool_n[streams[0]];
  std::vector<wn_tuning> cands;
  auto add = [&](uint32_t db, uint32_t nt, uint32_t oc, uint32_t wpc, uint32_t prio,
                 uint32_t spw = 1, uint32_t defer = 0, uint32_t group = 0,
                 uint32_t threads = 256) {
    wn_tuning t = cur;
    t.threads_per_stream = threads;
    t.group_items = group;
    t.defer_emission = defer;
    t.streams_per_wg = spw;
    t.lds_double_buffer = db;
    t.nontemporal_stores = nt;
    t.waves_per_simd = oc;
    t.wgs_per_cu = wpc;
    t.long_priority_pct = prio;
    cands.push_back(t);
  };
  // the deferred form is a candidate where it applies (and is otherwise ignored)
  const uint32_t keep_defer = cur.defer_emission;
  if (affine) {
    for (uint32_t spw : {1u, 2u, 4u, 8u})
      for (uint32_t db = 0; db < 2; ++db)
        add(db, 0, 0, cur.wgs_per_cu, cur.long_priority_pct, spw, keep_defer & 2u);
    // register caps for 5 and 6 waves per SIMD (one LDS buffer): their few
    // spills sit outside the pool loop, and the extra workgroup per compute
    // unit pays where the kernel waits on barriers rather than on memory
    // (16-bit outputs)
    for (uint32_t oc : {5u, 6u}) add(0, 0, oc, cur.wgs_per_cu, cur.long_priority_pct, 1, keep_defer & 2u);
    // 128 threads per stream for pools of 1024 to 4096 values
    const uint32_t n0 = nreq > 0 ? g->pool_n[streams[0]] : 0u;
    if (n0 >= 1024 && n0 <= 4096 && g->transform == 0)
      for (uint32_t db = 0; db < 2; ++db)
        add(db, 0, 0, cur.wgs_per_cu, cur.long_priority_pct, 1, keep_defer & 2u, 0, 128);
    add(1, 1, 0, cur.wgs_per_cu, cur.long_priority_pct, 1, keep_defer & 2u);
    if (nreq <= g->cus) add(1, 0, 0, cur.wgs_per_cu, cur.long_priority_pct, 1, keep_defer | 1u);
  } else {
    for (uint32_t group = 0; group < 2; ++group)
      for (uint32_t prio : {0u, 10u, 25u})
        for (uint32_t db = 0; db < 2; ++db)
          for (uint32_t wpc : {0u, 3u, 4u, 6u})
            add(db, 0, 0, wpc, prio, 1, keep_defer & 1u, group);
    add(1, 1, 0, 0, 25, 1, keep_defer & 1u);
    // 128 threads per item where every pool holds at most 2048 values
    uint32_t max_n = 0;
    for (uint32_t j = 0; j < nreq; ++j) max_n = std::max(max_n, g->pool_n[streams[j]]);
    if (max_n >= 1024 && max_n <= 2048 && g->transform == 0 && g->stride == 1)
      for (uint32_t prio : {0u, 25u})
        for (uint32_t db = 0; db < 2; ++db)
          for (uint32_t wpc : {0u, 4u, 8u}) add(db, 0, 0, wpc, prio, 1, keep_defer & 1u, 0, 128);
    for (uint32_t group = 0; group < 2; ++group)
      for (uint32_t prio : {0u, 25u, 50u})
        for (uint32_t wpc : {0u, 2u, 3u, 4u}) add(1, 0, 0, wpc, prio, 1, keep_defer | 2u, group);
  }

  // snapshot of the state, restored after every candidate
  const size_t hdr_bytes = sizeof(wn::StreamHdr) * g->num_streams;
  unsigned char *save = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  auto cleanup = [&]() {
    if (save) (void)hipFree(save);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  if ((e = hipMalloc(&save, g->arena_bytes + hdr_bytes)) != hipSuccess ||
      (e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "wn_autotune: scratch");
  }
  auto restore = [&]() -> hipError_t {
    hipError_t r = hipMemcpyAsync(g->d_arena, save, g->arena_bytes, hipMemcpyDeviceToDevice, st);
    if (r == hipSuccess)
      r = hipMemcpyAsync(g->d_hdr, save + g->arena_bytes, hdr_bytes, hipMemcpyDeviceToDevice, st);
    return r;
  };
  if ((e = hipMemcpyAsync(save, g->d_arena, g->arena_bytes, hipMemcpyDeviceToDevice, st)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(save + g->arena_bytes, g->d_hdr, hdr_bytes, hipMemcpyDeviceToDevice,
                          st)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "wn_autotune: snapshot");
  }
  // One measurement of a candidate: an untimed call, then the mean of three
  // calls back to back, as continuing calls run (timing a call right after the
  // state restore favoured launch shapes that are slower in steady state); the
  // state is restored afterwards.
  auto time_once = [&](const wn_tuning &t, float *ms) -> wn_status {
    wn_set_tuning(g, &t);
    wn_status r = enqueue_fill(g, nreq, streams, counts, out, out_dtype, st);
    if (r != WN_OK) return r;
    if ((e = hipEventRecord(t0, st)) != hipSuccess) return WN_EDEVICE;
    for (int i = 0; i < 3; ++i)
      if ((r = enqueue_fill(g, nreq, streams, counts, out, out_dtype, st)) != WN_OK) return r;
    if ((e = hipEventRecord(t1, st)) != hipSuccess || (e = restore()) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess ||
        (e = hipEventElapsedTime(ms, t0, t1)) != hipSuccess)
      return WN_EDEVICE;
    *ms /= 3.f;
    return WN_OK;
  };
  auto give_up = [&](wn_status r) -> wn_status {
    wn_set_tuning(g, &cur);
    (void)restore();
    (void)hipStreamSynchronize(st);
    cleanup();
    return r == WN_EDEVICE ? hip_fail(e, "wn_autotune: run") : r;
  };
  // A first measurement of candidate 0 warms caches and code objects and is
  // dropped.  Then every candidate twice (the better counts), and the three
  // fastest five more times each in turn, ranked by their median, so that
  // run-to-run noise of a few percent does not pick a candidate that is slower
  // on average.
  float ms = 0.f;
  wn_status r = time_once(cands[0], &ms);
  if (r != WN_OK) return give_up(r);
  std::vector<std::pair<float, size_t>> first;
  for (size_t c = 0; c < cands.size(); ++c) {
    float best2 = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      if ((r = time_once(cands[c], &ms)) != WN_OK) return give_up(r);
      best2 = std::min(best2, ms);
    }
    first.emplace_back(best2, c);
  }
  std::sort(first.begin(), first.end());
  const size_t nfinal = std::min<size_t>(3, first.size());
  std::vector<std::vector<float>> runs(nfinal);
  for (int rep = 0; rep < 5; ++rep)
    for (size_t f = 0; f < nfinal; ++f) {
      if ((r = time_once(cands[first[f].second], &ms)) != WN_OK) return give_up(r);
      runs[f].push_back(ms);
    }
  // Finalists within 1% of the best median are ties: the one earliest in the
  // candidate list wins (the list starts with the defaults), so that launch
  // variants equal within noise do not alternate from one run to the next.
  std::vector<float> med(nfinal);
  float best_ms = 1e30f;
  for (size_t f = 0; f < nfinal; ++f) {
    std::sort(runs[f].begin(), runs[f].end());
    med[f] = runs[f][runs[f].size() / 2];
    best_ms = std::min(best_ms, med[f]);
  }
  size_t pick = cands.size();
  for (size_t f = 0; f < nfinal; ++f)
    if (med[f] <= best_ms * 1.01f) pick = std::min(pick, first[f].second);
  const wn_tuning chosen = cands[pick];
  wn_set_tuning(g, &chosen);
  cleanup();
  if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_autotune: event");
  if (best) *best = chosen;
  return WN_OK;
}

size_t wn_state_size(const wn_gen *g) {
  if (!g) return 0;
  return sizeof(StateBlobHeader) + g->arena_bytes + sizeof(wn::StreamHdr) * g->num_streams;
}

wn_status wn_save_state(wn_gen *g, void *host_buf, size_t bytes) {
  if (!g || !host_buf) return fail(WN_EINVAL, "wn_save_state: NULL argument");
  if (bytes != wn_state_size(g))
    return fail(WN_EINVAL, "wn_save_state: buffer of %zu bytes, need %zu", bytes,
                wn_state_size(g));
  if (!g->seeded) return fail(WN_ESTATE, "wn_save_state: generator not seeded");
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess && g->has_last) e = hipEventSynchronize(g->last);
  if (e != hipSuccess) return hip_fail(e, "wn_save_state");
  const StateBlobHeader h = blob_header(g);
  auto *dst = static_cast<unsigned char *>(host_buf);
  std::memcpy(dst, &h, sizeof(h));
  if ((e = hipMemcpy(dst + sizeof(h), g->d_hdr, h.hdr_bytes, hipMemcpyDeviceToHost)) !=
          hipSuccess ||
      (e = hipMemcpy(dst + sizeof(h) + h.hdr_bytes, g->d_arena, h.arena_bytes,
                     hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "wn_save_state: copy");
  return WN_OK;
}

wn_status wn_load_state(wn_gen *g, const void *host_buf, size_t bytes) {
  if (!g || !host_buf) return fail(WN_EINVAL, "wn_load_state: NULL argument");
  if (bytes != wn_state_size(g))
    return fail(WN_EINVAL, "wn_load_state: buffer of %zu bytes, need %zu", bytes,
                wn_state_size(g));
  StateBlobHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  const StateBlobHeader want = blob_header(g);
  if (std::memcmp(&h, &want, sizeof(h)) != 0)
    return fail(WN_EINVAL, "wn_load_state: the state was saved under another configuration");
  const auto *src = static_cast<const unsigned char *>(host_buf);
  // Every saved header must describe this generator's own pool (size and
  // arena offset) with a cursor inside it: the kernels size and index LDS
  // and the arena from these fields.
  for (uint32_t s = 0; s < g->num_streams; ++s) {
    wn::StreamHdr hs;
    std::memcpy(&hs, src + sizeof(h) + size_t(s) * sizeof(hs), sizeof(hs));
    if (hs.n != g->pool_n[s] || hs.pool_off != g->pool_off[s] ||
        hs.cursor > positions_per_pool(g, hs.n) ||
        (hs.sflags & ~uint16_t(wn::kHeldExtreme | wn::kSeenByStats)) != 0)
      return fail(WN_EINVAL, "wn_load_state: stream %u's saved header does not fit this "
                             "generator (pool size, offset, cursor or flags)", s);
  }
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess && g->has_last) e = hipEventSynchronize(g->last);
  if (e != hipSuccess) return hip_fail(e, "wn_load_state");
  if ((e = hipMemcpy(g->d_hdr, src + sizeof(h), h.hdr_bytes, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(g->d_arena, src + sizeof(h) + h.hdr_bytes, h.arena_bytes,
                     hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "wn_load_state: copy");
  g->seeded = true;
  return WN_OK;
}

void wn_destroy(wn_gen *g) { release(g); }

}  // extern "C"

namespace wn {
void set_last_error(const char *msg) {
  std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg);
}
}  // namespace wn
