// C ABI of the Wallace normal generator: validation, device memory, work
// lists and launches.  Declared in include/wn.h.
//
// Nothing here computes normals: every step of generation runs in the kernels
// of wn_kernels.hip.  The host computes only the per-pool-size chi-square
// constants (Section 5.5) with plain IEEE arithmetic, once per generator.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "wn.h"
#include "wn_internal.hpp"

namespace {

thread_local std::string g_last_error;

wn_status fail(wn_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

wn_status hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? WN_ENOMEM : WN_EDEVICE, "%s: %s", what,
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

// A pinned staging buffer and its device twin for one work list.  A slot is
// reused only after the event recorded behind its last use has completed.
struct ListSlot {
  wn::WorkItem *host = nullptr;
  wn::WorkItem *dev = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

}  // namespace

struct wn_gen {
  int device = 0;
  uint32_t num_streams = 0;
  uint32_t R = 1, K = 0, chi2 = 0;
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
  uint32_t variant = 1;       // non-semantic kernel variant (wn_tuning); LDS double buffer
};

namespace {

wn::KernelCommon common(const wn_gen *g, uint32_t n) {
  wn::KernelCommon c;
  c.hdr = g->d_hdr;
  c.arena = g->d_arena;
  c.err = g->d_err;
  c.n = n;
  c.R = g->R;
  c.K = g->K;
  c.chi2 = g->chi2;
  c.cc = chi2_consts(n);
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

bool alloc_fault_injected() {
  const char *v = std::getenv("WN_FAULT_ALLOC");
  return v && v[0] == '1';
}

}  // namespace

extern "C" {

uint32_t wn_version(void) { return 10000u; }

const char *wn_last_error(void) { return g_last_error.c_str(); }

wn_status wn_create(const wn_config *cfg, wn_gen **out_gen) {
  if (!out_gen) return fail(WN_EINVAL, "wn_create: out_gen is NULL");
  *out_gen = nullptr;
  if (!cfg) return fail(WN_EINVAL, "wn_create: cfg is NULL");
  if (cfg->struct_size != sizeof(wn_config))
    return fail(WN_EINVAL, "wn_create: struct_size %u, expected %zu", cfg->struct_size,
                sizeof(wn_config));
  if (cfg->num_streams == 0) return fail(WN_EINVAL, "wn_create: num_streams must be >= 1");
  if (cfg->passes_per_output == 0 || cfg->passes_per_output > 64)
    return fail(WN_EINVAL, "wn_create: passes_per_output must be in [1, 64]");
  if (cfg->pool_dtype != WN_F32 && cfg->pool_dtype != WN_F64)
    return fail(WN_EINVAL, "wn_create: pool_dtype must be WN_F32 or WN_F64");
  if (cfg->chi2 < WN_CHI2_CUBIC || cfg->chi2 > WN_CHI2_WH)
    return fail(WN_EINVAL, "wn_create: unknown chi2 mode %d", int(cfg->chi2));
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
  g->num_streams = cfg->num_streams;
  g->R = cfg->passes_per_output;
  g->K = cfg->renorm_period;
  g->chi2 = uint32_t(cfg->chi2);
  g->pool_f64 = cfg->pool_dtype == WN_F64;
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
  if (alloc_fault_injected()) {
    delete g;
    return fail(WN_ENOMEM, "wn_create: device allocation failed (injected)");
  }
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
    hdr[s].cursor = g->pool_n[s] - 1;
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
    a.warmup = ilog2(g->sizes[i]) + 4;
    a.seed = seed;
    if ((e = wn::launch_seed(a, g->pool_f64, st)) != hipSuccess)
      return hip_fail(e, "wn_seed: launch");
  }
  if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_seed: event");
  g->seeded = true;
  return WN_OK;
}

wn_status wn_fill(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                  void *out, wn_dtype out_dtype, void *hip_stream) {
  if (!g) return fail(WN_EINVAL, "wn_fill: generator is NULL");
  if (nreq > 0 && (!streams || !counts))
    return fail(WN_EINVAL, "wn_fill: streams/counts are NULL with nreq = %u", nreq);
  if (out_dtype < WN_F64 || out_dtype > WN_F16)
    return fail(WN_EINVAL, "wn_fill: unknown output dtype %d", int(out_dtype));
  if (!g->pool_f64 && out_dtype == WN_F64)
    return fail(WN_ENOTSUP, "wn_fill: binary64 output needs a binary64 pool");
  uint64_t total = 0;
  bool ok = true;
  uint32_t bad = 0;
  for (uint32_t j = 0; j < nreq && ok; ++j) {
    const uint32_t s = streams[j];
    if (s >= g->num_streams) {
      ok = false;
      bad = j;
      break;
    }
    if (g->seen[s]) {
      ok = false;
      bad = j;
      break;
    }
    g->seen[s] = 1;
    if (counts[j] > (uint64_t(1) << 56) || total + counts[j] < total) {
      ok = false;
      bad = j;
      break;
    }
    total += counts[j];
  }
  for (uint32_t j = 0; j < nreq; ++j)
    if (streams[j] < g->num_streams) g->seen[streams[j]] = 0;
  if (!ok) {
    if (streams[bad] >= g->num_streams)
      return fail(WN_EINVAL, "wn_fill: request %u names stream %u of %u", bad, streams[bad],
                  g->num_streams);
    if (counts[bad] > (uint64_t(1) << 56))
      return fail(WN_EINVAL, "wn_fill: request %u count too large", bad);
    return fail(WN_EINVAL, "wn_fill: stream %u listed twice", streams[bad]);
  }
  if (total > 0 && !out) return fail(WN_EINVAL, "wn_fill: out is NULL with %llu values requested",
                                     (unsigned long long)total);
  if (!g->seeded) return fail(WN_ESTATE, "wn_fill: generator not seeded");
  if (total == 0) return WN_OK;

  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "wn_fill: hipSetDevice");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((e = order_after_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill: ordering");

  // Affine form (streams s0, s0+1, ... with equal counts, one pool size):
  // no work list upload.
  bool affine = nreq > 0;
  for (uint32_t j = 1; j < nreq && affine; ++j)
    affine = streams[j] == streams[0] + j && counts[j] == counts[0];
  if (affine)
    for (uint32_t j = 0; j < nreq && affine; ++j)
      affine = g->pool_n[streams[j]] == g->pool_n[streams[0]];
  if (affine) {
    wn::FillArgs a;
    a.c = common(g, g->pool_n[streams[0]]);
    a.items = nullptr;
    a.nitems = nreq;
    a.affine_s0 = streams[0];
    a.count_each = counts[0];
    a.out = out;
    a.variant = g->variant;
    if ((e = wn::launch_fill(a, g->pool_f64, uint32_t(out_dtype), st)) != hipSuccess)
      return hip_fail(e, "wn_fill: launch");
    if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
    return WN_OK;
  }

  // General form: a work list per pool size, grouped and ordered by size.
  ListSlot &slot = g->slots[g->next_slot];
  g->next_slot = (g->next_slot + 1) % 4;
  if (slot.pending) {
    if ((e = hipEventSynchronize(slot.done)) != hipSuccess)
      return hip_fail(e, "wn_fill: staging wait");
    slot.pending = false;
  }
  if (slot.cap < nreq) {
    if (slot.host) (void)hipHostFree(slot.host);
    if (slot.dev) (void)hipFree(slot.dev);
    slot.host = nullptr;
    slot.dev = nullptr;
    slot.cap = 0;
    const size_t cap = std::max<size_t>(nreq, 1024);
    if ((e = hipHostMalloc(&slot.host, cap * sizeof(wn::WorkItem), hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipMalloc(&slot.dev, cap * sizeof(wn::WorkItem))) != hipSuccess)
      return hip_fail(e, "wn_fill: work list allocation");
    slot.cap = cap;
  }
  std::vector<uint64_t> off(nreq);
  uint64_t acc = 0;
  for (uint32_t j = 0; j < nreq; ++j) {
    off[j] = acc;
    acc += counts[j];
  }
  // bucket by pool size, keeping request order inside a bucket
  std::vector<uint32_t> bucket_start(g->sizes.size() + 1, 0);
  auto size_index = [&](uint32_t n) {
    return uint32_t(std::lower_bound(g->sizes.begin(), g->sizes.end(), n) - g->sizes.begin());
  };
  for (uint32_t j = 0; j < nreq; ++j) bucket_start[size_index(g->pool_n[streams[j]]) + 1]++;
  for (size_t b = 0; b < g->sizes.size(); ++b) bucket_start[b + 1] += bucket_start[b];
  std::vector<uint32_t> fillpos(bucket_start.begin(), bucket_start.end() - 1);
  for (uint32_t j = 0; j < nreq; ++j) {
    const uint32_t b = size_index(g->pool_n[streams[j]]);
    wn::WorkItem &it = slot.host[fillpos[b]++];
    it.stream = streams[j];
    it.pad = 0;
    it.count = counts[j];
    it.out_off = off[j];
  }
  if ((e = hipMemcpyAsync(slot.dev, slot.host, nreq * sizeof(wn::WorkItem),
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "wn_fill: work list upload");
  for (size_t b = 0; b < g->sizes.size(); ++b) {
    const uint32_t cnt = bucket_start[b + 1] - bucket_start[b];
    if (cnt == 0) continue;
    wn::FillArgs a;
    a.c = common(g, g->sizes[b]);
    a.items = slot.dev + bucket_start[b];
    a.nitems = cnt;
    a.affine_s0 = 0;
    a.count_each = 0;
    a.out = out;
    a.variant = g->variant;
    if ((e = wn::launch_fill(a, g->pool_f64, uint32_t(out_dtype), st)) != hipSuccess)
      return hip_fail(e, "wn_fill: launch");
  }
  if ((e = hipEventRecord(slot.done, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
  slot.pending = true;
  if ((e = record_last(g, st)) != hipSuccess) return hip_fail(e, "wn_fill: event");
  return WN_OK;
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
  if (t->lds_double_buffer > 1 || t->nontemporal_stores > 1 || t->high_occupancy > 1 ||
      (t->high_occupancy && t->nontemporal_stores))
    return fail(WN_EINVAL, "wn_set_tuning: flags must be 0 or 1 (high_occupancy without "
                           "nontemporal_stores)");
  g->variant = t->lds_double_buffer | (t->nontemporal_stores << 1) | (t->high_occupancy << 2);
  return WN_OK;
}

wn_status wn_get_tuning(wn_gen *g, wn_tuning *t) {
  if (!g || !t) return fail(WN_EINVAL, "wn_get_tuning: NULL argument");
  t->struct_size = sizeof(wn_tuning);
  t->lds_double_buffer = g->variant & 1u;
  t->nontemporal_stores = (g->variant >> 1) & 1u;
  t->high_occupancy = (g->variant >> 2) & 1u;
  return WN_OK;
}

void wn_destroy(wn_gen *g) { release(g); }

}  // extern "C"
