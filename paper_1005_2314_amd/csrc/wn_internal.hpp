// Internal interface between the C ABI (wn_api.cpp) and the gfx950 kernels
// (wn_device.hpp, wn_launch_*.hip).  Not installed; plain structs only.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wn {

// Per-stream header in device memory, 64 bytes (one per stream, packed: a
// 128-byte stride measured 3% slower on the batched workload).  The pool
// itself lives in the state arena at byte offset pool_off, in natural element
// order.
struct StreamHdr {
  uint64_t xs;        // xorshift64 state
  uint64_t k;         // pools produced since seeding
  double f;           // scale factor of the current pool
  double xnext;       // withheld scaled value for the next chi-square sample
  double qlast;       // binary64 sum of squares of the current pool
  uint64_t pool_off;  // byte offset of the pool in the arena
  uint32_t n;         // pool size
  uint16_t cursor;    // next pool position to emit; n-1 = used up (n <= 16384)
  uint16_t sflags;    // statistics state of the current pool: kSeenByStats, kHeldExtreme
  double tprev;       // centred emitted sum of squares of the current pool (statistics)
};
static_assert(sizeof(StreamHdr) == 64, "header must stay 64 bytes");

// StreamHdr::sflags.  A statistics call pairs a new pool with its predecessor
// only when that predecessor was produced by a statistics call too (a plain
// fill that produces a pool clears the flags).
enum : uint16_t { kHeldExtreme = 1, kSeenByStats = 2 };

// Chi-square constants for one pool size (computed on the host).
struct Chi2Consts {
  double nu, A, b, fisher_root, wh_c, wh_shift;
};

// One unit of work: a stream, how many values it emits, where they go.
struct WorkItem {
  uint32_t stream;
  uint32_t req;      // index of the request (statistics partials are kept per request)
  uint64_t count;
  uint64_t out_off;  // element offset in the output
};

// Statistics of one request (fused statistics); reduced in request order.
struct StatsPartial {
  double moment[4];  // sums of y, y^2, y^3, y^4
  double t_sum, t_sumsq, t_lag;
  uint64_t count, pools, t_pairs;
  uint64_t x_pools, x_pairs;  // pools with an extreme value; successive pairs of them
};
static_assert(sizeof(StatsPartial) == 96, "partial layout");

constexpr uint32_t kHistBins = 4096;  // floor(256 y) + 2048 for y in [-8, 8)

// Device layout of wn_stats (include/wn.h).
struct StatsOut {
  uint64_t count;
  double moment[4];
  uint64_t below, above;
  uint64_t pools;
  double t_sum, t_sumsq;
  uint64_t t_pairs;
  double t_lag;
  uint64_t hist[kHistBins];
  uint64_t x_pools, x_pairs;
};

enum : uint32_t { kChi2Cubic = 0, kChi2Off = 1, kChi2Fisher = 2, kChi2WH = 3 };
enum : uint32_t { kOutF64 = 0, kOutF32 = 1, kOutBF16 = 2, kOutF16 = 3 };

constexpr int kNumSizes = 11;  // pool sizes 2^4 .. 2^14

struct KernelCommon {
  StreamHdr *hdr;
  unsigned char *arena;
  uint32_t *err;  // device fault word (bit 0: non-finite or zero sum of squares)
  uint32_t n;     // pool size of every item of a one-size launch (0 for mixed sizes)
  uint32_t R;     // passes per emitted pool
  uint32_t K;     // renormalisation period (0 = never)
  uint32_t chi2;  // chi-square mode
  uint32_t x_current;  // chi-square deviate from the current pool's last value (control)
  uint32_t has_mu;     // add mu to every output
  uint32_t transform;  // 0: the 4x4 family A1 D_k; 1: plane rotations
  uint32_t unit_sigma; // 1 when sigma == 1 (the scale is T(f) itself)
  uint32_t stride;     // thinning: every stride-th value of the underlying sequence (1 = all)
  uint32_t expo;       // 1: exponential variates, (a^2 + b^2)/2 of paired rows, n/2 - 1 per pool
  double sigma;        // folded into the scale: T(f * sigma)
  double mu;
  Chi2Consts cc[kNumSizes];  // per pool size, index log2(n) - 4
  double xthr[kNumSizes];    // extreme-value threshold per pool size (statistics)
};

struct SeedArgs {
  KernelCommon c;
  const uint32_t *streams;  // stream ids of this launch (all of pool size c.n)
  uint32_t nstreams;
  uint32_t warmup;  // warm-up passes
  uint64_t seed;
};

// Entry words of a persistent launch with pairs of items: the item index in
// the low 28 bits, the kind above: one item per workgroup, or a pair (items i,
// i+1, one per half of 128 threads).
constexpr uint32_t kEntryKindShift = 28;
constexpr uint32_t kEntryIndex = (1u << kEntryKindShift) - 1;
constexpr uint32_t kEntrySolo = 0, kEntryPair = 1;

struct FillArgs {
  KernelCommon c;
  const WorkItem *items = nullptr;  // device array, or null for the affine form below
  uint32_t nitems = 0;
  uint32_t affine_s0 = 0;           // affine form: item j = (s0 + j, count_each, j * count_each)
  uint64_t count_each = 0;
  uint32_t items_per_wg = 1;        // one-size launches: consecutive items per workgroup
  void *out = nullptr;
  uint32_t variant = 0;             // non-semantic kernel variant (wn_tuning)
  uint32_t *counter = nullptr;      // persistent form: next work item (reset by the launch)
  const uint32_t *entries = nullptr; // persistent form with groups: entry words (kEntry*)
  uint32_t prio_items = 0;          // persistent form: items [0, prio_items) run at priority 3
  uint32_t defer = 0;               // 1: the deferred form where it applies (latency-bound)
  StatsPartial *partials = nullptr; // fused statistics: one partial per request, or null
  StatsOut *stats = nullptr;        // fused statistics: histogram and tails accumulate here
};

// Launch-variant bit (FillArgs::variant) for 128 threads per stream in
// one-size launches of pools of 1024 and 2048 values (wn_tuning.threads_per_stream).
constexpr uint32_t kVariantThreads128 = 16u;

// The message wn_last_error() returns to the calling thread (wn_api.cpp).
void set_last_error(const char *msg);

// Enum fields and arguments come from C callers, who may pass any integer:
// validation reads their object representation as an integer (loading an
// out-of-range value as the C++ enum type is undefined behaviour).
template <typename E>
inline uint32_t enum_bits(const E &e) {
  static_assert(sizeof(E) == sizeof(uint32_t), "4-byte enums");
  uint32_t v;
  __builtin_memcpy(&v, &e, sizeof v);
  return v;
}

// wn_fill_stats_noalloc: the statically allocated partials (wn_noalloc.hip).
// noalloc_partials returns their device address on `device`, which must be the
// current device; the first call on a device looks it up.
constexpr uint32_t kNoAllocRequests = 1u << 16;  // WN_NOALLOC_MAX_REQUESTS
constexpr int kMaxDevices = 64;
hipError_t noalloc_partials(int device, StatsPartial **out);

// Fused statistics: zero `out` before a fill, and fold the request partials
// into it (binary64 sums in a fixed order) after the fill.
hipError_t stats_zero(StatsOut *out, hipStream_t s);
hipError_t zero_words(void *p, uint32_t nwords, hipStream_t s);  // a kernel, not a memset
hipError_t stats_reduce(const StatsPartial *partials, uint32_t nreq, StatsOut *out,
                        hipStream_t s);

// Launchers, one translation unit per pool type and output type
// (wn_launch_<pool>_<out>.hip, instances of wn_launch.hpp).  Return hipSuccess
// or the launch error.  The persistent launchers run items of pool sizes
// 1024..max_n (mixed) on `grid` workgroups (0 = as many as can be resident).
hipError_t seed_f32(const SeedArgs &a, hipStream_t s);
hipError_t seed_f64(const SeedArgs &a, hipStream_t s);
#define WN_DECLARE_LAUNCH_UNIT(P, Q)                                              \
  hipError_t fill_##P##_##Q(const FillArgs &a, hipStream_t s);                   \
  hipError_t persistent_##P##_##Q(const FillArgs &a, uint32_t max_n, uint32_t grid, \
                                  hipStream_t s);
WN_DECLARE_LAUNCH_UNIT(f32, f32)
WN_DECLARE_LAUNCH_UNIT(f32, bf16)
WN_DECLARE_LAUNCH_UNIT(f32, f16)
WN_DECLARE_LAUNCH_UNIT(f64, f64)
WN_DECLARE_LAUNCH_UNIT(f64, f32)
WN_DECLARE_LAUNCH_UNIT(f64, bf16)
WN_DECLARE_LAUNCH_UNIT(f64, f16)
#undef WN_DECLARE_LAUNCH_UNIT

inline hipError_t launch_seed(const SeedArgs &a, bool pool_f64, hipStream_t s) {
  return pool_f64 ? seed_f64(a, s) : seed_f32(a, s);
}
inline hipError_t launch_fill(const FillArgs &a, bool pool_f64, uint32_t out_dtype,
                              hipStream_t s) {
  if (pool_f64) {
    switch (out_dtype) {
      case kOutF64: return fill_f64_f64(a, s);
      case kOutF32: return fill_f64_f32(a, s);
      case kOutBF16: return fill_f64_bf16(a, s);
      case kOutF16: return fill_f64_f16(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (out_dtype) {
    case kOutF32: return fill_f32_f32(a, s);
    case kOutBF16: return fill_f32_bf16(a, s);
    case kOutF16: return fill_f32_f16(a, s);
    default: return hipErrorInvalidValue;
  }
}
inline hipError_t launch_fill_persistent(const FillArgs &a, bool pool_f64, uint32_t out_dtype,
                                         uint32_t max_n, uint32_t grid, hipStream_t s) {
  if (pool_f64) {
    switch (out_dtype) {
      case kOutF64: return persistent_f64_f64(a, max_n, grid, s);
      case kOutF32: return persistent_f64_f32(a, max_n, grid, s);
      case kOutBF16: return persistent_f64_bf16(a, max_n, grid, s);
      case kOutF16: return persistent_f64_f16(a, max_n, grid, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (out_dtype) {
    case kOutF32: return persistent_f32_f32(a, max_n, grid, s);
    case kOutBF16: return persistent_f32_bf16(a, max_n, grid, s);
    case kOutF16: return persistent_f32_f16(a, max_n, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wn
