// Launch helpers for the kernels of wn_device.hpp, templated on the pool type
// T and the output type O.  Each launch unit wn_launch_<pool>_<out>.hip
// instantiates them for one (T, O) pair, so that the units compile in
// parallel; every supported pool size and launch variant of that pair lives
// in its unit.
#pragma once

#include <type_traits>

#include "wn_device.hpp"

namespace wn {
namespace {

template <typename T>
constexpr bool kPoolF32 = std::is_same_v<T, float>;

// Before a launch: discard an error an earlier runtime call left behind (a
// failed allocation is reported by the next hipGetLastError, which would
// otherwise be taken for this launch's status), then allow the LDS size.
template <typename Kern>
hipError_t prepare(Kern kern, size_t lds) {
  (void)hipGetLastError();
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  return hipSuccess;
}

// ---- seeding ----------------------------------------------------------------------------
template <typename T, int NQ, bool SMALL, bool ROT>
hipError_t seed_t(const SeedArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes_for<T>(a.c.n, false, false);
  auto kern = k_seed<T, NQ, SMALL, ROT>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : kBlock;
  hipLaunchKernelGGL(kern, dim3(a.nstreams), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <typename T, bool ROT>
hipError_t seed_r(const SeedArgs &a, hipStream_t st) {
  switch (a.c.n) {
    case 1024: return seed_t<T, 1, false, ROT>(a, st);
    case 2048: return seed_t<T, 2, false, ROT>(a, st);
    case 4096: return seed_t<T, 4, false, ROT>(a, st);
    case 8192: return seed_t<T, 8, false, ROT>(a, st);
    case 16384: return seed_t<T, 16, false, ROT>(a, st);
    default: return seed_t<T, 1, true, ROT>(a, st);
  }
}

template <typename T>
hipError_t seed_n(const SeedArgs &a, hipStream_t st) {
  if (a.nstreams == 0) return hipSuccess;
  return a.c.transform ? seed_r<T, true>(a, st) : seed_r<T, false>(a, st);
}

// ---- one-size launches --------------------------------------------------------------------
template <typename T, typename O, int NQ, bool SMALL, bool DB, bool NT, int WPE = 1,
          bool STATS = false, bool ROT = false, int BDK = int(kBlock)>
hipError_t fill_t(const FillArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes_for<T>(BDK == 128 ? layout_n_128(a.c.n) : a.c.n, DB, STATS);
  auto kern = k_fill<T, O, NQ, SMALL, DB, NT, WPE, STATS, ROT, BDK>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : uint32_t(BDK);
  const uint32_t per = a.items_per_wg ? a.items_per_wg : 1;
  hipLaunchKernelGGL(kern, dim3((a.nitems + per - 1) / per), dim3(block), lds, st, a);
  return hipGetLastError();
}

// Non-semantic variants (identical results).  Binary32 pools of up to 8192
// values: bit 0 double-buffered LDS, bit 1 nontemporal output stores (with
// bit 0), bits 2-3 a register cap for 8, 6 or 5 waves per SIMD.  Binary64
// pools and the plane-rotation family run one variant.  Bit 4: pools of 1024
// to 4096 values without statistics, rotations, thinning or exponential
// variates run on 128 threads per stream (with bit 0 as above; the other bits
// do not apply).
template <typename T, typename O, int NQ>
hipError_t fill_v(const FillArgs &a, hipStream_t st) {
  constexpr bool db_fits = kPoolF32<T> && NQ <= 8;
  if constexpr (NQ <= 4) {
    if ((a.variant & kVariantThreads128) && !a.c.transform && !a.partials && a.c.stride == 1 &&
        !a.c.expo) {
      if (db_fits && (a.variant & 1u))
        return fill_t<T, O, 2 * NQ, false, db_fits, false, 1, false, false, 128>(a, st);
      return fill_t<T, O, 2 * NQ, false, false, false, 1, false, false, 128>(a, st);
    }
  }
  if (a.c.transform) {
    if (a.partials) return fill_t<T, O, NQ, false, db_fits, false, 1, true, true>(a, st);
    return fill_t<T, O, NQ, false, db_fits, false, 1, false, true>(a, st);
  }
  if (a.partials) {  // statistics: one LDS buffer unless bit 0 asks for two
    if constexpr (db_fits)
      if (a.variant & 1u) return fill_t<T, O, NQ, false, true, false, 1, true>(a, st);
    return fill_t<T, O, NQ, false, false, false, 4, true>(a, st);
  }
  if constexpr (db_fits) {
    const bool db = a.variant & 1u;
    switch ((a.variant >> 2) & 3u) {  // waves-per-SIMD cap: none, 8, 6, 5
      case 1: return db ? fill_t<T, O, NQ, false, true, false, 8>(a, st)
                        : fill_t<T, O, NQ, false, false, false, 8>(a, st);
      case 2: return db ? fill_t<T, O, NQ, false, true, false, 6>(a, st)
                        : fill_t<T, O, NQ, false, false, false, 6>(a, st);
      case 3: return db ? fill_t<T, O, NQ, false, true, false, 5>(a, st)
                        : fill_t<T, O, NQ, false, false, false, 5>(a, st);
      default: break;
    }
    if (a.variant & 2u) return fill_t<T, O, NQ, false, true, true>(a, st);
    if (db) return fill_t<T, O, NQ, false, true, false>(a, st);
  }
  return fill_t<T, O, NQ, false, false, false>(a, st);
}

// The deferred form (each pool's scale and emission inside the next pool's
// first pass), without statistics or thinning: one-size launches of pools of
// 1024 or 2048 values (at 4096 the copy of the finished pool costs more than
// the overlap saves), and persistent launches whose pools are at most 4096
// (items of 4096 there keep the plain loop).
inline bool defer_applies(const FillArgs &a, uint32_t max_n, uint32_t limit) {
  return a.defer && !a.partials && a.c.stride == 1 && !a.c.expo && max_n >= 1024 &&
         max_n <= limit;
}

template <typename T, typename O, int NQ, bool ROT>
hipError_t defer_t(const FillArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes_for<T>(a.c.n, true, false);
  auto kern = k_fill_defer<T, O, NQ, ROT>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(a.nitems), dim3(kBlock), lds, st, a);
  return hipGetLastError();
}

template <typename T, typename O, bool ROT>
hipError_t defer_n(const FillArgs &a, hipStream_t st) {
  return a.c.n == 1024 ? defer_t<T, O, 1, ROT>(a, st) : defer_t<T, O, 2, ROT>(a, st);
}

template <typename T, typename O>
hipError_t fill_n(const FillArgs &a, hipStream_t st) {
  if (a.nitems == 0) return hipSuccess;
  if (defer_applies(a, a.c.n, 2048))
    return a.c.transform ? defer_n<T, O, true>(a, st) : defer_n<T, O, false>(a, st);
  switch (a.c.n) {
    case 1024: return fill_v<T, O, 1>(a, st);
    case 2048: return fill_v<T, O, 2>(a, st);
    case 4096: return fill_v<T, O, 4>(a, st);
    case 8192: return fill_v<T, O, 8>(a, st);
    case 16384: return fill_v<T, O, 16>(a, st);
    default:
      if (a.c.transform) {
        if (a.partials) return fill_t<T, O, 1, true, false, false, 1, true, true>(a, st);
        return fill_t<T, O, 1, true, false, false, 1, false, true>(a, st);
      }
      if (a.partials) return fill_t<T, O, 1, true, false, false, 1, true>(a, st);
      return fill_t<T, O, 1, true, false, false>(a, st);
  }
}

// ---- persistent launches -----------------------------------------------------------------
// Items of pool sizes 1024..max_n (mixed), `grid` workgroups (0 = as many as
// can be resident); resets a.counter first (a kernel, not a memset, so that
// the two launches can be captured in a graph).
template <typename T, typename O, int MAXNQ, bool DB, bool NT, bool STATS = false,
          bool ROT = false, bool DEFER = false, bool PAIRS = false>
hipError_t persistent_t(const FillArgs &a, uint32_t grid, hipStream_t st) {
  const size_t lds = lds_bytes_for<T>(1024u * MAXNQ, DB, STATS);
  auto kern = k_fill_persistent<T, O, MAXNQ, DB, NT, STATS, ROT, DEFER, PAIRS>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  if (grid == 0) {  // as many workgroups as can be resident at once
    int per_cu = 0, dev = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds)) !=
            hipSuccess ||
        (e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
            hipSuccess)
      return e;
    grid = uint32_t(cus) * uint32_t(per_cu > 0 ? per_cu : 1);
  }
  (void)hipGetLastError();  // prepare() and the occupancy query may leave one
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, a.counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, st, a);
  return hipGetLastError();
}

// 128 threads per item (variant bit kVariantThreads128), pools of 1024 and 2048.
template <typename T, typename O, bool DB, bool NT>
hipError_t persistent128_t(const FillArgs &a, uint32_t grid, hipStream_t st) {
  const size_t lds = lds_bytes_for<T>(2048, DB, false);
  auto kern = k_fill_persistent128<T, O, DB, NT>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  if (grid == 0) {  // as many workgroups as can be resident at once
    int per_cu = 0, dev = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 128, lds)) !=
            hipSuccess ||
        (e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) !=
            hipSuccess)
      return e;
    grid = uint32_t(cus) * uint32_t(per_cu > 0 ? per_cu : 1);
  }
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, a.counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(128), lds, st, a);
  return hipGetLastError();
}

// Binary32 pools: bit 0 double-buffered LDS, bit 1 nontemporal stores (with
// two buffers).  Binary64 pools: two buffers only where they fit in LDS.
template <typename T, typename O, int MAXNQ>
hipError_t persistent_v(const FillArgs &a, uint32_t grid, hipStream_t st) {
  if constexpr (kPoolF32<T>) {
    static_assert(lds_bytes_for<T>(1024 * MAXNQ, true, true) <= kMaxLds,
                  "two binary32 pool buffers and the statistics fit in LDS");
    if (a.c.transform) {
      if (a.partials) return persistent_t<T, O, MAXNQ, true, false, true, true>(a, grid, st);
      return persistent_t<T, O, MAXNQ, true, false, false, true>(a, grid, st);
    }
    if (a.partials) return persistent_t<T, O, MAXNQ, true, false, true>(a, grid, st);
    switch (a.variant & 3u) {
      case 1: return persistent_t<T, O, MAXNQ, true, false>(a, grid, st);
      case 2:
      case 3: return persistent_t<T, O, MAXNQ, true, true>(a, grid, st);
      default: return persistent_t<T, O, MAXNQ, false, false>(a, grid, st);
    }
  } else {
    if (a.c.transform) {
      if (a.partials) return persistent_t<T, O, MAXNQ, false, false, true, true>(a, grid, st);
      return persistent_t<T, O, MAXNQ, false, false, false, true>(a, grid, st);
    }
    if (a.partials) return persistent_t<T, O, MAXNQ, false, false, true>(a, grid, st);
    if constexpr (lds_bytes_for<T>(1024 * MAXNQ, true, false) <= kMaxLds)
      if (a.variant & 1u) return persistent_t<T, O, MAXNQ, true, false>(a, grid, st);
    return persistent_t<T, O, MAXNQ, false, false>(a, grid, st);
  }
}

template <typename T, typename O>
hipError_t persistent_n(const FillArgs &a, uint32_t max_n, uint32_t grid, hipStream_t st) {
  if (a.nitems == 0) return hipSuccess;
  if (a.entries) {  // pairs of small-pool items (plain loop, A4 passes, pools up to 4096)
    if (a.partials || a.c.transform || a.c.stride != 1 || max_n > 4096)
      return hipErrorInvalidValue;
    if (a.defer)  // the items that run alone take the deferred form (two LDS buffers)
      return persistent_t<T, O, 4, true, false, false, false, true, true>(a, grid, st);
    if (a.variant & 1u)
      return persistent_t<T, O, 4, true, false, false, false, false, true>(a, grid, st);
    return persistent_t<T, O, 4, false, false, false, false, false, true>(a, grid, st);
  }
  if (defer_applies(a, max_n, 4096))  // two LDS buffers of the largest pool fit for both types
    return a.c.transform ? persistent_t<T, O, 4, true, false, false, true, true>(a, grid, st)
                         : persistent_t<T, O, 4, true, false, false, false, true>(a, grid, st);
  if ((a.variant & kVariantThreads128) && max_n <= 2048 && !a.partials && !a.c.transform &&
      a.c.stride == 1 && !a.c.expo) {
    if (kPoolF32<T> && (a.variant & 1u)) return persistent128_t<T, O, kPoolF32<T>, false>(a, grid, st);
    return persistent128_t<T, O, false, false>(a, grid, st);
  }
  if (max_n <= 4096) return persistent_v<T, O, 4>(a, grid, st);
  return persistent_v<T, O, 16>(a, grid, st);
}

}  // namespace
}  // namespace wn

// One launch unit: the exported launchers of pool type T (binary32 or
// binary64, named P) and output type O (named Q).
#define WN_LAUNCH_UNIT(T, P, O, Q)                                                           \
  namespace wn {                                                                             \
  hipError_t fill_##P##_##Q(const FillArgs &a, hipStream_t s) { return fill_n<T, O>(a, s); } \
  hipError_t persistent_##P##_##Q(const FillArgs &a, uint32_t max_n, uint32_t grid,         \
                                  hipStream_t s) {                                           \
    return persistent_n<T, O>(a, max_n, grid, s);                                            \
  }                                                                                          \
  }
