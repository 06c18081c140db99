// Launchers for binary64 pools: template instances of the kernels in
// wn_device.hpp for every supported pool size, output type and launch variant.

#include "wn_device.hpp"

namespace wn {
namespace {

using T = double;

size_t lds_bytes(uint32_t n, bool db, bool stats = false) {
  return lds_bytes_for<T>(n, db, stats);
}

template <typename Kern>
hipError_t prepare(Kern kern, size_t lds) {
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  return hipSuccess;
}

template <int NQ, bool SMALL, bool ROT = false>
hipError_t seed_t(const SeedArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes(a.c.n, false);
  auto kern = k_seed<T, NQ, SMALL, ROT>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : kBlock;
  hipLaunchKernelGGL(kern, dim3(a.nstreams), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <typename O, int NQ, bool SMALL, bool DB, bool NT, int WPE = 1, bool STATS = false,
          bool ROT = false>
hipError_t fill_t(const FillArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes(a.c.n, DB, STATS);
  auto kern = k_fill<T, O, NQ, SMALL, DB, NT, WPE, STATS, ROT>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : kBlock;
  const uint32_t per = a.items_per_wg ? a.items_per_wg : 1;
  hipLaunchKernelGGL(kern, dim3((a.nitems + per - 1) / per), dim3(block), lds, st, a);
  return hipGetLastError();
}

// Non-semantic variants (identical results): bit 0 double-buffered LDS,
// bit 1 nontemporal output stores, bit 2 at most 64 VGPRs (8 waves per SIMD).
template <typename O, int NQ>
hipError_t fill_v(const FillArgs &a, hipStream_t st) {
  if (a.c.transform) {  // plane rotations: one launch variant, tuning choices ignored
    constexpr bool db = false;
    if (a.partials) return fill_t<O, NQ, false, db, false, 1, true, true>(a, st);
    return fill_t<O, NQ, false, db, false, 1, false, true>(a, st);
  }
  if (a.partials) return fill_t<O, NQ, false, false, false, 1, true>(a, st);
  return fill_t<O, NQ, false, false, false>(a, st);
}

template <typename O, int MAXNQ, bool DB, bool NT, bool STATS = false, bool ROT = false>
hipError_t persistent_t(const FillArgs &a, uint32_t grid, hipStream_t st) {
  const size_t lds = lds_bytes(1024u * MAXNQ, DB, STATS);
  auto kern = k_fill_persistent<T, O, MAXNQ, DB, NT, STATS, ROT>;
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
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, a.counter);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, st, a);
  return hipGetLastError();
}

template <typename O, int MAXNQ>
hipError_t persistent_v(const FillArgs &a, uint32_t grid, hipStream_t st) {
  if (a.c.transform) {
    if (a.partials) return persistent_t<O, MAXNQ, false, false, true, true>(a, grid, st);
    return persistent_t<O, MAXNQ, false, false, false, true>(a, grid, st);
  }
  if (a.partials) return persistent_t<O, MAXNQ, false, false, true>(a, grid, st);
  // two buffers only where they fit in the 160 KiB of LDS
  if constexpr (lds_bytes_for<T>(1024 * MAXNQ, true, false) <= kMaxLds)
    if (a.variant & 1u) return persistent_t<O, MAXNQ, true, false>(a, grid, st);
  return persistent_t<O, MAXNQ, false, false>(a, grid, st);
}

template <typename O>
hipError_t persistent_n(const FillArgs &a, uint32_t max_n, uint32_t grid, hipStream_t st) {
  if (max_n <= 4096) return persistent_v<O, 4>(a, grid, st);
  return persistent_v<O, 16>(a, grid, st);
}

template <bool ROT>
hipError_t seed_r(const SeedArgs &a, hipStream_t st) {
  switch (a.c.n) {
    case 1024: return seed_t<1, false, ROT>(a, st);
    case 2048: return seed_t<2, false, ROT>(a, st);
    case 4096: return seed_t<4, false, ROT>(a, st);
    case 8192: return seed_t<8, false, ROT>(a, st);
    case 16384: return seed_t<16, false, ROT>(a, st);
    default: return seed_t<1, true, ROT>(a, st);
  }
}

hipError_t seed_n(const SeedArgs &a, hipStream_t st) {
  return a.c.transform ? seed_r<true>(a, st) : seed_r<false>(a, st);
}

template <typename O>
hipError_t fill_n(const FillArgs &a, hipStream_t st) {
  switch (a.c.n) {
    case 1024: return fill_v<O, 1>(a, st);
    case 2048: return fill_v<O, 2>(a, st);
    case 4096: return fill_v<O, 4>(a, st);
    case 8192: return fill_v<O, 8>(a, st);
    case 16384: return fill_v<O, 16>(a, st);
    default:
      if (a.c.transform) {
        if (a.partials) return fill_t<O, 1, true, false, false, 1, true, true>(a, st);
        return fill_t<O, 1, true, false, false, 1, false, true>(a, st);
      }
      if (a.partials) return fill_t<O, 1, true, false, false, 1, true>(a, st);
      return fill_t<O, 1, true, false, false>(a, st);
  }
}

}  // namespace

hipError_t f64_seed(const SeedArgs &a, hipStream_t s) {
  if (a.nstreams == 0) return hipSuccess;
  return seed_n(a, s);
}

hipError_t f64_fill(const FillArgs &a, uint32_t out_dtype, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  switch (out_dtype) {
    case kOutF64: return fill_n<double>(a, s);
    case kOutF32: return fill_n<float>(a, s);
    case kOutBF16: return fill_n<Bf16>(a, s);
    default: return fill_n<Half>(a, s);
  }
}

hipError_t f64_fill_persistent(const FillArgs &a, uint32_t out_dtype, uint32_t max_n,
                                  uint32_t grid, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  switch (out_dtype) {
    case kOutF64: return persistent_n<double>(a, max_n, grid, s);
    case kOutF32: return persistent_n<float>(a, max_n, grid, s);
    case kOutBF16: return persistent_n<Bf16>(a, max_n, grid, s);
    default: return persistent_n<Half>(a, max_n, grid, s);
  }
}

}  // namespace wn
