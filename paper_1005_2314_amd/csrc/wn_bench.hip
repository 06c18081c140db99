// Measurement kernels (include/wn_bench.h): HBM write ceiling, the
// generator's traffic without arithmetic, and a Box-Muller comparator.

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "wn_bench.h"
#include "wn_internal.hpp"

namespace {

constexpr uint32_t kBlock = 256;

wn_status launch_status(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return WN_OK;
  (void)what;
  return WN_EDEVICE;
}

int grid_for(uint64_t work_items) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint64_t want = (work_items + kBlock - 1) / kBlock;
  const uint64_t cap = uint64_t(cus) * 32;
  return int(want < cap ? (want ? want : 1) : cap);
}

// ---- pure stores ----------------------------------------------------------------
template <int W, bool NT>
__global__ __launch_bounds__(kBlock) void k_store(uint32_t *__restrict__ dst, uint64_t nvec) {
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < nvec; i += stride) {
    if constexpr (W == 4) {
      uint4 *p = reinterpret_cast<uint4 *>(dst) + i;
      if constexpr (NT) {
        __builtin_nontemporal_store(0u, &p->x);
        __builtin_nontemporal_store(0u, &p->y);
        __builtin_nontemporal_store(0u, &p->z);
        __builtin_nontemporal_store(0u, &p->w);
      } else {
        *p = make_uint4(0u, 0u, 0u, 0u);
      }
    } else {
      if constexpr (NT)
        __builtin_nontemporal_store(0u, dst + i);
      else
        dst[i] = 0u;
    }
  }
}

// Pure stores in runs: a persistent grid in which workgroup b writes runs
// b, b + grid, ... of `run` consecutive words (dword stores, one word per lane
// per instruction), the last run cut at nwords.
__global__ __launch_bounds__(kBlock) void k_store_runs(uint32_t *__restrict__ dst, uint64_t nwords,
                                                       uint32_t run) {
  const uint64_t nruns = (nwords + run - 1) / run;
  for (uint64_t j = blockIdx.x; j < nruns; j += gridDim.x) {
    const uint64_t lo = j * run;
    const uint64_t hi = lo + run < nwords ? lo + run : nwords;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) dst[i] = 0u;
  }
}

// ---- the fill's traffic, no arithmetic ------------------------------------------
// A plain streaming copy of one fill's bytes: work item j (one workgroup)
// reads its pool (n binary32) and 64-byte header at state + j (4n + 64),
// writes per_stream binary32 values to out + j per_stream as consecutive
// coalesced words (each wave 64 words per instruction), and writes the pool
// and header back.  The same bytes as the generator's fill of that request,
// in the simplest order: the practical ceiling of the fill on this traffic.
template <int NQ>
__global__ __launch_bounds__(kBlock) void k_traffic(unsigned char *__restrict__ state,
                                                    float *__restrict__ out, uint32_t n,
                                                    uint64_t per_stream) {
  const uint32_t j = blockIdx.x;
  const uint32_t tid = threadIdx.x;
  float *pool = reinterpret_cast<float *>(state + size_t(j) * (size_t(n) * 4 + 64));
  uint4 *hdr = reinterpret_cast<uint4 *>(state + size_t(j) * (size_t(n) * 4 + 64) + size_t(n) * 4);
  float y[4 * NQ];
#pragma unroll
  for (int k = 0; k < 4 * NQ; ++k) y[k] = pool[k * kBlock + tid];
  uint4 h = make_uint4(0, 0, 0, 0);
  if (tid < 4) h = hdr[tid];
  float *o = out + size_t(j) * per_stream;
  // the values written are the pool's, repeated
  const uint64_t chunk = uint64_t(4 * NQ) * kBlock;
  for (uint64_t b = 0; b < per_stream; b += chunk) {
#pragma unroll
    for (int k = 0; k < 4 * NQ; ++k) {
      const uint64_t i = b + uint64_t(k) * kBlock + tid;
      if (i < per_stream) o[i] = y[k];
    }
  }
  // the empty asm keeps the compiler from dropping the write-back of values
  // it has just loaded from the same addresses
#pragma unroll
  for (int k2 = 0; k2 < 4 * NQ; ++k2) {
    asm volatile("" : "+v"(y[k2]));
    pool[k2 * kBlock + tid] = y[k2];
  }
  if (tid < 4) {
    asm volatile("" : "+v"(h.x), "+v"(h.y), "+v"(h.z), "+v"(h.w));
    hdr[tid] = h;
  }
}

// ---- Box-Muller over Philox4x32-10 ------------------------------------------------
// Philox4x32 round: two 32x32->64 products of the multipliers with counter words
// 0 and 2, xored with words 1 and 3 and the key; the key is bumped by the Weyl
// constants between rounds (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k.x += W0;
      k.y += W1;
    }
    const uint32_t lo0 = M0 * c.x, hi0 = __umulhi(M0, c.x);
    const uint32_t lo1 = M1 * c.z, hi1 = __umulhi(M1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

template <typename O, bool FAST>
__global__ __launch_bounds__(kBlock) void k_box_muller(O *__restrict__ out, uint64_t nquads,
                                                       uint2 key) {
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < nquads; i += stride) {
    const uint4 x = philox4x32_10(make_uint4(uint32_t(i), uint32_t(i >> 32), 0u, 0u), key);
    O z[4];
    if constexpr (sizeof(O) == 8) {
      const double s = 0x1p-32;
      const double u0 = (double(x.x) + 0.5) * s, u1 = (double(x.y) + 0.5) * s;
      const double u2 = (double(x.z) + 0.5) * s, u3 = (double(x.w) + 0.5) * s;
      const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
      double s0, c0, s1, c1;
      sincospi(2.0 * u1, &s0, &c0);
      sincospi(2.0 * u3, &s1, &c1);
      z[0] = r0 * c0;
      z[1] = r0 * s0;
      z[2] = r1 * c1;
      z[3] = r1 * s1;
    } else {
      const float s = 0x1p-32f;
      const float u0 = (float(x.x) + 0.5f) * s, u1 = (float(x.y) + 0.5f) * s;
      const float u2 = (float(x.z) + 0.5f) * s, u3 = (float(x.w) + 0.5f) * s;
      float r0, r1, s0, c0, s1, c1;
      if constexpr (FAST) {
        r0 = __fsqrt_rn(-2.0f * __logf(u0));
        r1 = __fsqrt_rn(-2.0f * __logf(u2));
        __sincosf(6.2831853071795865f * u1, &s0, &c0);
        __sincosf(6.2831853071795865f * u3, &s1, &c1);
      } else {
        r0 = sqrtf(-2.0f * logf(u0));
        r1 = sqrtf(-2.0f * logf(u2));
        sincospif(2.0f * u1, &s0, &c0);
        sincospif(2.0f * u3, &s1, &c1);
      }
      z[0] = r0 * c0;
      z[1] = r0 * s0;
      z[2] = r1 * c1;
      z[3] = r1 * s1;
    }
    if constexpr (sizeof(O) == 8) {
      double2 *o = reinterpret_cast<double2 *>(out + 4 * i);
      o[0] = make_double2(z[0], z[1]);
      o[1] = make_double2(z[2], z[3]);
    } else {
      reinterpret_cast<float4 *>(out)[i] = make_float4(z[0], z[1], z[2], z[3]);
    }
  }
}

}  // namespace

extern "C" {

wn_status wn_bench_store(void *dst, uint64_t bytes, uint32_t width_dwords, void *hip_stream) {
  const bool nt = (width_dwords & 0x100u) != 0;
  const bool runs = (width_dwords & 0x200u) != 0;
  width_dwords &= 0xFFu;
  if (!dst || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0 ||
      (width_dwords != 1 && width_dwords != 4) || (runs && (nt || width_dwords != 1)))
    return WN_EINVAL;
  if (runs) {
    (void)hipGetLastError();  // an earlier call's error is not this launch's
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipLaunchKernelGGL(k_store_runs, dim3(uint32_t(cus) * 4), dim3(kBlock), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<uint32_t *>(dst),
                       bytes / 4, 65536u);
    return launch_status("wn_bench_store");
  }
  (void)hipGetLastError();  // an earlier call's error is not this launch's
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const uint64_t nvec = bytes / (4 * width_dwords);
  const int grid = grid_for(nvec / 4);
  auto *d = static_cast<uint32_t *>(dst);
  if (width_dwords == 4 && nt)
    hipLaunchKernelGGL((k_store<4, true>), dim3(grid), dim3(kBlock), 0, st, d, nvec);
  else if (width_dwords == 4)
    hipLaunchKernelGGL((k_store<4, false>), dim3(grid), dim3(kBlock), 0, st, d, nvec);
  else if (nt)
    hipLaunchKernelGGL((k_store<1, true>), dim3(grid), dim3(kBlock), 0, st, d, nvec);
  else
    hipLaunchKernelGGL((k_store<1, false>), dim3(grid), dim3(kBlock), 0, st, d, nvec);
  return launch_status("wn_bench_store");
}

wn_status wn_bench_traffic(void *state, void *out, uint32_t num_streams, uint32_t pool_n,
                           uint64_t per_stream, void *hip_stream) {
  if (!state || !out || num_streams == 0) return WN_EINVAL;
  (void)hipGetLastError();  // an earlier call's error is not this launch's
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  auto *s = static_cast<unsigned char *>(state);
  auto *o = static_cast<float *>(out);
  switch (pool_n) {
    case 1024: hipLaunchKernelGGL(k_traffic<1>, dim3(num_streams), dim3(kBlock), 0, st, s, o, pool_n, per_stream); break;
    case 2048: hipLaunchKernelGGL(k_traffic<2>, dim3(num_streams), dim3(kBlock), 0, st, s, o, pool_n, per_stream); break;
    case 4096: hipLaunchKernelGGL(k_traffic<4>, dim3(num_streams), dim3(kBlock), 0, st, s, o, pool_n, per_stream); break;
    case 8192: hipLaunchKernelGGL(k_traffic<8>, dim3(num_streams), dim3(kBlock), 0, st, s, o, pool_n, per_stream); break;
    case 16384: hipLaunchKernelGGL(k_traffic<16>, dim3(num_streams), dim3(kBlock), 0, st, s, o, pool_n, per_stream); break;
    default: return WN_EINVAL;
  }
  return launch_status("wn_bench_traffic");
}

wn_status wn_bench_box_muller(void *out, uint64_t count, wn_dtype out_dtype, uint64_t seed,
                              int fast, void *hip_stream) {
  if (!out || count % 4 != 0 || reinterpret_cast<uintptr_t>(out) % 16 != 0) return WN_EINVAL;
  const uint32_t od = wn::enum_bits(out_dtype);
  if (od != WN_F32 && od != WN_F64) return WN_EINVAL;
  if (od == WN_F64 && fast) return WN_EINVAL;
  (void)hipGetLastError();  // an earlier call's error is not this launch's
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const uint64_t nquads = count / 4;
  const uint2 key = make_uint2(uint32_t(seed), uint32_t(seed >> 32));
  const int grid = grid_for(nquads);
  if (out_dtype == WN_F64)
    hipLaunchKernelGGL((k_box_muller<double, false>), dim3(grid), dim3(kBlock), 0, st,
                       static_cast<double *>(out), nquads, key);
  else if (fast)
    hipLaunchKernelGGL((k_box_muller<float, true>), dim3(grid), dim3(kBlock), 0, st,
                       static_cast<float *>(out), nquads, key);
  else
    hipLaunchKernelGGL((k_box_muller<float, false>), dim3(grid), dim3(kBlock), 0, st,
                       static_cast<float *>(out), nquads, key);
  return launch_status("wn_bench_box_muller");
}

}  // extern "C"
