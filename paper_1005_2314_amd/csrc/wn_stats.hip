// Fused statistics, host side of the device work: zeroing the result and the
// final reduction of the per-request partials (wn_fill_stats in wn_api.cpp).

#include <algorithm>

#include "wn_device.hpp"

namespace wn {
namespace {

__global__ __launch_bounds__(kBlock) void k_stats_zero(uint64_t *words, uint32_t nwords) {
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < nwords; i += gridDim.x * kBlock)
    words[i] = 0u;
}

// One workgroup: thread t adds partials t, t+256, t+512, ... in that order,
// then a pairwise tree over the 256 threads (waves, then the 4 waves) gives
// each binary64 total; the integer counts need no order.  The histogram and
// its tails were accumulated by the fill itself.
__global__ __launch_bounds__(kBlock) void k_stats_reduce(const StatsPartial *p, uint32_t nreq,
                                                         StatsOut *out) {
  __shared__ double slots[7][4];
  __shared__ unsigned long long icount[5];
  const uint32_t t = threadIdx.x;
  if (t < 5) icount[t] = 0ull;
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0;
  for (uint32_t j = t; j < nreq; j += kBlock) {
    const StatsPartial &q = p[j];
    acc[0] = __dadd_rn(acc[0], q.moment[0]);
    acc[1] = __dadd_rn(acc[1], q.moment[1]);
    acc[2] = __dadd_rn(acc[2], q.moment[2]);
    acc[3] = __dadd_rn(acc[3], q.moment[3]);
    acc[4] = __dadd_rn(acc[4], q.t_sum);
    acc[5] = __dadd_rn(acc[5], q.t_sumsq);
    acc[6] = __dadd_rn(acc[6], q.t_lag);
    c0 += q.count;
    c1 += q.pools;
    c2 += q.t_pairs;
    c3 += q.x_pools;
    c4 += q.x_pairs;
  }
  __syncthreads();
  atomicAdd(&icount[0], c0);
  atomicAdd(&icount[1], c1);
  atomicAdd(&icount[2], c2);
  atomicAdd(&icount[3], c3);
  atomicAdd(&icount[4], c4);
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    const double w = wave_pairwise_sum(acc[f]);
    if ((t & 63) == 0) slots[f][t >> 6] = w;
  }
  __syncthreads();
  if (t == 0) {
    double tot[7];
#pragma unroll
    for (int f = 0; f < 7; ++f)
      tot[f] = __dadd_rn(__dadd_rn(slots[f][0], slots[f][1]), __dadd_rn(slots[f][2], slots[f][3]));
    out->moment[0] = tot[0];
    out->moment[1] = tot[1];
    out->moment[2] = tot[2];
    out->moment[3] = tot[3];
    out->t_sum = tot[4];
    out->t_sumsq = tot[5];
    out->t_lag = tot[6];
    out->count = icount[0];
    out->pools = icount[1];
    out->t_pairs = icount[2];
    out->x_pools = icount[3];
    out->x_pairs = icount[4];
  }
}

}  // namespace

hipError_t zero_words(void *p, uint32_t nwords, hipStream_t s) {
  const uint32_t grid = std::min<uint32_t>(1024u, (nwords + kBlock - 1) / kBlock + 1);
  (void)hipGetLastError();  // an earlier call's error is not this launch's
  hipLaunchKernelGGL(k_stats_zero, dim3(grid), dim3(kBlock), 0, s, static_cast<uint64_t *>(p),
                     nwords);
  return hipGetLastError();
}

hipError_t stats_zero(StatsOut *out, hipStream_t s) {
  return zero_words(out, uint32_t(sizeof(StatsOut) / 8), s);
}

hipError_t stats_reduce(const StatsPartial *partials, uint32_t nreq, StatsOut *out,
                        hipStream_t s) {
  (void)hipGetLastError();  // an earlier call's error is not this launch's
  hipLaunchKernelGGL(k_stats_reduce, dim3(1), dim3(kBlock), 0, s, partials, nreq, out);
  return hipGetLastError();
}

}  // namespace wn
