// Quality-constrained choice of the semantic parameters (include/wn.h):
// the statistics battery (wn_quality_check) and the choice of pool size n and
// passes per emitted pool R (wn_tune_config).  Section 5.7 names these two as
// the remedies for finite-pool effects: a larger pool, and discarding pools
// (R passes between emitted pools emit one pool in R).  The choice is a
// configuration the caller creates its generator from, so the values always
// follow from a stated configuration.  Host code over the public entry points.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wn.h"
#include "wn_internal.hpp"

namespace {

// report through wn_last_error()
wn_status tune_fail(wn_status s, const char *fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(msg, sizeof(msg), fmt, ap);
  va_end(ap);
  wn::set_last_error(msg);
  return s;
}

bool pool_size_ok(uint32_t n) { return n >= 16 && n <= 16384 && (n & (n - 1)) == 0; }

// Statistics where only one direction is a defect: a histogram that fits the
// normal law worse than chance, and adjacent extreme pools more often than
// independence (clustering).
bool one_sided(int i) { return i == WN_Q_HIST || i == WN_Q_EXTREME_PAIRS; }

// P(Z < x) for a standard normal Z
double normal_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Add the statistics of one call to a running total (host copies).  The lag
// pairs of successive calls chain, so the total is the statistics of the
// calls' concatenated output.
void accumulate(wn_stats &acc, const wn_stats &s) {
  acc.count += s.count;
  for (int k = 0; k < 4; ++k) acc.moment[k] += s.moment[k];
  acc.below += s.below;
  acc.above += s.above;
  acc.pools += s.pools;
  acc.t_sum += s.t_sum;
  acc.t_sumsq += s.t_sumsq;
  acc.t_pairs += s.t_pairs;
  acc.t_lag += s.t_lag;
  for (int b = 0; b < 4096; ++b) acc.hist[b] += s.hist[b];
  acc.x_pools += s.x_pools;
  acc.x_pairs += s.x_pairs;
}

}  // namespace

extern "C" {

wn_status wn_quality_check(const wn_stats *st, uint32_t pool_n, double z_max, wn_quality *q) {
  if (!st || !q) return tune_fail(WN_EINVAL, "wn_quality_check: NULL argument");
  if (!pool_size_ok(pool_n))
    return tune_fail(WN_EINVAL, "wn_quality_check: pool size %u", pool_n);
  if (!(z_max > 0.0)) return tune_fail(WN_EINVAL, "wn_quality_check: z_max must be positive");
  if (st->count < 2 || st->pools < 2)
    return tune_fail(WN_EINVAL, "wn_quality_check: too few values (%llu) or pools (%llu)",
                     (unsigned long long)st->count, (unsigned long long)st->pools);
  std::memset(q, 0, sizeof(*q));
  const double N = double(st->count);
  const double m1 = st->moment[0] / N, m2 = st->moment[1] / N;
  const double m3 = st->moment[2] / N, m4 = st->moment[3] / N;
  const double var = m2 - m1 * m1;
  const double mu3 = m3 - 3.0 * m1 * m2 + 2.0 * m1 * m1 * m1;
  const double mu4 = m4 - 4.0 * m1 * m3 + 6.0 * m1 * m1 * m2 - 3.0 * m1 * m1 * m1 * m1;
  // normal moments and their standard errors for N independent values
  q->z[WN_Q_MEAN] = m1 / std::sqrt(1.0 / N);
  q->z[WN_Q_VAR] = (var - 1.0) / std::sqrt(2.0 / N);
  q->z[WN_Q_SKEW] = (mu3 / std::pow(var, 1.5)) / std::sqrt(6.0 / N);
  q->z[WN_Q_KURT] = (mu4 / (var * var) - 3.0) / std::sqrt(24.0 / N);
  // histogram against the normal law: cells with an expected count of at
  // least 5, the rest (and the two tails) merged into one cell
  {
    double chi2 = 0.0, rest_obs = double(st->below + st->above);
    double rest_exp = N * 2.0 * normal_cdf(-8.0);
    int cells = 0;
    for (int b = 0; b < 4096; ++b) {
      const double lo = (b - 2048) / 256.0, hi = (b - 2047) / 256.0;
      const double e = N * (normal_cdf(hi) - normal_cdf(lo));
      if (e >= 5.0) {
        const double d = double(st->hist[b]) - e;
        chi2 += d * d / e;
        ++cells;
      } else {
        rest_obs += double(st->hist[b]);
        rest_exp += e;
      }
    }
    if (rest_exp > 0.0) {
      const double d = rest_obs - rest_exp;
      chi2 += d * d / rest_exp;
      ++cells;
    }
    const double dof = double(cells - 1);
    q->z[WN_Q_HIST] = (chi2 - dof) / std::sqrt(2.0 * dof);
  }
  // pool sums of the emitted values: chi-square with n - 1 degrees of freedom
  // (mean n - 1, variance 2 (n - 1)); successive pools uncorrelated
  const double P = double(st->pools);
  const double nu = double(pool_n - 1);
  const double tm = st->t_sum / P;
  const double tv = st->t_sumsq / P - tm * tm;
  q->z[WN_Q_POOL_MEAN] = tm / std::sqrt(2.0 * nu / P);
  q->z[WN_Q_POOL_VAR] = (tv / (2.0 * nu) - 1.0) / std::sqrt(2.0 / P);
  if (st->t_pairs > 0 && tv > 0.0) {
    const double corr = (st->t_lag / double(st->t_pairs) - tm * tm) / tv;
    q->z[WN_Q_POOL_LAG] = corr * std::sqrt(double(st->t_pairs));
  }
  // adjacent pools both holding an extreme value (Section 5.7), against
  // independence: t_pairs p^2 expected; overlapping pairs (k-1, k), (k, k+1)
  // share a pool, which gives the variance t_pairs p^2 (1 + 2p - 3p^2)
  const double p = double(st->x_pools) / P;
  const double ex = double(st->t_pairs) * p * p;
  if (ex > 0.0) {
    const double sd = std::sqrt(ex * (1.0 + 2.0 * p - 3.0 * p * p));
    q->z[WN_Q_EXTREME_PAIRS] = (double(st->x_pairs) - ex) / sd;
  }
  q->passed = 1;
  for (int i = 0; i < WN_QUALITY_NZ; ++i) {
    const double z = one_sided(i) ? q->z[i] : std::fabs(q->z[i]);
    if (!(z <= z_max)) {
      q->passed = 0;
      q->failed_mask |= 1u << i;
    }
  }
  return WN_OK;
}

wn_status wn_tune_config(const wn_config *base, const wn_quality_tuning *opts, uint32_t nreq,
                         const uint32_t *streams, const uint64_t *counts, void *out,
                         wn_dtype out_dtype, uint64_t seed, void *hip_stream, wn_config *chosen,
                         wn_tune_candidate *report, uint32_t report_cap, uint32_t *nreport) {
  const char *who = "wn_tune_config";
  if (!base || !chosen) return tune_fail(WN_EINVAL, "%s: base or chosen is NULL", who);
  if (base->struct_size != sizeof(wn_config))
    return tune_fail(WN_EINVAL, "%s: base must be a full-size wn_config", who);
  if (report_cap > 0 && !report) return tune_fail(WN_EINVAL, "%s: report is NULL", who);
  if (nreq == 0 || !streams || !counts || !out)
    return tune_fail(WN_EINVAL, "%s: the timed request is empty or has a NULL array", who);
  if (wn::enum_bits(out_dtype) > WN_F16)
    return tune_fail(WN_EINVAL, "%s: unknown output dtype %u", who, wn::enum_bits(out_dtype));
  wn_quality_tuning o;
  std::memset(&o, 0, sizeof(o));
  if (opts) {
    if (opts->struct_size != sizeof(wn_quality_tuning))
      return tune_fail(WN_EINVAL, "%s: opts->struct_size %u, expected %zu", who,
                       opts->struct_size, sizeof(wn_quality_tuning));
    o = *opts;
  }
  std::vector<uint32_t> sizes, passes;
  for (uint32_t i = 0; i < 8 && o.pool_sizes[i]; ++i) sizes.push_back(o.pool_sizes[i]);
  for (uint32_t i = 0; i < 8 && o.passes[i]; ++i) passes.push_back(o.passes[i]);
  if (sizes.empty()) sizes = {1024, 2048, 4096};
  if (passes.empty()) passes = {1, 2, 3};
  for (uint32_t n : sizes)
    if (!pool_size_ok(n)) return tune_fail(WN_EINVAL, "%s: candidate pool size %u", who, n);
  for (uint32_t r : passes)
    if (r == 0 || r > 64) return tune_fail(WN_EINVAL, "%s: candidate R %u", who, r);
  if (base->pool_n) sizes = {0};  // per-stream pool sizes stay as configured
  const uint64_t calib = o.calib_values ? o.calib_values : (uint64_t(1) << 30);
  const double z_max = o.z_max > 0.0 ? o.z_max : 5.0;
  uint64_t out_cap = 0;
  for (uint32_t j = 0; j < nreq; ++j) out_cap += counts[j];
  if (out_cap == 0) return tune_fail(WN_EINVAL, "%s: the timed request asks for no values", who);

  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  wn_stats *d_stats = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipSetDevice(base->device);
  if (e == hipSuccess) e = hipMalloc(&d_stats, sizeof(wn_stats));
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  std::vector<wn_stats> host(2);
  auto cleanup = [&]() {
    if (d_stats) (void)hipFree(d_stats);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  };
  if (e != hipSuccess) {
    cleanup();
    return tune_fail(e == hipErrorOutOfMemory ? WN_ENOMEM : WN_EDEVICE, "%s: %s", who,
                     hipGetErrorString(e));
  }

  uint32_t nrep = 0;
  float best_ms = 0.f;
  bool have = false;
  wn_config best = *base;
  wn_status status = WN_OK;
  for (uint32_t n : sizes) {
    for (uint32_t R : passes) {
      wn_config cfg = *base;
      cfg.passes_per_output = R;
      if (n) cfg.default_pool_n = n;
      wn_tune_candidate cand;
      std::memset(&cand, 0, sizeof(cand));
      cand.pool_n = n;
      cand.R = R;
      wn_gen *g = nullptr;
      wn_status s = wn_create(&cfg, &g);
      if (s == WN_OK) s = wn_seed(g, seed, hip_stream);
      // the battery, per distinct pool size: calibration draws from the
      // streams of that size, in calls that fit the caller's buffer
      std::vector<uint32_t> distinct;
      if (s == WN_OK) {
        if (base->pool_n) {
          distinct.assign(base->pool_n, base->pool_n + base->num_streams);
          std::sort(distinct.begin(), distinct.end());
          distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
        } else {
          distinct = {n};
        }
      }
      cand.passed = s == WN_OK ? 1u : 0u;
      for (uint32_t d : distinct) {
        if (s != WN_OK) break;
        std::vector<uint32_t> ids;
        for (uint32_t i = 0; i < base->num_streams; ++i)
          if ((base->pool_n ? base->pool_n[i] : n) == d) ids.push_back(i);
        // at most as many streams as the buffer holds one value each of
        if (ids.size() > out_cap) ids.resize(size_t(out_cap));
        const uint64_t per_total = std::max<uint64_t>(1, calib / ids.size());
        const uint64_t per_call = std::max<uint64_t>(1, std::min(per_total, out_cap / ids.size()));
        wn_stats &acc = host[0];
        std::memset(&acc, 0, sizeof(acc));
        std::vector<uint64_t> cnt(ids.size());
        for (uint64_t done = 0; done < per_total && s == WN_OK;) {
          const uint64_t c = std::min(per_call, per_total - done);
          std::fill(cnt.begin(), cnt.end(), c);
          s = wn_fill_stats(g, uint32_t(ids.size()), ids.data(), cnt.data(), out, out_dtype,
                            d_stats, hip_stream);
          if (s == WN_OK &&
              ((e = hipMemcpyAsync(&host[1], d_stats, sizeof(wn_stats), hipMemcpyDeviceToHost,
                                   st)) != hipSuccess ||
               (e = hipStreamSynchronize(st)) != hipSuccess))
            s = WN_EDEVICE;
          if (s == WN_OK) accumulate(acc, host[1]);
          done += c;
        }
        if (s != WN_OK) break;
        wn_quality q;
        if ((s = wn_quality_check(&acc, d, z_max, &q)) != WN_OK) break;
        if (!q.passed) cand.passed = 0;
        cand.failed_mask |= q.failed_mask;
        for (int i = 0; i < WN_QUALITY_NZ; ++i) {
          const double z = one_sided(i) ? q.z[i] : std::fabs(q.z[i]);
          cand.worst_z = std::max(cand.worst_z, z);
        }
      }
      // time the caller's request with the candidates that pass: one untimed
      // call, then three back to back
      if (s == WN_OK && cand.passed) {
        for (int i = 0; i < 4 && s == WN_OK; ++i) {
          if (i == 1 && (e = hipEventRecord(t0, st)) != hipSuccess) s = WN_EDEVICE;
          if (s == WN_OK) s = wn_fill(g, nreq, streams, counts, out, out_dtype, hip_stream);
        }
        float ms = 0.f;
        if (s == WN_OK && ((e = hipEventRecord(t1, st)) != hipSuccess ||
                           (e = hipEventSynchronize(t1)) != hipSuccess ||
                           (e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess))
          s = WN_EDEVICE;
        cand.ms = ms / 3.f;
      }
      if (s != WN_OK) {
        if (s == WN_EDEVICE && e != hipSuccess)
          tune_fail(s, "%s: candidate n=%u R=%u: %s", who, n, R, hipGetErrorString(e));
        else
          tune_fail(s, "%s: candidate n=%u R=%u: %s", who, n, R, wn_last_error());
        wn_destroy(g);
        status = s;
        break;
      }
      wn_destroy(g);
      if (nrep < report_cap) report[nrep] = cand;
      ++nrep;
      if (cand.passed && (!have || cand.ms < best_ms)) {
        have = true;
        best_ms = cand.ms;
        best = cfg;
      }
    }
    if (status != WN_OK) break;
  }
  cleanup();
  if (nreport) *nreport = nrep;
  if (status != WN_OK) return status;
  if (!have)
    return tune_fail(WN_ENOTSUP, "%s: no candidate passed the statistics at z_max = %g", who,
                     z_max);
  *chosen = best;
  return WN_OK;
}

}  // extern "C"
