// The C ABI's host paths that need no device, under the host address and
// undefined-behaviour sanitizers (built by test_host_sanitizers.py from the
// library's host sources and abi_stubs.cpp; test infrastructure only):
// configuration validation of every field and struct version, the per-stream
// pool-size array, NULL handling of every entry point, the chi-square
// constants, the extreme-value threshold, the statistics battery and the
// error messages.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "wn.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, wn_last_error());
    ++failures;
  }
}

wn_config base(uint32_t ns, uint32_t n) {
  wn_config c;
  std::memset(&c, 0, sizeof(c));
  c.struct_size = sizeof(wn_config);
  c.num_streams = ns;
  c.default_pool_n = n;
  c.passes_per_output = 2;
  c.pool_dtype = WN_F32;
  c.chi2 = WN_CHI2_CUBIC;
  c.renorm_period = 16;
  c.stddev = 1.0;
  return c;
}

// A configuration the library accepts fails only for want of a device.
void valid(const wn_config &c, const char *what) {
  wn_gen *g = reinterpret_cast<wn_gen *>(1);
  const wn_status s = wn_create(&c, &g);
  expect(s == WN_EDEVICE && g == nullptr, what);
  expect(std::strlen(wn_last_error()) > 0, "message after EDEVICE");
}

void invalid(const wn_config &c, const char *what) {
  wn_gen *g = reinterpret_cast<wn_gen *>(1);
  expect(wn_create(&c, &g) == WN_EINVAL && g == nullptr, what);
}

}  // namespace

int main() {
  // every field, each version of the struct
  valid(base(4, 1024), "plain");
  for (uint32_t n = 16; n <= 16384; n *= 2) valid(base(3, n), "pool size");
  {
    wn_config c = base(2, 1024);
    c.struct_size = WN_CONFIG_V1_SIZE;
    c.emit_stride = 99;
    c.variate = static_cast<wn_variate>(7);
    valid(c, "version 1 ignores later fields");
    c.struct_size = WN_CONFIG_V2_SIZE;
    c.emit_stride = 99;
    valid(c, "version 2 ignores later fields");
  }
  std::vector<uint32_t> sizes(100000);
  for (size_t i = 0; i < sizes.size(); ++i) sizes[i] = 16u << (i % 11);
  {
    wn_config c = base(uint32_t(sizes.size()), 0);
    c.pool_n = sizes.data();
    valid(c, "per-stream sizes");
    sizes[77777] = 3000;
    invalid(c, "per-stream size not a power of two");
    sizes[77777] = 1024;
  }
  const struct {
    const char *what;
    void (*edit)(wn_config &);
  } bad[] = {
      {"no streams", [](wn_config &c) { c.num_streams = 0; }},
      {"too many streams", [](wn_config &c) { c.num_streams = (1u << 24) + 1; }},
      {"pool 1000", [](wn_config &c) { c.default_pool_n = 1000; }},
      {"pool 8", [](wn_config &c) { c.default_pool_n = 8; }},
      {"pool 32768", [](wn_config &c) { c.default_pool_n = 32768; }},
      {"R 0", [](wn_config &c) { c.passes_per_output = 0; }},
      {"R 65", [](wn_config &c) { c.passes_per_output = 65; }},
      {"pool dtype", [](wn_config &c) { c.pool_dtype = WN_BF16; }},
      {"chi2", [](wn_config &c) { c.chi2 = static_cast<wn_chi2>(9); }},
      {"chi2 source", [](wn_config &c) { c.chi2_source = static_cast<wn_chi2_source>(2); }},
      {"transform", [](wn_config &c) { c.transform = static_cast<wn_transform>(5); }},
      {"stddev 0", [](wn_config &c) { c.stddev = 0.0; }},
      {"stddev inf", [](wn_config &c) { c.stddev = INFINITY; }},
      {"mean nan", [](wn_config &c) { c.mean = NAN; }},
      {"stride 17", [](wn_config &c) { c.emit_stride = 17; }},
      {"variate 2", [](wn_config &c) { c.variate = static_cast<wn_variate>(2); }},
      {"exponential with mean", [](wn_config &c) { c.variate = WN_EXPONENTIAL; c.mean = 1.0; }},
      {"exponential with stride", [](wn_config &c) { c.variate = WN_EXPONENTIAL; c.emit_stride = 2; }},
      {"struct size", [](wn_config &c) { c.struct_size = 8; }},
  };
  for (const auto &b : bad) {
    wn_config c = base(2, 1024);
    b.edit(c);
    invalid(c, b.what);
  }
  wn_gen *g = nullptr;
  expect(wn_create(nullptr, &g) == WN_EINVAL, "null config");
  wn_config c = base(2, 1024);
  expect(wn_create(&c, nullptr) == WN_EINVAL, "null out");

  // NULL generator everywhere
  uint32_t s[2] = {0, 1};
  uint64_t n[2] = {5, 5};
  float out[16];
  wn_stream_info info;
  wn_tuning t;
  std::memset(&t, 0, sizeof(t));
  t.struct_size = sizeof(t);
  expect(wn_seed(nullptr, 1, nullptr) == WN_EINVAL, "seed");
  expect(wn_fill(nullptr, 2, s, n, out, WN_F32, nullptr) == WN_EINVAL, "fill");
  wn_stats *dev_stats = reinterpret_cast<wn_stats *>(out);  // never dereferenced: g is NULL
  expect(wn_fill_stats(nullptr, 2, s, n, out, WN_F32, dev_stats, nullptr) == WN_EINVAL,
         "fill_stats");
  expect(wn_fill_stats_noalloc(nullptr, 2, s, n, out, WN_F32, dev_stats, nullptr) == WN_EINVAL,
         "fill_stats_noalloc");
  expect(wn_sync(nullptr) == WN_EINVAL, "sync");
  expect(wn_get_stream(nullptr, 0, &info, nullptr) == WN_EINVAL, "get_stream");
  expect(wn_set_tuning(nullptr, &t) == WN_EINVAL, "set_tuning");
  expect(wn_get_tuning(nullptr, &t) == WN_EINVAL, "get_tuning");
  expect(wn_autotune(nullptr, 2, s, n, out, WN_F32, nullptr, &t) == WN_EINVAL, "autotune");
  expect(wn_state_size(nullptr) == 0, "state_size");
  expect(wn_save_state(nullptr, out, 4) == WN_EINVAL, "save_state");
  expect(wn_load_state(nullptr, out, 4) == WN_EINVAL, "load_state");
  wn_destroy(nullptr);
  expect(wn_version() > 0, "version");

  // the host-only helpers
  double k6[6], prev = 0.0;
  for (uint32_t m = 16; m <= 16384; m *= 2) {
    expect(wn_chi2_constants(m, k6) == WN_OK && k6[0] == double(m), "chi2 constants");
    expect(wn_extreme_threshold(m) > prev, "threshold grows with n");
    prev = wn_extreme_threshold(m);
  }
  expect(wn_chi2_constants(1000, k6) == WN_EINVAL, "chi2 constants, bad n");
  expect(wn_chi2_constants(1024, nullptr) == WN_EINVAL, "chi2 constants, null");
  expect(std::isnan(wn_extreme_threshold(1000)), "threshold, bad n");

  // the battery on synthetic statistics: exact normal moments and histogram
  wn_stats st;
  std::memset(&st, 0, sizeof(st));
  const double N = 1e9;
  st.count = uint64_t(N);
  st.moment[0] = 0.0;
  st.moment[1] = N;
  st.moment[2] = 0.0;
  st.moment[3] = 3.0 * N;
  for (int b = 0; b < 4096; ++b) {
    const double lo = (b - 2048) / 256.0, hi = lo + 1.0 / 256.0;
    st.hist[b] = uint64_t(std::llround(N * 0.5 * (std::erf(hi / std::sqrt(2.0)) -
                                                  std::erf(lo / std::sqrt(2.0)))));
  }
  st.pools = uint64_t(N / 4095);
  st.t_sumsq = 2.0 * 4095 * double(st.pools);
  st.t_pairs = st.pools - 1;
  wn_quality q;
  expect(wn_quality_check(&st, 4096, 5.0, &q) == WN_OK, "quality check");
  expect(q.passed == 1, "exact normal statistics pass");
  st.moment[3] = 3.1 * N;
  expect(wn_quality_check(&st, 4096, 5.0, &q) == WN_OK && (q.failed_mask & (1u << WN_Q_KURT)),
         "kurtosis off fails");
  expect(wn_quality_check(nullptr, 4096, 5.0, &q) == WN_EINVAL, "quality, null stats");
  expect(wn_quality_check(&st, 1000, 5.0, &q) == WN_EINVAL, "quality, bad n");
  expect(wn_quality_check(&st, 4096, 0.0, &q) == WN_EINVAL, "quality, z_max");
  st.count = 1;
  expect(wn_quality_check(&st, 4096, 5.0, &q) == WN_EINVAL, "quality, one value");

  // the semantic tuner refuses bad arguments before it needs a device
  wn_config chosen;
  uint32_t nrep = 0;
  expect(wn_tune_config(nullptr, nullptr, 2, s, n, out, WN_F32, 1, nullptr, &chosen, nullptr, 0,
                        &nrep) == WN_EINVAL, "tune_config, null base");
  expect(wn_tune_config(&c, nullptr, 2, s, n, out, WN_F32, 1, nullptr, nullptr, nullptr, 0,
                        &nrep) == WN_EINVAL, "tune_config, null chosen");
  expect(wn_tune_config(&c, nullptr, 2, s, n, out, static_cast<wn_dtype>(11), 1, nullptr, &chosen,
                        nullptr, 0, &nrep) == WN_EINVAL, "tune_config, bad dtype");
  std::printf("failures %d\n", failures);
  return failures ? 1 : 0;
}
