// Drives the CPU oracle through every configuration family under the host
// address and undefined-behaviour sanitizers (built by test_host_sanitizers.py
// together with the oracle's own source; test infrastructure only).
#include "../../oracle/wn_oracle.cpp"

#include <cstdio>
#include <vector>

namespace {

int failures = 0;

void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++failures;
  }
}

struct Case {
  uint32_t n, R, f64, chi2, K, hazard, trace, xcur, transform, stride, variate;
  double mean, stddev;
};

void run(const Case &c) {
  orc_config cfg{};
  cfg.num_streams = 3;
  cfg.default_pool_n = c.n;
  cfg.R = c.R;
  cfg.pool_f64 = c.f64;
  cfg.chi2 = c.chi2;
  cfg.K = c.K;
  cfg.hazard = c.hazard;
  cfg.trace = c.trace;
  cfg.x_current = c.xcur;
  cfg.transform = c.transform;
  cfg.emit_stride = c.stride;
  cfg.mean = c.mean;
  cfg.stddev = c.stddev;
  cfg.variate = c.variate;
  const uint32_t sizes[3] = {c.n, c.n, c.n > 16 ? c.n / 2 : c.n};
  void *g = orc_create(&cfg, sizes);
  expect(g != nullptr, "create");
  if (!g) return;
  orc_seed(g, 12345);
  const uint32_t streams[3] = {2, 0, 1};
  for (uint32_t dt = c.f64 ? 0 : 1; dt < 4; ++dt) {
    for (uint64_t a : {uint64_t(0), uint64_t(1), uint64_t(c.n) + 3, uint64_t(5) * c.n}) {
      const uint64_t counts[3] = {a, a / 2 + 1, a ? a - 1 : 7};
      const uint64_t total = counts[0] + counts[1] + counts[2];
      std::vector<double> out(total + 1);
      expect(orc_fill(g, 3, streams, counts, out.data(), dt, 0) == 0, "fill");
    }
  }
  orc_stream_info info{};
  std::vector<double> pool(c.n);
  for (uint32_t s = 0; s < 3; ++s) expect(orc_stream_get(g, s, &info, pool.data()) == 0, "stream");
  expect(orc_stream_get(g, 3, &info, nullptr) != 0, "stream out of range");
  if (c.trace) {
    std::vector<double> tr(6 * 64);
    expect(orc_trace_get(g, 1, tr.data(), 64) > 0, "trace");
  }
  const uint64_t bad[2] = {1, 1};
  const uint32_t twice[2] = {0, 0};
  const uint32_t range[1] = {7};
  std::vector<double> out(4);
  expect(orc_fill(g, 2, twice, bad, out.data(), 1, 0) != 0, "stream twice");
  expect(orc_fill(g, 1, range, bad, out.data(), 1, 0) != 0, "stream out of range");
  orc_destroy(g);
}

}  // namespace

int main() {
  std::vector<Case> cases;
  for (uint32_t f64 = 0; f64 < 2; ++f64)
    for (uint32_t n : {16u, 64u, 256u, 1024u, 4096u}) {
      cases.push_back({n, 2, f64, 0, 4, 0, 1, 0, 0, 1, 0, 0.0, 1.0});   // plain, traced
      cases.push_back({n, 1, f64, 1, 0, 0, 0, 0, 0, 3, 0, 0.0, 1.0});   // rescale off, thinned
      cases.push_back({n, 3, f64, 2, 16, 0, 0, 1, 0, 1, 0, 1.5, 2.0});  // Fisher, current x, mu/sigma
      cases.push_back({n, 2, f64, 3, 16, 0, 0, 0, 1, 1, 0, 0.0, 1.0});  // Wilson-Hilferty, rotations
      cases.push_back({n, 2, f64, 0, 16, 0, 0, 0, 0, 1, 1, 0.0, 1.0});  // exponential
      for (uint32_t hz = 1; hz <= 4; ++hz) cases.push_back({n, 1, f64, 0, 16, hz, 0, 0, 0, 1, 0, 0.0, 1.0});
    }
  for (const Case &c : cases) run(c);

  // configurations the oracle refuses
  orc_config bad{};
  bad.num_streams = 1;
  bad.default_pool_n = 64;
  bad.R = 1;
  bad.stddev = 1.0;
  bad.variate = 1;
  bad.mean = 1.0;
  expect(orc_create(&bad, nullptr) == nullptr, "exponential with mean");
  bad.variate = 2;
  bad.mean = 0.0;
  expect(orc_create(&bad, nullptr) == nullptr, "unknown variate");
  bad.variate = 0;
  bad.stddev = 0.0;
  expect(orc_create(&bad, nullptr) == nullptr, "zero stddev");
  expect(orc_create(nullptr, nullptr) == nullptr, "null config");

  // the building blocks
  uint64_t st = 1, draws[8];
  orc_xorshift64(&st, 8, draws);
  for (uint32_t n : {16u, 256u, 4096u, 16384u}) {
    std::vector<uint32_t> idx(n);
    for (uint32_t hz = 0; hz <= 3; ++hz) orc_gather_index(draws[0], draws[1], n, hz, idx.data());
    expect(orc_warmup_passes(n, 0) > 0 && orc_warmup_passes(n, 1) > 0, "warm-up");
    expect(orc_extreme_threshold(n) > 0.0, "threshold");
  }
  std::printf("cases %zu failures %d\n", cases.size(), failures);
  return failures ? 1 : 0;
}
