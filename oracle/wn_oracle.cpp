// CPU oracle for Wallace's maximum-entropy normal generator, as described in
// R. P. Brent, "Some Comments on C. S. Wallace's Random Number Generators"
// (arXiv 1005.2314).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, obviously correct
// statement of what the generator computes.  Only the test-suite, the smoke
// check and the CPU-baseline leg of the benchmark may load it.  It shares no
// code, header, table or constant generator with the GPU library; neither side
// includes or links the other.
//
// Every step runs in scalar C++ in the order the algorithm states it.  Build
// with -ffp-contract=off and without fast-math so that every + - * / sqrt is a
// single IEEE-754 round-to-nearest-even operation (x86-64 SSE, no x87).
//
// Numbered readings (R1..R13) are the places where the paper is silent or
// leaves a choice open; each is stated where it is used.
//
// Parity status of every function below: pinned by the CPU tests (hand-worked
// passes on a 16-element pool, the printed A1 matrix, published SplitMix64
// output, GF(2) jump-ahead of xorshift64, exact rational sums, the closed form
// of the chi-square constant, Monte-Carlo moments of the chi-square sample,
// library RNE conversions).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------
// Uniform source.  §3 and §5.8: a small-state, long-period integer uniform
// generator is used for initialisation and for choosing the transform of each
// pass (at least once per pool, which carries its period over to the normal
// generator).  R1: xorshift64 with shifts (13, 7, 17) (Marsaglia 2003); the
// returned value is the new state.
// ---------------------------------------------------------------------------
inline uint64_t xorshift64_next(uint64_t &state) {
  uint64_t x = state;
  x ^= x << 13;
  x ^= x >> 7;
  x ^= x << 17;
  state = x;
  return x;
}

// R2: per-stream seeding.  The xorshift state of stream s is output number
// s+1 of SplitMix64 (Steele, Lea, Flood 2014) started from `seed`; a zero
// result (a fixed point of xorshift) is replaced by the golden-ratio constant.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;

inline uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

inline uint64_t stream_state(uint64_t seed, uint64_t stream) {
  uint64_t z = splitmix64_mix(seed + (stream + 1) * kGolden);
  return z == 0 ? kGolden : z;
}

// ---------------------------------------------------------------------------
// Pass parameters.  §5.2: several orthogonal transforms with random signs so
// that the expected transform entry vanishes; §5.3: the transform is held
// fixed within an inner loop; §5.4: mixing through affine maps j -> alpha*j +
// gamma (mod a power of two) with odd alpha.
//
// R3: the pool of n values is viewed as 4 rows of L = n/4 columns (element
// index i = m*L + q).  Each pass draws two uniforms u1, u2 and splits them
// into four 32-bit fields F0 = u1[31:0], F1 = u1[63:32], F2 = u2[31:0],
// F3 = u2[63:32].  Row m is read through the map
//     q -> (alpha_m * q + gamma_m) mod L,
// gamma_m = F_m mod L, alpha_m = 2 * ((F_m >> 12) mod (L/2)) + 1 (odd), and
// the matrix index is k = F0 >> 30.  The bit fields are disjoint for L <= 4096.
// ---------------------------------------------------------------------------
struct PassParams {
  int k;
  uint32_t alpha[4];
  uint32_t gamma[4];
};

PassParams decode_pass(uint64_t u1, uint64_t u2, uint32_t L) {
  const uint32_t F[4] = {uint32_t(u1), uint32_t(u1 >> 32), uint32_t(u2),
                         uint32_t(u2 >> 32)};
  PassParams p;
  for (int m = 0; m < 4; ++m) {
    p.gamma[m] = F[m] & (L - 1);
    p.alpha[m] = 2u * ((F[m] >> 12) & (L / 2 - 1)) + 1u;
  }
  p.k = int(F[0] >> 30);
  return p;
}

// ---------------------------------------------------------------------------
// The 4x4 transform.  §5.3 prints A1 = (1/2)[[1,1,-1,1],[1,-1,1,1],
// [1,-1,-1,-1],[-1,-1,-1,1]] and states that A1 times a 4-vector takes seven
// additions and one halving.  With t = (a+b+c+d)/2 the rows are
// (t-c, t-b, a-t, d-t).  R4: "A2, A3, A4 are similar" is read as
// A_{k+1} = A1 * D_k with the sign matrices D_k below, so that the four
// matrices sum to zero and the mean of every entry over a random k vanishes
// (§5.2).  Each D_k is applied as a sign flip of the inputs.
// ---------------------------------------------------------------------------
constexpr int kSign[4][4] = {
    {+1, +1, +1, +1},  // D0: A1 itself
    {-1, -1, +1, -1},  // D1
    {-1, +1, -1, -1},  // D2
    {+1, -1, -1, +1},  // D3
};

template <class T>
inline void quad_transform(const T x[4], int k, T y[4]) {
  const T a = kSign[k][0] > 0 ? x[0] : -x[0];
  const T b = kSign[k][1] > 0 ? x[1] : -x[1];
  const T c = kSign[k][2] > 0 ? x[2] : -x[2];
  const T d = kSign[k][3] > 0 ? x[3] : -x[3];
  const T s = (a + b) + (c + d);
  const T t = s * T(0.5);
  y[0] = t - c;
  y[1] = t - b;
  y[2] = a - t;
  y[3] = d - t;
}

// ---------------------------------------------------------------------------
// Plane rotations (§5.3, the rann4 form): R(theta) = [[c, s], [-s, c]] with
// c = (1 - t^2)/(1 + t^2), s = 2t/(1 + t^2), t held fixed for a whole pass;
// theta itself is never computed.  R16: the pool is 2 rows of H = n/2; each
// row is read through its own odd-multiplier affine map (rann4's pi1, pi2,
// §5.4) from F0 (row 0) and F1 (row 1): gamma = F mod H,
// alpha = 2((F >> 13) mod H/2) + 1 (bit fields disjoint for H <= 8192);
// t = (F2 >> 8) 2^-24 in [0, 1); F3 bits 0 and 1 flip the signs of c and s
// (so that the mean of every entry over passes vanishes, §5.2).  c and s are
// computed in binary64 (t^2, 1 - t^2 and 1 + t^2 are exact) and rounded to
// the pool type.  Pair q: a = row0[pi0(q)], b = row1[pi1(q)];
// new row0[q] = c a + s b, new row1[q] = c b - s a (products and sums each
// rounded in the pool type).
// ---------------------------------------------------------------------------
struct RotParams {
  uint32_t alpha[2], gamma[2];
  double c, s;
};

RotParams decode_rotation(uint64_t u1, uint64_t u2, uint32_t H) {
  const uint32_t F[4] = {uint32_t(u1), uint32_t(u1 >> 32), uint32_t(u2), uint32_t(u2 >> 32)};
  RotParams p;
  for (int r = 0; r < 2; ++r) {
    p.gamma[r] = F[r] & (H - 1);
    p.alpha[r] = 2u * ((F[r] >> 13) & (H / 2 - 1)) + 1u;
  }
  const double t = double(F[2] >> 8) * 0x1p-24;
  const double tt = t * t;
  p.c = (1.0 - tt) / (1.0 + tt);
  p.s = (2.0 * t) / (1.0 + tt);
  if (F[3] & 1u) p.c = -p.c;
  if (F[3] & 2u) p.s = -p.s;
  return p;
}

template <class T>
void run_rotation_pass(std::vector<T> &P, const RotParams &p, std::vector<T> &scratch) {
  const uint32_t n = uint32_t(P.size());
  const uint32_t H = n / 2;
  const T c = T(p.c), s = T(p.s);
  scratch.assign(n, T(0));
  for (uint32_t q = 0; q < H; ++q) {
    const T a = P[(p.alpha[0] * q + p.gamma[0]) & (H - 1)];
    const T b = P[H + ((p.alpha[1] * q + p.gamma[1]) & (H - 1))];
    const T ca = c * a, sb = s * b, cb = c * b, sa = s * a;
    scratch[q] = ca + sb;
    scratch[H + q] = cb - sa;
  }
  P.swap(scratch);
}

// Negative controls for the mixing requirement of §5.4 (several plausible
// schemes fail).  Only the oracle has them; the tests use them to show that
// the statistical checks can fail.
enum Hazard : uint32_t {
  kHazNone = 0,
  kHazGlobalAffine = 1,  // one affine map over all n positions: partner sets never change
  kHazInPlace = 2,       // results written back to the positions they were read from
  kHazSharedMap = 3,     // all four rows read through row 0's map
  kHazCurrentX = 4,      // chi-square sample from the current pool's withheld value
};

// Source position of row m, column q for one pass (the gather map).
inline uint32_t gather_index(const PassParams &p, uint32_t n, uint32_t m,
                             uint32_t q, uint32_t hazard) {
  const uint32_t L = n / 4;
  switch (hazard) {
    case kHazGlobalAffine:
      return (p.alpha[0] * (m * L + q) + p.gamma[0]) & (n - 1);
    case kHazSharedMap:
      return m * L + ((p.alpha[0] * q + p.gamma[0]) & (L - 1));
    default:
      return m * L + ((p.alpha[m] * q + p.gamma[m]) & (L - 1));
  }
}

// One pass (§5.1: the new pool is an orthogonal transform of the old one).
// R5: all quadruples are formed from the old pool; the result of column q goes
// to positions m*L + q (identity write map), i.e. the new pool is the
// transform of a row-wise permutation of the old one.
template <class T>
void run_pass(std::vector<T> &P, const PassParams &p, uint32_t hazard,
              std::vector<T> &scratch) {
  const uint32_t n = uint32_t(P.size());
  const uint32_t L = n / 4;
  scratch.assign(n, T(0));
  for (uint32_t q = 0; q < L; ++q) {
    uint32_t src[4];
    T x[4], y[4];
    for (uint32_t m = 0; m < 4; ++m) {
      src[m] = gather_index(p, n, m, q, hazard);
      x[m] = P[src[m]];
    }
    quad_transform(x, p.k, y);
    for (uint32_t m = 0; m < 4; ++m) {
      const uint32_t dst = hazard == kHazInPlace ? src[m] : m * L + q;
      scratch[dst] = y[m];
    }
  }
  P.swap(scratch);
}

// ---------------------------------------------------------------------------
// Sum of squares (§5.5: the pool's sum of squares is what the rescale acts
// on).  R6: squares and sums in binary64, in an order fixed by the pool's own
// 4 x L shape (the rows and columns the passes use, §5.4), so that the result
// is a function of the pool alone:
//   c_q = ((x_{0,q}^2 + x_{1,q}^2) + x_{2,q}^2) + x_{3,q}^2   (column q of the
//         4 x L pool, rows in order), q = 0..L-1;
//   Q   = balanced pairwise sum of c_0 .. c_{L-1} in column order (each node
//         adds its left half's sum to its right half's sum).
// The paper fixes only the quantity; this order is a choice of the build.
// ---------------------------------------------------------------------------
double pairwise_sum(const double *a, uint32_t len) {
  if (len == 1) return a[0];
  const uint32_t h = len / 2;
  return pairwise_sum(a, h) + pairwise_sum(a + h, h);
}

template <class T>
double sum_of_squares(const T *P, uint32_t n) {
  const uint32_t L = n / 4;
  std::vector<double> col(L);
  for (uint32_t q = 0; q < L; ++q) {
    double acc = double(P[q]) * double(P[q]);
    for (uint32_t m = 1; m < 4; ++m) {
      const double v = double(P[m * L + q]);
      acc = acc + v * v;
    }
    col[q] = acc;
  }
  return pairwise_sum(col.data(), L);
}

// Rescale the pool so that its sum of squares is n: g = sqrt(n / Q),
// x <- T(double(x) * g).  Used by initialisation and (R9) periodically, to
// stop rounding drift of the invariant sum of squares.
template <class T>
void renormalise(std::vector<T> &P, double Q) {
  const double g = std::sqrt(double(P.size()) / Q);
  for (auto &v : P) v = T(double(v) * g);
}

// ---------------------------------------------------------------------------
// Chi-square sample (§5.5).  The pool's sum of squares should be chi-square
// with nu = n degrees of freedom; one value per pool is withheld and drives an
// approximate chi-square sample S, and the emitted values are scaled so that
// the pool's sum of squares becomes S.  Default (R7): the cubic-corrected form
//   S = A (x^2 - 1) + sqrt(2 (nu - A^2)) x + nu,
// where A is the small root of A^3 - 3 nu A + 2 nu = 0, found here by eight
// Newton steps from 2/3 (only + - * / are used, so host and device agree bit
// for bit; the closed form 2 sqrt(nu) sin(asin(1/sqrt(nu))/3) pins it).
// The evaluation order is S = (A*(x*x - 1) + b*x) + nu.
// Also available: the Fisher form 2 chi2 ~ (x + sqrt(2 nu - 1))^2 and the
// Wilson-Hilferty form chi2 ~ nu (c x + 1 - c^2)^3 with c = sqrt(2/(9 nu)).
// ---------------------------------------------------------------------------
enum Chi2Mode : uint32_t { kChi2Cubic = 0, kChi2Off = 1, kChi2Fisher = 2, kChi2WH = 3 };

struct Chi2Consts {
  double nu, A, b;        // cubic form
  double fisher_root;     // sqrt(2 nu - 1)
  double wh_c, wh_shift;  // sqrt(2/(9 nu)), 1 - 2/(9 nu)
};

Chi2Consts chi2_consts(uint32_t n) {
  Chi2Consts c;
  c.nu = double(n);
  double A = 2.0 / 3.0;
  for (int it = 0; it < 8; ++it) {
    const double num = ((A * A) * A - (3.0 * c.nu) * A) + 2.0 * c.nu;
    const double den = 3.0 * (A * A) - 3.0 * c.nu;
    A = A - num / den;
  }
  c.A = A;
  c.b = std::sqrt(2.0 * (c.nu - A * A));
  c.fisher_root = std::sqrt(2.0 * c.nu - 1.0);
  const double w = 2.0 / (9.0 * c.nu);
  c.wh_c = std::sqrt(w);
  c.wh_shift = 1.0 - w;
  return c;
}

double chi2_sample(const Chi2Consts &c, uint32_t mode, double x) {
  switch (mode) {
    case kChi2Fisher: {
      const double r = x + c.fisher_root;
      return (r * r) * 0.5;
    }
    case kChi2WH: {
      const double r = c.wh_c * x + c.wh_shift;
      return c.nu * ((r * r) * r);
    }
    default:
      return (c.A * (x * x - 1.0) + c.b * x) + c.nu;
  }
}

// ---------------------------------------------------------------------------
// Output conversions, round to nearest even.
// ---------------------------------------------------------------------------
uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return uint16_t((u >> 16) | 0x0040u);  // quiet NaN
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return uint16_t(u >> 16);
}

// binary32 -> binary16 from the definition: scale the magnitude to units of
// the target's last place and round that integer with rint (RNE mode).
uint16_t f32_to_f16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint16_t sign = uint16_t((u >> 16) & 0x8000u);
  const double a = std::fabs(double(f));
  if (std::isnan(f)) return uint16_t(sign | 0x7E00u);
  if (a >= 65520.0) return uint16_t(sign | 0x7C00u);  // rounds to infinity
  if (a < 0x1p-14) {                                  // subnormal range: units of 2^-24
    const double r = std::rint(a * 0x1p24);             // may reach 1024 = smallest normal
    return uint16_t(sign | uint16_t(r));
  }
  int e;
  std::frexp(a, &e);  // a = mant * 2^e, mant in [0.5, 1)
  e -= 1;             // a in [2^e, 2^(e+1))
  double r = std::rint(std::ldexp(a, 10 - e));  // in [1024, 2048]
  if (r == 2048.0) {
    r = 1024.0;
    e += 1;
  }
  if (e > 15) return uint16_t(sign | 0x7C00u);
  return uint16_t(sign | uint16_t((e + 15) << 10) | uint16_t(int(r) - 1024));
}

enum OutDtype : uint32_t { kOutF64 = 0, kOutF32 = 1, kOutBF16 = 2, kOutF16 = 3 };

template <class T>
inline void store_out(void *out, uint64_t pos, T y, uint32_t dtype) {
  switch (dtype) {
    case kOutF64:
      static_cast<double *>(out)[pos] = double(y);
      break;
    case kOutF32:
      static_cast<float *>(out)[pos] = float(y);
      break;
    case kOutBF16:
      static_cast<uint16_t *>(out)[pos] = f32_to_bf16(float(y));
      break;
    default:
      static_cast<uint16_t *>(out)[pos] = f32_to_f16(float(y));
      break;
  }
}

// ---------------------------------------------------------------------------
// Generator state of one stream.
// ---------------------------------------------------------------------------
struct PoolRecord {  // per produced pool, for the statistical tests
  double Q, S, f, x, Temit;
  double zmax;  // largest |T(P[i] T(f))| over the n-1 emitted positions
};

// Extreme-value threshold for pools of n values (Section 5.7: a value large
// enough to appear about once in ten pools).  q is the two-sided normal
// quantile with P(|Z| > q) = erfc(q / sqrt 2) = 0.1 / n, found by bisection on
// erfc (decreasing); c_n is q rounded up to a multiple of 2^-8.
double extreme_threshold(uint32_t n) {
  const double target = 0.1 / double(n);
  double lo = 0.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (std::erfc(mid / std::sqrt(2.0)) > target)
      lo = mid;
    else
      hi = mid;
  }
  return std::ceil(hi * 256.0) / 256.0;
}

template <class T>
struct Stream {
  bool ready = false;
  uint32_t n = 0;
  uint64_t xs = 0;       // xorshift state
  uint64_t k = 0;        // pools produced since seeding
  uint32_t cursor = 0;   // next pool index to emit; n-1 = pool exhausted
  double f = 1.0;        // scale of the current pool
  double xnext = 0.0;    // withheld (scaled) value for the next chi-square sample
  double qlast = 0.0;    // sum of squares of the current pool
  std::vector<T> P;
  std::vector<T> scratch;
  std::vector<PoolRecord> trace;
};

// R8: the initial pool, before any renormalisation: one uniform per element,
// its top 23 bits shifted to a symmetric half-integer grid,
// P[i] = ((v >> 41) - 2^22 + 1/2) 2^-22 (exact in binary32).
template <class T>
void initial_pool(uint64_t &xs, T *P, uint32_t n) {
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t v = xorshift64_next(xs);
    const double c = double(int64_t(v >> 41) - (int64_t(1) << 22)) + 0.5;
    P[i] = T(c * 0x1p-22);
  }
}

struct Config {
  uint32_t num_streams;
  uint32_t R;       // passes per emitted pool
  uint32_t chi2;    // Chi2Mode
  uint32_t K;       // renormalisation period in pools; 0 = never
  uint32_t hazard;  // Hazard (negative controls)
  uint32_t warmup;  // 0 = log2(n) + 4
  uint32_t trace;   // record PoolRecord per pool
  uint32_t x_current;  // chi-square deviate from the current pool (fastnorm's choice)
  uint32_t transform;  // 0: the 4x4 family; 1: plane rotations
  double mean;         // added to every output when non-zero
  double stddev;       // folded into the scale
  uint32_t stride;     // the stream returns every stride-th underlying value
  uint32_t variate;    // 0: normal; 1: exponential (R23)
};

// R23: exponential variates (Section 5 names the exponential as the
// maximum-entropy law under E x = 1, x >= 0; the paper gives no transform).
// If a and b are independent N(0,1), (a^2 + b^2)/2 is exactly Exp(1) (the
// chi-square law with two degrees of freedom, halved).  A pool of the normal
// generator is 4 rows of L; its exponential position j = m*L + q (m = 0, 1)
// pairs the scaled values of rows m and m+2 in column q, which pairs every
// element once and leaves out only the withheld element n-1 with its partner
// (row 1, column L-1): n/2 - 1 exponential values per pool.  With the
// chi-square rescale the sum of a pool's exponential values is half the
// scaled sum of squares of its n-2 paired normals, so it varies from pool to
// pool as the maximum-entropy argument requires (Section 5.5).
inline uint32_t positions_per_pool(uint32_t n, uint32_t variate) {
  return variate == 1 ? n / 2 - 1 : n - 1;
}

inline uint32_t ilog2(uint32_t v) {
  uint32_t r = 0;
  while ((1u << r) < v) ++r;
  return r;
}

// Warm-up passes (R11): log2(n) + 4 for the 4x4 family; a rotation joins 2
// values instead of 4, so its dependency sets grow half as fast: 2 log2(n) + 4.
inline uint32_t warmup_passes(uint32_t n, uint32_t transform) {
  return transform == 1 ? 2 * ilog2(n) + 4 : ilog2(n) + 4;
}

template <class T>
struct Gen {
  Config cfg;
  uint64_t seed = 0;
  bool seeded = false;
  std::vector<uint32_t> pool_n;
  std::vector<Stream<T>> streams;

  // R8: initialisation (§5.8: the uniform generator serves for
  // initialisation).  P[i] from the top 23 bits of successive uniforms,
  // shifted to a symmetric half-integer grid: ((v>>41) - 2^22 + 0.5) * 2^-22,
  // exact in binary32.  Renormalise to a sum of squares of n, run
  // W = log2(n) + 4 warm-up passes (nothing emitted), renormalise again.
  // The withheld value for the first chi-square sample is the last element.
  void init_stream(uint32_t s) {
    Stream<T> &st = streams[s];
    st.n = pool_n[s];
    st.xs = stream_state(seed, s);
    st.P.assign(st.n, T(0));
    initial_pool(st.xs, st.P.data(), st.n);
    renormalise(st.P, sum_of_squares(st.P.data(), st.n));
    const uint32_t W = cfg.warmup ? cfg.warmup : warmup_passes(st.n, cfg.transform);
    for (uint32_t w = 0; w < W; ++w) one_pass(st);
    renormalise(st.P, sum_of_squares(st.P.data(), st.n));
    st.qlast = sum_of_squares(st.P.data(), st.n);
    st.xnext = double(st.P[st.n - 1]);
    st.k = 0;
    st.cursor = positions_per_pool(st.n, cfg.variate);
    st.f = 1.0;
    st.trace.clear();
    st.ready = true;
  }

  void one_pass(Stream<T> &st) {
    const uint64_t u1 = xorshift64_next(st.xs);
    const uint64_t u2 = xorshift64_next(st.xs);
    if (cfg.transform == 1)
      run_rotation_pass(st.P, decode_rotation(u1, u2, st.n / 2), st.scratch);
    else
      run_pass(st.P, decode_pass(u1, u2, st.n / 4), cfg.hazard, st.scratch);
  }

  // Produce pool k (§5.5 and §5.7): R9 renormalise every K pools using the
  // previous pool's sum of squares; R passes (§5.7's option of emitting only
  // some pools, generalised to R passes between emitted pools);
  // sum of squares; chi-square sample from the withheld value of the previous
  // pool (the fastnorm2 choice, §5.5); scale factor f = sqrt(S / Q).
  // R10: x for the next pool is the withheld value scaled by f.  R11: the
  // stored pool is never multiplied by f; only emitted values are.
  void produce_pool(Stream<T> &st, const Chi2Consts &cc) {
    if (st.k > 0 && cfg.K > 0 && st.k % cfg.K == 0) renormalise(st.P, st.qlast);
    for (uint32_t r = 0; r < cfg.R; ++r) one_pass(st);
    const double Q = sum_of_squares(st.P.data(), st.n);
    const double last = double(st.P[st.n - 1]);
    double x = st.xnext;
    if (cfg.hazard == kHazCurrentX || cfg.x_current) x = last;
    double S = 0.0, f = 1.0;
    if (cfg.chi2 != kChi2Off) {
      S = chi2_sample(cc, cfg.chi2, x);
      f = std::sqrt(S / Q);
    }
    st.f = f;
    st.xnext = f * last;
    st.qlast = Q;
    if (cfg.trace) {
      // the standardised values the pool will emit: T(P[i] * T(f)), i < n-1
      const T fT = T(f);
      double zmax = 0.0;
      for (uint32_t i = 0; i + 1 < st.n; ++i)
        zmax = std::max(zmax, std::fabs(double(T(st.P[i] * fT))));
      st.trace.push_back({Q, S, f, x, (f * f) * (Q - last * last), zmax});
    }
    st.k += 1;
    st.cursor = 0;
  }

  // R12: one emitted value is y_i = T(P[i] * T(f * sigma)) for i = 0..n-2,
  // plus T(mu) in the pool type when mu != 0 (Section 5.5: sigma and mu ride
  // on the scale), cast to the output type with round-to-nearest-even (a
  // binary64 pool goes to the 16-bit types through binary32).  fill(c)
  // continues the stream: values left in the current pool are emitted first.
  void fill_stream(uint32_t s, uint64_t count, void *out, uint64_t off, uint32_t dtype) {
    Stream<T> &st = streams[s];
    if (!st.ready) init_stream(s);
    const Chi2Consts cc = chi2_consts(st.n);
    const T muT = T(cfg.mean);
    if (cfg.variate == 1) {
      // R23: position j = m*L + q of a pool is (a*a + b*b) * 1/2 in the pool
      // type, a and b the scaled values of rows m and m+2 in column q
      const uint32_t np = positions_per_pool(st.n, 1);
      const uint32_t L = st.n / 4;
      while (count > 0) {
        if (st.cursor == np) produce_pool(st, cc);
        const T fT = T(st.f * cfg.stddev);
        const uint64_t take = std::min<uint64_t>(count, np - st.cursor);
        for (uint64_t j = 0; j < take; ++j) {
          const uint32_t pos = st.cursor + uint32_t(j);
          const uint32_t m = pos / L, q = pos % L;
          const T a = st.P[m * L + q] * fT;
          const T b = st.P[(m + 2) * L + q] * fT;
          const T aa = a * a;
          const T bb = b * b;
          const T e = (aa + bb) * T(0.5);
          store_out(out, off + j, e, dtype);
        }
        st.cursor += uint32_t(take);
        off += take;
        count -= take;
      }
      return;
    }
    if (cfg.stride > 1) {
      // Section 5.7's option of keeping only some values, for any stride t: the stream is
      // every t-th value of the underlying sequence (the n-1 emitted positions
      // of pool 0, then of pool 1, ...), starting with the first.  Position j
      // of the current pool (index k-1) is underlying value (k-1)(n-1) + j.
      while (count > 0) {
        if (st.cursor == st.n - 1) produce_pool(st, cc);
        const T fT = T(st.f * cfg.stddev);
        const uint64_t first = (st.k - 1) * uint64_t(st.n - 1);
        while (st.cursor < st.n - 1 && count > 0) {
          if ((first + st.cursor) % cfg.stride == 0) {
            T y = st.P[st.cursor] * fT;
            if (cfg.mean != 0.0) y = y + muT;
            store_out(out, off, y, dtype);
            ++off;
            --count;
          }
          ++st.cursor;
        }
      }
      return;
    }
    while (count > 0) {
      if (st.cursor == st.n - 1) produce_pool(st, cc);
      const T fT = T(st.f * cfg.stddev);
      const uint64_t take = std::min<uint64_t>(count, st.n - 1 - st.cursor);
      for (uint64_t j = 0; j < take; ++j) {
        T y = st.P[st.cursor + j] * fT;
        if (cfg.mean != 0.0) y = y + muT;
        store_out(out, off + j, y, dtype);
      }
      st.cursor += uint32_t(take);
      off += take;
      count -= take;
    }
  }
};

struct OrcGen {
  uint32_t pool_f64;
  Gen<float> g32;
  Gen<double> g64;
};

}  // namespace

// ===========================================================================
// C interface (ctypes), test infrastructure only.
// ===========================================================================
extern "C" {

struct orc_config {
  uint32_t num_streams;
  uint32_t default_pool_n;
  uint32_t R;
  uint32_t pool_f64;
  uint32_t chi2;
  uint32_t K;
  uint32_t hazard;
  uint32_t warmup;
  uint32_t trace;
  uint32_t x_current;
  uint32_t transform;
  uint32_t emit_stride;  // 0 or 1: every value; t: every t-th value
  double mean;
  double stddev;
  uint32_t variate;      // 0: normal; 1: exponential (R23)
};

struct orc_stream_info {
  uint64_t xs, k;
  uint32_t n, cursor;
  double f, xnext, qlast;
};

uint64_t orc_xorshift64(uint64_t *state, uint32_t count, uint64_t *out) {
  uint64_t v = 0;
  for (uint32_t i = 0; i < count; ++i) {
    v = xorshift64_next(*state);
    if (out) out[i] = v;
  }
  return v;
}

uint64_t orc_stream_state(uint64_t seed, uint64_t stream) { return stream_state(seed, stream); }

void orc_decode(uint64_t u1, uint64_t u2, uint32_t L, int32_t *k, uint32_t *alpha,
                uint32_t *gamma) {
  const PassParams p = decode_pass(u1, u2, L);
  *k = p.k;
  for (int m = 0; m < 4; ++m) {
    alpha[m] = p.alpha[m];
    gamma[m] = p.gamma[m];
  }
}

// Gather map of one pass: idx[m*L + q] = source position of row m, column q.
void orc_gather_index(uint64_t u1, uint64_t u2, uint32_t n, uint32_t hazard, uint32_t *idx) {
  const PassParams p = decode_pass(u1, u2, n / 4);
  for (uint32_t m = 0; m < 4; ++m)
    for (uint32_t q = 0; q < n / 4; ++q) idx[m * (n / 4) + q] = gather_index(p, n, m, q, hazard);
}

static PassParams make_params(int32_t k, const uint32_t *alpha, const uint32_t *gamma) {
  PassParams p;
  p.k = k;
  for (int m = 0; m < 4; ++m) {
    p.alpha[m] = alpha[m];
    p.gamma[m] = gamma[m];
  }
  return p;
}

void orc_pass_f32(float *P, uint32_t n, int32_t k, const uint32_t *alpha, const uint32_t *gamma,
                  uint32_t hazard) {
  std::vector<float> v(P, P + n), s;
  run_pass(v, make_params(k, alpha, gamma), hazard, s);
  std::copy(v.begin(), v.end(), P);
}

void orc_pass_f64(double *P, uint32_t n, int32_t k, const uint32_t *alpha, const uint32_t *gamma,
                  uint32_t hazard) {
  std::vector<double> v(P, P + n), s;
  run_pass(v, make_params(k, alpha, gamma), hazard, s);
  std::copy(v.begin(), v.end(), P);
}

void orc_transform_f64(const double *x, int32_t k, double *y) { quad_transform(x, k, y); }

void orc_decode_rotation(uint64_t u1, uint64_t u2, uint32_t H, uint32_t *alpha, uint32_t *gamma,
                         double *cs) {
  const RotParams p = decode_rotation(u1, u2, H);
  for (int r = 0; r < 2; ++r) {
    alpha[r] = p.alpha[r];
    gamma[r] = p.gamma[r];
  }
  cs[0] = p.c;
  cs[1] = p.s;
}

static RotParams make_rot(const uint32_t *alpha, const uint32_t *gamma, double c, double s) {
  RotParams p;
  for (int r = 0; r < 2; ++r) {
    p.alpha[r] = alpha[r];
    p.gamma[r] = gamma[r];
  }
  p.c = c;
  p.s = s;
  return p;
}

void orc_rotation_pass_f32(float *P, uint32_t n, const uint32_t *alpha, const uint32_t *gamma,
                           double c, double s) {
  std::vector<float> v(P, P + n), t;
  run_rotation_pass(v, make_rot(alpha, gamma, c, s), t);
  std::copy(v.begin(), v.end(), P);
}

void orc_rotation_pass_f64(double *P, uint32_t n, const uint32_t *alpha, const uint32_t *gamma,
                           double c, double s) {
  std::vector<double> v(P, P + n), t;
  run_rotation_pass(v, make_rot(alpha, gamma, c, s), t);
  std::copy(v.begin(), v.end(), P);
}

uint32_t orc_warmup_passes(uint32_t n, uint32_t transform) { return warmup_passes(n, transform); }

// Initial pool of stream `stream` (before renormalisation and warm-up);
// returns the xorshift state after it.
uint64_t orc_initial_pool_f32(uint64_t seed, uint64_t stream, uint32_t n, float *P) {
  uint64_t xs = stream_state(seed, stream);
  initial_pool(xs, P, n);
  return xs;
}
uint64_t orc_initial_pool_f64(uint64_t seed, uint64_t stream, uint32_t n, double *P) {
  uint64_t xs = stream_state(seed, stream);
  initial_pool(xs, P, n);
  return xs;
}

double orc_sumsq_f32(const float *P, uint32_t n) { return sum_of_squares(P, n); }
double orc_sumsq_f64(const double *P, uint32_t n) { return sum_of_squares(P, n); }

void orc_chi2_consts(uint32_t n, double *A, double *b) {
  const Chi2Consts c = chi2_consts(n);
  *A = c.A;
  *b = c.b;
}

void orc_chi2_sample(uint32_t n, uint32_t mode, const double *x, double *S, uint64_t count) {
  const Chi2Consts c = chi2_consts(n);
  for (uint64_t i = 0; i < count; ++i) S[i] = chi2_sample(c, mode, x[i]);
}

void orc_cvt_bf16(const float *x, uint16_t *y, uint64_t count) {
  for (uint64_t i = 0; i < count; ++i) y[i] = f32_to_bf16(x[i]);
}

void orc_cvt_f16(const float *x, uint16_t *y, uint64_t count) {
  for (uint64_t i = 0; i < count; ++i) y[i] = f32_to_f16(x[i]);
}

void *orc_create(const orc_config *cfg, const uint32_t *pool_n) {
  if (!cfg || cfg->num_streams == 0 || cfg->R == 0) return nullptr;
  auto *g = new OrcGen();
  g->pool_f64 = cfg->pool_f64;
  if (!(cfg->stddev > 0.0) || cfg->transform > 1 || cfg->emit_stride > 16 || cfg->variate > 1 ||
      (cfg->variate == 1 && (cfg->mean != 0.0 || cfg->stddev != 1.0 || cfg->emit_stride > 1))) {
    delete g;
    return nullptr;
  }
  Config c{cfg->num_streams, cfg->R,         cfg->chi2,      cfg->K,    cfg->hazard, cfg->warmup,
           cfg->trace,       cfg->x_current, cfg->transform, cfg->mean, cfg->stddev,
           cfg->emit_stride ? cfg->emit_stride : 1u, cfg->variate};
  std::vector<uint32_t> ns(cfg->num_streams);
  for (uint32_t s = 0; s < cfg->num_streams; ++s) {
    ns[s] = pool_n ? pool_n[s] : cfg->default_pool_n;
    if (ns[s] < 16 || ns[s] > 16384 || (ns[s] & (ns[s] - 1))) {
      delete g;
      return nullptr;
    }
  }
  g->g32.cfg = c;
  g->g64.cfg = c;
  if (g->pool_f64) {
    g->g64.pool_n = ns;
    g->g64.streams.resize(cfg->num_streams);
  } else {
    g->g32.pool_n = ns;
    g->g32.streams.resize(cfg->num_streams);
  }
  return g;
}

void orc_destroy(void *h) { delete static_cast<OrcGen *>(h); }

// Seeding is lazy: a stream is initialised the first time it is used, which
// gives the same result as initialising every stream up front.
void orc_seed(void *h, uint64_t seed) {
  auto *g = static_cast<OrcGen *>(h);
  if (g->pool_f64) {
    g->g64.seed = seed;
    for (auto &s : g->g64.streams) s.ready = false;
  } else {
    g->g32.seed = seed;
    for (auto &s : g->g32.streams) s.ready = false;
  }
}

// Requests are served in parallel (distinct streams are independent);
// outputs are concatenated in request order.  Returns 0 on success.
int orc_fill(void *h, uint32_t nreq, const uint32_t *streams, const uint64_t *counts, void *out,
             uint32_t dtype, int threads) {
  auto *g = static_cast<OrcGen *>(h);
  const uint32_t ns = g->pool_f64 ? g->g64.cfg.num_streams : g->g32.cfg.num_streams;
  if (!g->pool_f64 && dtype == kOutF64) return 5;
  std::vector<uint64_t> off(nreq + 1, 0);
  std::vector<char> seen(ns, 0);
  for (uint32_t j = 0; j < nreq; ++j) {
    if (streams[j] >= ns || seen[streams[j]]) return 1;
    seen[streams[j]] = 1;
    off[j + 1] = off[j] + counts[j];
  }
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t j = 0; j < int64_t(nreq); ++j) {
    if (g->pool_f64)
      g->g64.fill_stream(streams[j], counts[j], out, off[j], dtype);
    else
      g->g32.fill_stream(streams[j], counts[j], out, off[j], dtype);
  }
  return 0;
}

int orc_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Stream state after the calls so far (initialising the stream if needed).
// `pool` (nullable) receives the n pool values in the pool's own type.
int orc_stream_get(void *h, uint32_t s, orc_stream_info *info, void *pool) {
  auto *g = static_cast<OrcGen *>(h);
  auto fill_info = [&](auto &gen) {
    if (s >= gen.streams.size()) return 1;
    auto &st = gen.streams[s];
    if (!st.ready) gen.init_stream(s);
    *info = {st.xs, st.k, st.n, st.cursor, st.f, st.xnext, st.qlast};
    if (pool) std::memcpy(pool, st.P.data(), st.P.size() * sizeof(st.P[0]));
    return 0;
  };
  return g->pool_f64 ? fill_info(g->g64) : fill_info(g->g32);
}

double orc_extreme_threshold(uint32_t n) { return extreme_threshold(n); }

// Per-pool records {Q, S, f, x, T, zmax} of stream s (tracing must be on).
uint64_t orc_trace_get(void *h, uint32_t s, double *buf, uint64_t max_records) {
  auto *g = static_cast<OrcGen *>(h);
  auto get = [&](auto &gen) -> uint64_t {
    if (s >= gen.streams.size()) return 0;
    const auto &tr = gen.streams[s].trace;
    const uint64_t c = std::min<uint64_t>(max_records, tr.size());
    for (uint64_t i = 0; i < c; ++i) {
      buf[6 * i + 0] = tr[i].Q;
      buf[6 * i + 1] = tr[i].S;
      buf[6 * i + 2] = tr[i].f;
      buf[6 * i + 3] = tr[i].x;
      buf[6 * i + 4] = tr[i].Temit;
      buf[6 * i + 5] = tr[i].zmax;
    }
    return c;
  };
  return g->pool_f64 ? get(g->g64) : get(g->g32);
}

}  // extern "C"
