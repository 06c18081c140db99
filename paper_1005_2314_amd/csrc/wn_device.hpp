// gfx950 device code of the Wallace maximum-entropy normal generator
// (included by the launch units wn_launch_<pool>_<out>.hip through
// wn_launch.hpp, and by wn_stats.hip)
// (R. P. Brent, "Some Comments on C. S. Wallace's Random Number Generators",
// Section 5).
//
// One workgroup owns one stream at a time.  Its pool lives in LDS for the whole
// work item; every thread also keeps the pool elements it last wrote in
// registers, in the layout
//     element i = m*L + c*BD + tid,   m = 0..3 (row), c = 0..NQ-1,
// where L = n/4 is the row length, BD = min(256, L) the block size and
// NQ = L/BD the quadruples per thread.  With this layout
//   * a pass gathers quadruple q = c*BD + tid: consecutive lanes read row
//     positions (alpha*q + gamma) mod L with an odd stride alpha, so the 64
//     lanes of a wave hit 64 distinct LDS banks;
//   * the results go back to positions m*L + q (consecutive lanes, consecutive
//     words), again conflict-free;
//   * thread tid holds whole columns q = c*BD + tid of the 4 x L pool, so the
//     binary64 column sums of the sum of squares (rows in order) need no data
//     movement; the balanced tree over the L columns then runs through a
//     wave-local LDS transposition, DPP lane trees and a few LDS slots;
//   * emission writes, for each (m, c), 64 consecutive output words per wave
//     straight from registers: coalesced stores with no LDS staging.
// There is no MFMA here: the transform is a 4-point stencil, not a dense
// contraction.  The path is bound by HBM writes of the output and the state.
//
// Floating point: the library is built with -ffp-contract=off; binary64 steps
// use the explicit _rn intrinsics so that every operation is one correctly
// rounded IEEE operation in the stated order, matching a scalar CPU
// evaluation bit for bit.

#pragma once

#include "wn_internal.hpp"

// Internal linkage: each launch unit gets its own copy of these definitions.
// Debug builds (WN_POISON_LDS=1, the library libwn_poison.so): every LDS pool
// write is preceded by a fill of the whole buffer with NaN, through a thread
// mapping other than the writes', and a barrier.  A position that a write
// misses, or a read that a missing barrier lets run before the writes, then
// carries NaN into the results, which the parity tests see.
#ifndef WN_POISON_LDS
#define WN_POISON_LDS 0
#endif

namespace wn {
namespace {

constexpr uint32_t kBlock = 256;
constexpr size_t kMaxLds = 160 * 1024;  // LDS per compute unit (gfx950)

// ---- uniform source (Sections 3 and 5.8) -----------------------------------
// xorshift64 with shifts (13, 7, 17); the result is the new state.
__device__ __forceinline__ uint64_t xs_next(uint64_t &s) {
  uint64_t x = s;
  x ^= x << 13;
  x ^= x >> 7;
  x ^= x << 17;
  s = x;
  return x;
}

// Stream seeding: output number stream+1 of SplitMix64 from `seed`
// (increment 0x9E3779B97F4A7C15 and the two-multiply finaliser); 0 -> the
// increment, since 0 is a fixed point of xorshift.
__device__ __forceinline__ uint64_t stream_seed(uint64_t seed, uint64_t stream) {
  const uint64_t inc = 0x9E3779B97F4A7C15ull;
  uint64_t z = seed + (stream + 1) * inc;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return z == 0 ? inc : z;
}

// ---- pass parameters (Sections 5.2-5.4) --------------------------------------
// Two draws give four 32-bit fields F0..F3 (low then high half of each draw).
// Row m is read through q -> (alpha_m q + gamma_m) mod L with
// gamma_m = F_m mod L and odd alpha_m = 2((F_m >> 12) mod L/2) + 1; the
// transform index is the top two bits of F0.
struct PassParams {
  uint32_t k;  // 0..3: matrix A_{k+1}; kRotation: a plane-rotation pass
  uint32_t alpha[4];
  uint32_t gamma[4];
  double c, s;  // rotation passes only
};

constexpr uint32_t kRotation = 4;

__device__ __forceinline__ PassParams decode(uint64_t u1, uint64_t u2, uint32_t L) {
  const uint32_t F[4] = {uint32_t(u1), uint32_t(u1 >> 32), uint32_t(u2), uint32_t(u2 >> 32)};
  PassParams p;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    p.gamma[m] = F[m] & (L - 1);
    p.alpha[m] = 2u * ((F[m] >> 12) & (L / 2 - 1)) + 1u;
  }
  p.k = F[0] >> 30;
  p.c = p.s = 0.0;
  return p;
}

// Plane-rotation passes (Section 5.3, the rann4 form; Section 5.4 for the
// maps).  The pool is two rows of H = n/2; row r is read through
// q -> (alpha_r q + gamma_r) mod H with gamma_r = F_r mod H and odd
// alpha_r = 2((F_r >> 13) mod H/2) + 1.  t = (F2 >> 8) 2^-24 in [0, 1) gives
// c = (1 - t^2)/(1 + t^2) and s = 2t/(1 + t^2), computed in binary64 (t^2,
// 1 - t^2, 1 + t^2 and 2t are exact, each quotient is rounded once); bits 0
// and 1 of F3 negate c and s.  The angle itself is never formed.
__device__ __forceinline__ PassParams decode_rotation(uint64_t u1, uint64_t u2, uint32_t H) {
  const uint32_t F[4] = {uint32_t(u1), uint32_t(u1 >> 32), uint32_t(u2), uint32_t(u2 >> 32)};
  PassParams p;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    p.gamma[r] = F[r] & (H - 1);
    p.alpha[r] = 2u * ((F[r] >> 13) & (H / 2 - 1)) + 1u;
  }
  p.alpha[2] = p.alpha[3] = p.gamma[2] = p.gamma[3] = 0u;
  p.k = kRotation;
  const double t = __dmul_rn(double(F[2] >> 8), 0x1p-24);
  const double tt = __dmul_rn(t, t);
  const double den = __dadd_rn(1.0, tt);
  double c = __ddiv_rn(__dsub_rn(1.0, tt), den);
  double sn = __ddiv_rn(__dadd_rn(t, t), den);
  if (F[3] & 1u) c = -c;
  if (F[3] & 2u) sn = -sn;
  p.c = c;
  p.s = sn;
  return p;
}

// the pass parameters of the transform family for pool rows of length L = n/4
template <bool ROT>
__device__ __forceinline__ PassParams decode_for(uint64_t u1, uint64_t u2, uint32_t L) {
  if constexpr (ROT) return decode_rotation(u1, u2, 2 * L);
  return decode(u1, u2, L);
}

// ---- the 4x4 transform (Section 5.3) -----------------------------------------
// Matrix K is A1 * D_K: the inputs' signs are flipped by D_K (compile-time
// here, so the flips become free source modifiers), then
// t = ((a+b)+(c+d))/2 and y = (t-c, t-b, a-t, d-t): seven additions and one
// halving, the printed A1 when K = 0.
// D0 = (+,+,+,+), D1 = (-,-,+,-), D2 = (-,+,-,-), D3 = (+,-,-,+).
template <int K, typename T>
__device__ __forceinline__ void quad(T a, T b, T c, T d, T (&y)[4]) {
  if (K == 1 || K == 2) a = -a;
  if (K == 1 || K == 3) b = -b;
  if (K == 2 || K == 3) c = -c;
  if (K == 1 || K == 2) d = -d;
  const T s = (a + b) + (c + d);
  const T t = s * T(0.5);
  y[0] = t - c;
  y[1] = t - b;
  y[2] = a - t;
  y[3] = d - t;
}

// One rotation (c, s) of the pair (a, b): (c a + s b, c b - s a), every product
// and sum rounded in the pool type (no fused multiply-add).
__device__ __forceinline__ void rotate(float c, float s, float a, float b, float &y0, float &y1) {
  y0 = __fadd_rn(__fmul_rn(c, a), __fmul_rn(s, b));
  y1 = __fsub_rn(__fmul_rn(c, b), __fmul_rn(s, a));
}
__device__ __forceinline__ void rotate(double c, double s, double a, double b, double &y0,
                                       double &y1) {
  y0 = __dadd_rn(__dmul_rn(c, a), __dmul_rn(s, b));
  y1 = __dsub_rn(__dmul_rn(c, b), __dmul_rn(s, a));
}

// ---- binary64 helpers ----------------------------------------------------------
__device__ __forceinline__ double sq_add(double acc, float v) {
  // the square of a binary32 value is exact in binary64, so the fused form
  // rounds exactly once, like acc + v*v
  const double d = double(v);
  return __fma_rn(d, d, acc);
}
__device__ __forceinline__ double sq_add(double acc, double v) {
  return __dadd_rn(acc, __dmul_rn(v, v));
}

__device__ __forceinline__ double chi2_sample(const Chi2Consts &c, uint32_t mode, double x) {
  if (mode == kChi2Fisher) {
    const double r = __dadd_rn(x, c.fisher_root);
    return __dmul_rn(__dmul_rn(r, r), 0.5);
  }
  if (mode == kChi2WH) {
    const double r = __dadd_rn(__dmul_rn(c.wh_c, x), c.wh_shift);
    return __dmul_rn(c.nu, __dmul_rn(__dmul_rn(r, r), r));
  }
  // (A*(x*x - 1) + b*x) + nu
  const double t1 = __dmul_rn(c.A, __dsub_rn(__dmul_rn(x, x), 1.0));
  return __dadd_rn(__dadd_rn(t1, __dmul_rn(c.b, x)), c.nu);
}

// The chi-square sample of chi2_sample() with the mode chosen by selects
// rather than branches (every variant is evaluated; the same operations, so
// the same result, for the selected one).
__device__ __forceinline__ double chi2_sample_sel(const Chi2Consts &c, uint32_t mode, double x) {
  const double rf = __dadd_rn(x, c.fisher_root);
  const double fisher = __dmul_rn(__dmul_rn(rf, rf), 0.5);
  const double rw = __dadd_rn(__dmul_rn(c.wh_c, x), c.wh_shift);
  const double wh = __dmul_rn(c.nu, __dmul_rn(__dmul_rn(rw, rw), rw));
  const double t1 = __dmul_rn(c.A, __dsub_rn(__dmul_rn(x, x), 1.0));
  const double cubic = __dadd_rn(__dadd_rn(t1, __dmul_rn(c.b, x)), c.nu);
  return mode == kChi2Fisher ? fisher : mode == kChi2WH ? wh : cubic;
}

// v with its sign bit flipped when m = 0x80000000 (exact, like a negation)
__device__ __forceinline__ float flip_sign(float v, uint32_t m) {
  return __uint_as_float(__float_as_uint(v) ^ m);
}
__device__ __forceinline__ double flip_sign(double v, uint32_t m) {
  return __hiloint2double(int(uint32_t(__double2hiint(v)) ^ m), __double2loint(v));
}

// ---- cross-lane moves of binary64 values --------------------------------------------
// DPP (data-parallel primitive) reads of another lane's register, as two 32-bit
// moves.  Controls: quad_perm [1,0,3,2] (0xB1) and [2,3,0,1] (0x4E) exchange
// neighbours and pairs inside a group of 4 lanes; row_half_mirror (0x141)
// reverses each group of 8, row_mirror (0x140) each row of 16, so after the
// first two steps every lane sees a lane of the other half of its group.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = uint64_t(__double_as_longlong(v));
  const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(u)), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, true);
  return __longlong_as_double(int64_t((uint64_t(uint32_t(hi)) << 32) | uint32_t(lo)));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = uint64_t(__double_as_longlong(v));
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u)), lane));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(u >> 32)), lane));
  return __longlong_as_double(int64_t((uint64_t(hi) << 32) | lo));
}

// Balanced pairwise sum over the 64 lanes of a full wave, lane order: four
// levels inside rows of 16 lanes (each lane adds the matching lane of the
// other half of its group; addition commutes, so both halves hold the same
// bits), then (row0 + row1) + (row2 + row3).  Every lane returns the sum.
__device__ __forceinline__ double wave_pairwise_sum(double v) {
  v = __dadd_rn(v, dpp_f64<0xB1>(v));
  v = __dadd_rn(v, dpp_f64<0x4E>(v));
  v = __dadd_rn(v, dpp_f64<0x141>(v));
  v = __dadd_rn(v, dpp_f64<0x140>(v));
  return __dadd_rn(__dadd_rn(readlane_f64(v, 0), readlane_f64(v, 16)),
                   __dadd_rn(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Balanced pairwise sum inside each group of G consecutive lanes (G = 4, 8 or
// 16), lane order; every lane of a group returns its group's sum.  The wave
// must be fully active (DPP reads other lanes' registers).
template <int G>
__device__ __forceinline__ double group_pairwise_sum(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "groups of 4, 8 or 16 lanes");
  v = __dadd_rn(v, dpp_f64<0xB1>(v));
  v = __dadd_rn(v, dpp_f64<0x4E>(v));
  if constexpr (G >= 8) v = __dadd_rn(v, dpp_f64<0x141>(v));
  if constexpr (G >= 16) v = __dadd_rn(v, dpp_f64<0x140>(v));
  return v;
}

// Balanced pairwise sum of v[0..N) in index order (N a power of two).
template <int N>
__device__ __forceinline__ double pairwise(const double *v) {
  if constexpr (N == 1) {
    return v[0];
  } else {
    return __dadd_rn(pairwise<N / 2>(v), pairwise<N / 2>(v + N / 2));
  }
}

// Keeps the compiler from moving LDS accesses across this point.  No
// instruction is needed: the LDS performs the operations of one wave in the
// order they are issued, so a lane reads what other lanes of its wave wrote
// before.
__device__ __forceinline__ void wave_lds_order() { asm volatile("" ::: "memory"); }

// ---- output casts (round to nearest even) ---------------------------------------
struct Bf16 {
  uint16_t u;
};
struct Half {
  uint16_t u;
};

// Binary32 to bfloat16, rounded to nearest even: the hardware conversion
// (v_cvt_pk_bf16_f32).  On MI355X it equals round-to-nearest-even written out
// in integer arithmetic on every binary32 bit pattern that is not a NaN
// (checked exhaustively over all 2^32 patterns, denormals kept); the
// generator never produces a NaN.  The empty asm keeps the binary32 value as
// computed.
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  asm volatile("" : "+v"(f));
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}
// The binary32 value must exist before the conversion: without the empty asm
// the compiler folds "multiply then convert" into v_fma_mixlo_f16, which rounds
// the exact product to binary16 once instead of rounding to binary32 first.
__device__ __forceinline__ uint16_t f16_bits(float f) {
  asm volatile("" : "+v"(f));
  const _Float16 h = static_cast<_Float16>(f);
  return __builtin_bit_cast(uint16_t, h);
}

// Two binary32 values to two 16-bit codes in one conversion (the first in
// the low half): the same round-to-nearest-even as one at a time, with each
// binary32 value pinned first as above.
typedef float F32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 Bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 F16x2 __attribute__((ext_vector_type(2)));
template <typename O>
struct Cast2;
template <>
struct Cast2<Bf16> {
  __device__ static uint32_t from(float a, float b) {
    asm volatile("" : "+v"(a), "+v"(b));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(F32x2{a, b}, Bf16x2));
  }
};
template <>
struct Cast2<Half> {
  __device__ static uint32_t from(float a, float b) {
    asm volatile("" : "+v"(a), "+v"(b));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(F32x2{a, b}, F16x2));
  }
};

template <typename O>
struct Cast;
template <>
struct Cast<float> {
  __device__ static float from(float v) { return v; }
  __device__ static float from(double v) { return float(v); }
};
template <>
struct Cast<double> {
  __device__ static double from(double v) { return v; }
  __device__ static double from(float v) { return double(v); }
};
template <>
struct Cast<Bf16> {
  __device__ static Bf16 from(float v) { return Bf16{bf16_bits(v)}; }
  __device__ static Bf16 from(double v) { return Bf16{bf16_bits(float(v))}; }
};
template <>
struct Cast<Half> {
  __device__ static Half from(float v) { return Half{f16_bits(v)}; }
  __device__ static Half from(double v) { return Half{f16_bits(float(v))}; }
};

// ---- fused statistics -----------------------------------------------------------------
// The emitted value as the statistics see it: binary32 for the binary32 and
// 16-bit outputs (every such value is exact in binary32), binary64 for binary64.
__device__ __forceinline__ float widen(float v) { return v; }
__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ float widen(Bf16 v) { return __uint_as_float(uint32_t(v.u) << 16); }
__device__ __forceinline__ float widen(Half v) { return float(__builtin_bit_cast(_Float16, v.u)); }

// LDS histogram slots: 0 counts y < -8, 1 + b bin b (floor(256 y) + 2048 = b),
// kHistBins + 1 counts y >= 8
constexpr uint32_t kHistSlots = kHistBins + 2;
// statistics LDS: 16 partial-sum slots, 4 per-wave flag words, the histogram
constexpr size_t kStatsLds =
    16 * sizeof(double) + 4 * sizeof(uint32_t) + ((kHistSlots * 4 + 15) / 16) * 16;
static_assert(((kHistSlots * 4 + 15) / 16) * 16 - kHistSlots * 4 >= 8,
              "the histogram's padding holds the persistent kernel's item word");

// Per-thread binary64 sums of y .. y^4 in emission order, and the
// workgroup's LDS histogram: bin floor(256 y) + 2048 for y in [-8, 8).  The
// square y2 is rounded once (exact for a binary32 y); y^3 and y^4 enter their
// sums through one fused multiply-add each.  The bin is taken in the value's
// own type, where 256 y is exact, with no branch: floor(256 y) converted to an
// integer (out-of-range values saturate) and clamped to [-2049, 2048], so that
// -2049 stands for y < -8 and 2048 for y >= 8; the slot is that plus 2049.
struct StatsAcc {
  double m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
  uint32_t *hist = nullptr;
  __device__ __forceinline__ void moments(double y) {
    const double y2 = __dmul_rn(y, y);
    m1 = __dadd_rn(m1, y);
    m2 = __dadd_rn(m2, y2);
    m3 = __fma_rn(y2, y, m3);
    m4 = __fma_rn(y2, y2, m4);
  }
  // floor(z) clamped to [-2049, 2048] (in floating point, so that the
  // conversion to an integer is always in range)
  __device__ __forceinline__ static int32_t bin_of(float z) {
    return int32_t(__builtin_amdgcn_fmed3f(floorf(z), -2049.0f, 2048.0f));
  }
  __device__ __forceinline__ static int32_t bin_of(double z) {
    return int32_t(fmin(fmax(floor(z), -2049.0), 2048.0));
  }
  template <typename V>
  __device__ __forceinline__ void bin(V y) {
    atomicAdd(hist + (bin_of(y * V(256)) + 2049), 1u);
  }
  __device__ __forceinline__ void add(float y) {
    moments(double(y));
    bin(y);
  }
  __device__ __forceinline__ void add(double y) {
    moments(y);
    bin(y);
  }
};

// ---- LDS layout ---------------------------------------------------------------------
// LDS of one workgroup (all dynamic, from local address 0):
//   pool buffer(s)              n * sizeof(T), twice with two buffers
//   sum-of-squares scratch      4 waves x 2 x 64 binary64 (NQ > 1 only)
//   partial-sum slots           two sets of 4 * NQ binary64, used alternately
//   4 words for broadcasts (0: seeding; 1, 2: the pair form's pool counts;
//     3: spare, the persistent kernel's item word when it is the last)
//   with statistics: 16 slots, 4 flag words and the histogram.
// Every part grows with n, so a persistent launch sized for its largest pool
// holds every smaller pool's layout below its own last 8 bytes.
constexpr size_t kMiscLds = 4 * sizeof(uint64_t);

__host__ __device__ constexpr uint32_t nq_of(uint32_t n) { return n >= 1024 ? n / 1024 : 1u; }
// columns per thread handled in one round of the sum-of-squares transposition
// (two: a 4 KiB scratch keeps three workgroups per compute unit for the
// statistics kernel, with two pool buffers and its histogram)
__host__ __device__ constexpr uint32_t sq_round(uint32_t nq) { return nq < 2 ? nq : 2u; }

template <typename T>
__host__ __device__ constexpr size_t pool_lds(uint32_t n, bool db) {
  return size_t(n) * sizeof(T) * (db ? 2 : 1);
}
__host__ __device__ constexpr size_t sq_scratch_lds(uint32_t n) {
  return nq_of(n) > 1 ? size_t(sq_round(nq_of(n))) * 4 * 64 * sizeof(double) : 0;
}
__host__ __device__ constexpr uint32_t slot_set(uint32_t n) { return 4 * nq_of(n); }
// The LDS layout an item of n values on 128 threads alone uses: that of a
// 256-thread item of at least 2048 values, whose sum-of-squares scratch and
// slots cover two columns per thread and per round (n = 1024 has none).
__host__ __device__ constexpr uint32_t layout_n_128(uint32_t n) { return n < 2048 ? 2048u : n; }
template <typename T>
__host__ __device__ constexpr size_t slots_off(uint32_t n, bool db) {
  return pool_lds<T>(n, db) + sq_scratch_lds(n);
}
template <typename T>
__host__ __device__ constexpr size_t misc_off(uint32_t n, bool db) {
  return slots_off<T>(n, db) + 2 * size_t(slot_set(n)) * sizeof(double);
}
template <typename T>
__host__ __device__ constexpr size_t lds_bytes_for(uint32_t n, bool db, bool stats) {
  return misc_off<T>(n, db) + kMiscLds + (stats ? kStatsLds : 0);
}

// ---- the per-workgroup pool engine ------------------------------------------------
// SMALL: pools with L < 256, launched with BD = L threads and NQ = 1.
// DB: two LDS pool buffers; a pass reads one and writes the other, so it needs
// one barrier instead of two (twice the LDS).
//
// Barrier discipline: every LDS pool write is followed by a barrier before the
// pool is read again; sumsq() ends with a barrier that also publishes the pool
// writes before it.  Successive sumsq() calls use the two slot sets in turn,
// so the next call's slot writes never meet this call's slot reads (every
// wave has read them before it reaches the next call's barrier).
// BD: threads per item: 256 (one item per workgroup) or 128 (two items per
// workgroup, one per half: the pair form of persistent launches).  The layout
// and the results are the same for both: element i = m*L + c*BD + tid, with
// NQ = L/BD.
template <typename T, int NQ, bool SMALL, bool DB, int BD = int(kBlock)>
struct Engine {
  static_assert(BD == 256 || BD == 128, "items of 256 or 128 threads");
  static constexpr uint32_t kWaves = uint32_t(BD) / 64;  // waves per item
  static constexpr uint32_t kSet = kWaves * NQ;           // partial-sum slots per set
  T *base;      // LDS: pool buffer 0, then buffer 1 when DB
  double *red;  // LDS: two sets of kSet partial-sum slots
  double *sqs;  // LDS: the sum-of-squares transposition scratch of this item's waves (NQ > 1)
  uint32_t Lr;  // row length for SMALL pools (else the compile-time BD * NQ)
  uint32_t tid; // thread index within the item
  uint32_t cb;  // buffer holding the pool (0, or 1 when DB)
  uint32_t rs;  // slot set of the next sumsq() (0 or 1)
  uint32_t lbase;  // LDS address of base (0, or a half's pool area in the pair form)
  T y[NQ][4];   // y[c][m] = element m*L + c*BD + tid

  // The item's threads meet (both halves of a pair take every barrier).
  __device__ __forceinline__ static void sync() { __syncthreads(); }

  __device__ __forceinline__ uint32_t len() const { return SMALL ? Lr : uint32_t(BD) * NQ; }
  __device__ __forceinline__ uint32_t bd() const { return SMALL ? Lr : uint32_t(BD); }
  __device__ __forceinline__ uint32_t pool_n() const { return 4 * len(); }

  __device__ __forceinline__ uint32_t pos(int m, int c) const {
    return uint32_t(m) * len() + uint32_t(c) * bd() + tid;
  }

  // LDS buffer b (b is a compile-time constant wherever it matters, so the
  // buffer offset can go into the LDS instruction's immediate field)
  __device__ __forceinline__ T *buf(uint32_t b) const { return base + b * pool_n(); }

  // The same buffer as a local-address-space pointer.  The kernels that use
  // the engine have no static LDS, so dynamic LDS starts at local address 0
  // (the build's device-assembly check enforces this), and the buffer's
  // address is a constant: the gather needs no address add per access.
  using LdsT = __attribute__((address_space(3))) const T;
  __device__ __forceinline__ LdsT *lds_buf(uint32_t b) const {
    return reinterpret_cast<LdsT *>(uintptr_t(lbase + b * pool_n() * uint32_t(sizeof(T))));
  }
  __device__ __forceinline__ T *cur() const { return DB ? buf(cb) : base; }

  // WN_POISON_LDS builds: NaN into every position of buffer P (thread tid
  // takes positions j*BD + BD-1-tid), then a barrier.  A no-op otherwise.
  // kPoisonBarriers: the barriers it adds to each pass.
  static constexpr uint32_t kPoisonBarriers = WN_POISON_LDS != 0 ? 1u : 0u;
  __device__ __forceinline__ void poison(T *P) const {
    if constexpr (WN_POISON_LDS != 0) {
      const uint32_t B = bd();
      for (uint32_t j = 0; j < pool_n() / B; ++j) P[j * B + (B - 1 - tid)] = T(__builtin_nan(""));
      sync();
    }
  }

  __device__ __forceinline__ void load_global(const T *__restrict__ g) {
    T *P = cur();
    poison(P);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const T v = g[pos(m, c)];
        y[c][m] = v;
        P[pos(m, c)] = v;
      }
  }

  __device__ __forceinline__ void load_lds() {
    const T *P = cur();
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) y[c][m] = P[pos(m, c)];
  }

  __device__ __forceinline__ void store_global(T *__restrict__ g) const {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) g[pos(m, c)] = y[c][m];
  }

  // write the registers to the buffer holding the pool
  __device__ __forceinline__ void write_lds() {
    T *P = cur();
    poison(P);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) P[pos(m, c)] = y[c][m];
  }

  // y <- T(double(y) * g)
  __device__ __forceinline__ void scale(double g) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) y[c][m] = T(__dmul_rn(double(y[c][m]), g));
  }

  // Byte offsets within row m of the gathers of columns q = c*BD + tid: the
  // row position (alpha_m q + gamma_m) mod L, one add to step c and one mask
  // per element.  alpha_m is odd, so the columns c and c + NQ/2 read positions
  // L/2 apart (mod L): the second half of the offsets is the first half with
  // the top bit of the row offset flipped, one XOR each.
  __device__ __forceinline__ void quad_offsets(const PassParams &p, int m,
                                               uint32_t (&ad)[NQ]) const {
    const uint32_t L = len();
    constexpr uint32_t W = sizeof(T);
    const uint32_t mask = (L - 1) * W;
    const uint32_t a = p.alpha[m];
    const uint32_t first = __umul24(a * W, tid) + p.gamma[m] * W;
    const uint32_t step = a * bd() * W;
#pragma unroll
    for (int c = 0; c < NQ; ++c)
      ad[c] = (NQ >= 2 && c >= NQ / 2) ? (ad[c - NQ / 2] ^ (L * W / 2))
                                       : ((first + step * uint32_t(c)) & mask);
  }

  // Byte offsets within row r (of H = 2L) of the gathers of pairs
  // q = h*L + c*BD + tid: ad[h][c] for the position (alpha_r q + gamma_r) mod H.
  // alpha_r is odd, so h = 1 reads L positions (half the row) from h = 0: the
  // top bit of the offset flipped.
  __device__ __forceinline__ void pair_offsets(const PassParams &p, int r,
                                               uint32_t (&ad)[2][NQ]) const {
    const uint32_t L = len();
    constexpr uint32_t W = sizeof(T);
    const uint32_t mask = (2 * L - 1) * W;
    const uint32_t a = p.alpha[r];
    const uint32_t first = __umul24(a * W, tid) + p.gamma[r] * W;
    const uint32_t step = a * bd() * W;
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      ad[0][c] = (first + step * uint32_t(c)) & mask;
      ad[1][c] = ad[0][c] ^ (L * W);
    }
  }

  // Gather quadruples from buffer RB and transform them with matrix K; row
  // and buffer offsets are immediates.
  // RN: apply the renormalisation scale g to every gathered value first.
  template <int K, int RB, bool RN>
  __device__ __forceinline__ void gather_transform(const PassParams &p, double g) {
    LdsT *P = lds_buf(RB);
    const uint32_t L = len();
    using LdsB = __attribute__((address_space(3))) const unsigned char;
    T x[NQ][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint32_t ad[NQ];
      quad_offsets(p, m, ad);
      LdsB *row = reinterpret_cast<LdsB *>(P + uint32_t(m) * L);
#pragma unroll
      for (int c = 0; c < NQ; ++c) x[c][m] = *reinterpret_cast<LdsT *>(row + ad[c]);
    }
    if constexpr (RN) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][m] = T(__dmul_rn(double(x[c][m]), g));
    }
#pragma unroll
    for (int c = 0; c < NQ; ++c) quad<K>(x[c][0], x[c][1], x[c][2], x[c][3], y[c]);
  }

  // Gather the pairs of a rotation pass from buffer RB and rotate them.  Pair
  // q = h*L + c*BD + tid (h = 0, 1) reads row 0 at (alpha_0 q + gamma_0) mod H
  // and row 1 at (alpha_1 q + gamma_1) mod H, H = 2L, and writes row 0 and row 1
  // position q, which are elements h*L + c*BD + tid and (h+2)*L + c*BD + tid:
  // the registers y[c][h] and y[c][h+2] of this thread.
  template <int RB, bool RN>
  __device__ __forceinline__ void gather_rotate(const PassParams &p, double g) {
    LdsT *P = lds_buf(RB);
    const uint32_t H = 2 * len();
    using LdsB = __attribute__((address_space(3))) const unsigned char;
    T x[NQ][4];  // x[c][h + 2r]: row r's operand of pair h*L + c*BD + tid
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      uint32_t ad[2][NQ];
      pair_offsets(p, r, ad);
      LdsB *row = reinterpret_cast<LdsB *>(P + uint32_t(r) * H);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][h + 2 * r] = *reinterpret_cast<LdsT *>(row + ad[h][c]);
    }
    if constexpr (RN) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][m] = T(__dmul_rn(double(x[c][m]), g));
    }
    const T cT = T(p.c), sT = T(p.s);
#pragma unroll
    for (int c = 0; c < NQ; ++c)
#pragma unroll
      for (int h = 0; h < 2; ++h) rotate(cT, sT, x[c][h], x[c][h + 2], y[c][h], y[c][h + 2]);
  }

  // ROT (compile-time, so that each family's kernels carry only their own
  // gather): a rotation pass; otherwise A_{k+1} by the runtime k.
  template <int RB, bool ROT, bool RN>
  __device__ __forceinline__ void pass_from(const PassParams &p, double g) {
    constexpr int WB = DB ? 1 - RB : RB;
    if constexpr (ROT) {
      gather_rotate<RB, RN>(p, g);
    } else {
      switch (p.k) {
        case 0: gather_transform<0, RB, RN>(p, g); break;
        case 1: gather_transform<1, RB, RN>(p, g); break;
        case 2: gather_transform<2, RB, RN>(p, g); break;
        default: gather_transform<3, RB, RN>(p, g); break;
      }
    }
    if (!DB) sync();
    T *W = buf(WB);
    poison(W);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) W[pos(m, c)] = y[c][m];
  }

  template <bool ROT, bool RN>
  __device__ __forceinline__ void pass_rn(const PassParams &p, double g) {
    if (DB && cb != 0) {
      pass_from<1, ROT, RN>(p, g);
    } else {
      pass_from<0, ROT, RN>(p, g);
    }
    if (DB) cb ^= 1u;
  }

  // One pass: gather from the LDS pool, transform, write the new pool.  The
  // caller places a barrier before the next read of the pool.  `renorm`
  // applies the renormalisation scale g to every gathered value first (each
  // element is gathered exactly once per pass, so this equals rescaling the
  // whole pool before the pass).  The two cases are separate code, so that
  // the common one carries no select between scaled and plain values.
  template <bool ROT>
  __device__ __forceinline__ void pass(const PassParams &p, bool renorm, double g) {
    if (renorm)
      pass_rn<ROT, true>(p, g);
    else
      pass_rn<ROT, false>(p, g);
  }

  // The gathers of gather_transform (quadruples) and gather_rotate (pairs,
  // x[c][h + 2r] = row r's operand of pair h*L + c*BD + tid) on their own, for
  // pass_finish_from (the plain passes fuse them with the transform).
  template <int RB>
  __device__ __forceinline__ void load_quads(const PassParams &p, T (&x)[NQ][4]) const {
    LdsT *P = lds_buf(RB);
    const uint32_t L = len();
    using LdsB = __attribute__((address_space(3))) const unsigned char;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      uint32_t ad[NQ];
      quad_offsets(p, m, ad);
      LdsB *row = reinterpret_cast<LdsB *>(P + uint32_t(m) * L);
#pragma unroll
      for (int c = 0; c < NQ; ++c) x[c][m] = *reinterpret_cast<LdsT *>(row + ad[c]);
    }
  }

  template <int RB>
  __device__ __forceinline__ void load_pairs(const PassParams &p, T (&x)[NQ][4]) const {
    LdsT *P = lds_buf(RB);
    const uint32_t H = 2 * len();
    using LdsB = __attribute__((address_space(3))) const unsigned char;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      uint32_t ad[2][NQ];
      pair_offsets(p, r, ad);
      LdsB *row = reinterpret_cast<LdsB *>(P + uint32_t(r) * H);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][h + 2 * r] = *reinterpret_cast<LdsT *>(row + ad[h][c]);
    }
  }

  // A pass that also finishes the previous pool, whose values are still in y.
  // `chain` (register arithmetic only: that pool's scale) comes first in
  // program order; the values are copied aside; the pass follows with no
  // branch (the signs of D_k as sign-bit masks); `put` stores the copy last.
  // With no branch between the chain and the stores, the compiler interleaves
  // the chain's binary64 latency with the gathers, the transform and the pool
  // writes.  The results are those of pass() and of emitting the copy.
  template <bool ROT, bool RENORM, int RB, typename Chain, typename Put>
  __device__ __forceinline__ void pass_finish_from(const PassParams &p, double g, Chain &&chain,
                                                   Put &&put) {
    constexpr int WB = DB ? 1 - RB : RB;
    chain();
    T prev[NQ][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) prev[c][m] = y[c][m];
    T x[NQ][4];
    if constexpr (ROT) {
      load_pairs<RB>(p, x);
    } else {
      load_quads<RB>(p, x);
    }
    if constexpr (RENORM) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][m] = T(__dmul_rn(double(x[c][m]), g));
    }
    if constexpr (ROT) {
      const T cT = T(p.c), sT = T(p.s);
#pragma unroll
      for (int c = 0; c < NQ; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h) rotate(cT, sT, x[c][h], x[c][h + 2], y[c][h], y[c][h + 2]);
    } else {
      // D_k: a and d negated for k = 1, 2; b for k = 1, 3; c for k = 2, 3
      const uint32_t k = p.k;
      const uint32_t sa = (k == 1 || k == 2) ? 0x80000000u : 0u;
      const uint32_t sb = (k & 1u) ? 0x80000000u : 0u;
      const uint32_t sc = (k >= 2) ? 0x80000000u : 0u;
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const T a = flip_sign(x[c][0], sa), b = flip_sign(x[c][1], sb);
        const T cc = flip_sign(x[c][2], sc), d = flip_sign(x[c][3], sa);
        quad<0>(a, b, cc, d, y[c]);
      }
    }
    if (!DB) sync();
    T *W = buf(WB);
    poison(W);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) W[pos(m, c)] = y[c][m];
    put(prev);
  }

  template <bool ROT, bool RENORM, typename Chain, typename Put>
  __device__ __forceinline__ void pass_finish(const PassParams &p, double g, Chain &&chain,
                                              Put &&put) {
    if (DB && cb != 0) {
      pass_finish_from<ROT, RENORM, 1>(p, g, chain, put);
    } else {
      pass_finish_from<ROT, RENORM, 0>(p, g, chain, put);
    }
    if (DB) cb ^= 1u;
  }

  // Positions 0 .. n-2 of a pool held in v (the layout of y), as
  // T(v * fT) (+ muT when mu, a select), to out[obase + i].
  template <typename O>
  __device__ __forceinline__ void put_whole(const T (&v)[NQ][4], O *__restrict__ out,
                                            uint64_t obase, T fT, bool mu, T muT) const {
    const uint32_t L = len();
    O *dst = out + obase + tid;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const T s = v[c][m] * fT;
        const O o = Cast<O>::from(mu ? T(s + muT) : s);
        if (m < 3 || c < NQ - 1 || tid < bd() - 1) dst[uint32_t(m) * L + uint32_t(c) * bd()] = o;
      }
  }

  // the pool's last element (the withheld one), after the barrier that
  // published the pass writes
  __device__ __forceinline__ T last() const { return cur()[pool_n() - 1]; }

  // Sum of squares of the pool held in y, in the order fixed by the pool's
  // 4 x L shape: column sums c_q = ((x_0q^2 + x_1q^2) + x_2q^2) + x_3q^2, then
  // the balanced pairwise tree over the L columns in column order, all in
  // binary64.  Thread tid holds columns q = c*BD + tid (c = 0..NQ-1).
  //   NQ = 1 (and SMALL): one column per thread; the tree over the threads
  //   is the tree over the columns.
  //   NQ > 1: the tree's nodes of 64 columns are the blocks (c, wave)
  //   = columns c*BD + 64w .. +63.  Each wave writes its column sums to its
  //   own LDS scratch and reads them back transposed: lane l takes NQ
  //   consecutive columns of block (c, w), c = l / G, G = 64 / NQ, and sums
  //   them in-lane; a DPP tree over each group of G lanes gives the block's
  //   node.  The (BD/64) NQ nodes go to LDS slots in column order (c major,
  //   wave minor), and every thread finishes the tree over them.
  // Ends with a barrier; every thread returns the same value.
  __device__ __forceinline__ double sumsq() {
    double col[NQ];
#pragma unroll
    for (int c = 0; c < NQ; ++c) {
      double acc = sq_add(0.0, y[c][0]);
#pragma unroll
      for (int m = 1; m < 4; ++m) acc = sq_add(acc, y[c][m]);
      col[c] = acc;
    }
    double *slots = red + rs * kSet;
    rs ^= 1u;
    if constexpr (NQ == 1) {
      return block_sum(col[0], slots);
    } else {
      constexpr int CR = int(sq_round(NQ));  // columns per thread per round
      constexpr int G = 64 / NQ;             // lanes per block (c, w)
      const uint32_t lane = tid & 63u, w = tid >> 6;
      const uint32_t cl = lane / G, gl = lane % G;  // this lane's block and group slot
      double *sc = sqs + w * (CR * 64);
      double node = 0.0;
#pragma unroll
      for (int r = 0; r < NQ / CR; ++r) {
        if (r > 0) wave_lds_order();  // the previous round's reads come first
#pragma unroll
        for (int j = 0; j < CR; ++j) sc[j * 64 + lane] = col[r * CR + j];
        wave_lds_order();
        if (NQ == CR || cl / CR == uint32_t(r)) {
          const double *src = sc + (cl % CR) * 64 + gl * NQ;
          double v[NQ];
#pragma unroll
          for (int j = 0; j < NQ; ++j) v[j] = src[j];
          node = pairwise<NQ>(v);
        }
      }
      if constexpr (G <= 16) {
        node = group_pairwise_sum<G>(node);
        if (gl == 0) slots[cl * kWaves + w] = node;
      } else {  // NQ = 2: blocks of 32 lanes, rows of 16 combined by lane reads
        node = group_pairwise_sum<16>(node);
        const double b0 = __dadd_rn(readlane_f64(node, 0), readlane_f64(node, 16));
        const double b1 = __dadd_rn(readlane_f64(node, 32), readlane_f64(node, 48));
        if (lane < 2) slots[lane * kWaves + w] = lane == 0 ? b0 : b1;
      }
      __syncthreads();
      // the tree over the kSet nodes: lane i of each wave takes node i, a DPP
      // tree over the first kSet lanes, lane 0's result to every thread
      const double v = lane < kSet ? slots[lane] : 0.0;
      if constexpr (kSet <= 16) {
        return readlane_f64(group_pairwise_sum<int(kSet)>(v), 0);
      } else if constexpr (kSet == 32) {
        const double r = group_pairwise_sum<16>(v);
        return __dadd_rn(readlane_f64(r, 0), readlane_f64(r, 16));
      } else {
        static_assert(kSet == 64, "4, 8, 16, 32 or 64 nodes");
        return wave_pairwise_sum(v);
      }
    }
  }

  // Balanced pairwise sum of one value per thread over the BD threads in
  // thread order (lanes of a wave, then the waves), through 4 LDS slots.
  // Ends with a barrier; every thread returns the same value.  Two calls on
  // the same slots must be separated by a barrier.
  __device__ __forceinline__ double block_sum(double acc, double *slots) const {
    const uint32_t B = bd();
    if (B >= 64) {
      acc = wave_pairwise_sum(acc);
    } else {
      for (uint32_t w = 1; w < B; w <<= 1) acc = __dadd_rn(acc, __shfl_xor(acc, int(w)));
    }
    if (B > 64 && (tid & 63) == 0) slots[tid >> 6] = acc;
    __syncthreads();
    if (B == 128) return __dadd_rn(slots[0], slots[1]);
    if (B == 256) return __dadd_rn(__dadd_rn(slots[0], slots[1]), __dadd_rn(slots[2], slots[3]));
    return acc;
  }

  // Largest |P[i]| over this thread's elements except the withheld n-1.
  __device__ __forceinline__ T max_abs_emitted() const {
    T mx = T(0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const T v = y[c][m] < T(0) ? -y[c][m] : y[c][m];
        if ((m < 3 || c < NQ - 1 || tid < bd() - 1) && v > mx) mx = v;
      }
    return mx;
  }

  // Block-wide OR of one predicate per thread through 4 LDS flag words (one
  // per wave).  Ends with a barrier; two calls must be separated by a barrier.
  __device__ __forceinline__ bool block_any(bool p, uint32_t *flags) const {
    const bool w = __ballot(p) != 0ull;
    if ((tid & 63) == 0) flags[tid >> 6] = w ? 1u : 0u;
    __syncthreads();
    const uint32_t nw = (bd() + 63) / 64;
    uint32_t any = flags[0];
    for (uint32_t i = 1; i < nw; ++i) any |= flags[i];
    return any != 0u;
  }

  template <bool NT, typename O>
  __device__ __forceinline__ static void put(O *p, O v) {
    if constexpr (!NT) {
      *p = v;
    } else if constexpr (sizeof(O) == 2) {
      __builtin_nontemporal_store(v.u, &p->u);
    } else {
      __builtin_nontemporal_store(v, p);
    }
  }

  // Emit pool positions [lo, hi) scaled by fT to out[obase + (i - lo)]; with
  // STATS, also accumulate each emitted value into `sa`.
  // T(P[i] * fT), plus muT in the pool type when MU
  template <bool MU>
  __device__ __forceinline__ static T scaled(T v, T fT, T muT) {
    const T y = v * fT;
    if constexpr (MU) return T(y + muT);
    return y;
  }

  template <bool NT, bool STATS, bool MU, typename O>
  __device__ __forceinline__ void emit(O *__restrict__ out, uint64_t obase, uint32_t lo,
                                       uint32_t hi, T fT, StatsAcc *sa, T muT) const {
    const uint32_t L = len();
    if (lo == 0 && hi == 4 * L - 1) {
      // a whole pool: every position but the withheld last one.  Each row's
      // base is wave-uniform (scalar registers) and the lane's byte offset
      // one 32-bit register, so the stores take the scalar-base form with
      // the column offsets as immediates
      unsigned char *const ob = reinterpret_cast<unsigned char *>(out + obase);
      uint32_t row[4];
      // each row's byte offset for this lane, kept as it is in a 32-bit
      // register (else the compiler folds it into a per-lane 64-bit base and
      // adds the row offsets to that with vector instructions)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        row[m] = (uint32_t(m) * L + tid) * uint32_t(sizeof(O));
        asm("" : "+v"(row[m]));
      }
      auto dst = [&](int m, int c) {
        return reinterpret_cast<O *>(ob + uint64_t(row[m]) + uint64_t(uint32_t(c) * bd()) * sizeof(O));
      };
      if constexpr (sizeof(O) == 2 && NQ % 2 == 0) {
        // 16-bit outputs: columns c and c+1 converted together
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
          for (int c = 0; c < NQ; c += 2) {
            const uint32_t pk = Cast2<O>::from(float(scaled<MU>(y[c][m], fT, muT)),
                                               float(scaled<MU>(y[c + 1][m], fT, muT)));
            const O v0{uint16_t(pk)}, v1{uint16_t(pk >> 16)};
            put<NT>(dst(m, c), v0);
            if constexpr (STATS) sa->add(widen(v0));
            if (m < 3 || c + 1 < NQ - 1 || tid < bd() - 1) {
              put<NT>(dst(m, c + 1), v1);
              if constexpr (STATS) sa->add(widen(v1));
            }
          }
        return;
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
          const O v = Cast<O>::from(scaled<MU>(y[c][m], fT, muT));
          if (m < 3 || c < NQ - 1 || tid < bd() - 1) {
            put<NT>(dst(m, c), v);
            if constexpr (STATS) sa->add(widen(v));
          }
        }
        // with statistics, one row's values at a time: the scheduler would
        // otherwise keep every value's binary64 conversion in flight, and the
        // registers would not fit four workgroups per compute unit
        if constexpr (STATS) __builtin_amdgcn_sched_barrier(0);
      }
      return;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const uint32_t i = pos(m, c);
        if (i >= lo && i < hi) {
          const O v = Cast<O>::from(scaled<MU>(y[c][m], fT, muT));
          put<NT>(out + (obase + (i - lo)), v);
          if constexpr (STATS) sa->add(widen(v));
        }
      }
  }

  // Exponential positions [lo, hi) of the pool held in y to out[obase + (j - lo)]:
  // position j = m*L + c*BD + tid (m = 0, 1) is ((a*a) + (b*b)) * 1/2 in the
  // pool type, a = T(y[c][m] * fT) and b = T(y[c][m+2] * fT): half the sum of
  // squares of two scaled values of the pool, rows m and m+2 of one column.
  template <bool NT, typename O>
  __device__ __forceinline__ void emit_expo(O *__restrict__ out, uint64_t obase, uint32_t lo,
                                            uint32_t hi, T fT) const {
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const uint32_t j = pos(m, c);
        if (j >= lo && j < hi) {
          const T a = y[c][m] * fT;
          const T b = y[c][m + 2] * fT;
          const T aa = a * a;
          const T bb = b * b;
          put<NT>(out + (obase + (j - lo)), Cast<O>::from(T((aa + bb) * T(0.5))));
        }
      }
  }

  // Thinned emission: positions j0, j0 + t, ..., j0 + (take-1) t go to
  // out[obase], out[obase + 1], ... (every t-th value of the stream).
  template <bool NT, bool STATS, typename O>
  __device__ __forceinline__ void emit_thin(O *__restrict__ out, uint64_t obase, uint32_t j0,
                                            uint32_t t, uint32_t take, T fT, StatsAcc *sa,
                                            bool has_mu, T muT) const {
    const uint32_t span = (take - 1) * t;  // last position - j0
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const uint32_t i = pos(m, c);
        const uint32_t d = i - j0;  // wraps past span when i < j0
        if (i >= j0 && d <= span && d % t == 0) {
          const O v = Cast<O>::from(has_mu ? scaled<true>(y[c][m], fT, muT)
                                           : scaled<false>(y[c][m], fT, muT));
          put<NT>(out + (obase + d / t), v);
          if constexpr (STATS) sa->add(widen(v));
        }
      }
  }
};

template <typename T, int NQ, bool SMALL, bool DB>
__device__ __forceinline__ Engine<T, NQ, SMALL, DB> make_engine(unsigned char *smem, uint32_t n) {
  Engine<T, NQ, SMALL, DB> e;
  e.base = reinterpret_cast<T *>(smem);
  e.sqs = reinterpret_cast<double *>(smem + pool_lds<T>(n, DB));
  e.red = reinterpret_cast<double *>(smem + slots_off<T>(n, DB));
  e.Lr = n / 4;
  e.tid = threadIdx.x;
  e.cb = 0;
  e.rs = 0;
  e.lbase = 0;
  return e;
}

// The engine of half h (threads 128h .. 128h+127) of a workgroup whose LDS
// is laid out for pools of nmax values (the pair form): pool buffer(s) in the
// h-th half of the pool area (n <= nmax / 2), the transposition scratch of its
// two waves and half of the slot area.  Both halves fit in the layout of one
// pool of nmax values.
template <typename T, int NQ, bool DB>
__device__ __forceinline__ Engine<T, NQ, false, DB, 128> make_half_engine(unsigned char *smem,
                                                                          uint32_t n, uint32_t nmax,
                                                                          uint32_t h) {
  Engine<T, NQ, false, DB, 128> e;
  e.lbase = h * uint32_t(pool_lds<T>(nmax, DB) / 2);
  e.base = reinterpret_cast<T *>(smem + e.lbase);
  e.sqs = reinterpret_cast<double *>(smem + pool_lds<T>(nmax, DB) + h * (sq_scratch_lds(nmax) / 2));
  e.red = reinterpret_cast<double *>(smem + slots_off<T>(nmax, DB)) + h * slot_set(nmax);
  e.Lr = n / 4;
  e.tid = threadIdx.x & 127u;
  e.cb = 0;
  e.rs = 0;
  return e;
}

// min(count, room) for a wave-uniform 64-bit count, in 32-bit arithmetic with
// no compare.  gfx950 has no scalar 64-bit less-than; written as a compare and
// select, the compiler has been seen to evaluate the compare into VCC but take
// the select from a stale SCC (which made the persistent kernel emit whole
// requests from one pool).
// A value every lane of the wave holds, as a scalar (so that the item's
// counters and output offsets live in scalar registers and the stores can
// address the output with a scalar base and per-lane 32-bit offsets).  The
// builtin returns int: each word goes back to uint32_t before any widening,
// so that a low word with bit 31 set is not sign-extended into the high word.
__device__ __forceinline__ uint32_t uniform32(uint32_t v) {
  return uint32_t(__builtin_amdgcn_readfirstlane(int(v)));
}
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t hi = uniform32(uint32_t(v >> 32));
  const uint32_t lo = uniform32(uint32_t(v));
  return (uint64_t(hi) << 32) | uint64_t(lo);
}

__device__ __forceinline__ uint32_t take_of(uint64_t count, uint32_t room) {
  const uint32_t big = uint32_t((0ull - (count >> 32)) >> 32);  // all ones if count >= 2^32
  return uniform32(min(uint32_t(count) | big, room));
}

__device__ __forceinline__ void flag_fault(uint32_t *err, double Q) {
  if (!(Q > 0.0) || !(Q < __builtin_huge_val())) atomicOr(err, 1u);
}

// ---- LDS regions after the partial-sum slots (offsets from misc_off) ----------------
// broadcast word w (0 .. 3)
__device__ __forceinline__ uint64_t *misc_word(unsigned char *smem, size_t misc, int w) {
  return reinterpret_cast<uint64_t *>(smem + misc) + w;
}

// the statistics' 16 partial-sum slots (four sets of 4)
__device__ __forceinline__ double *stats_slots(unsigned char *smem, size_t misc) {
  return reinterpret_cast<double *>(smem + misc + kMiscLds);
}

__device__ __forceinline__ uint32_t *stats_flags(unsigned char *smem, size_t misc) {
  return reinterpret_cast<uint32_t *>(stats_slots(smem, misc) + 16);
}

__device__ __forceinline__ uint32_t *stats_hist(unsigned char *smem, size_t misc) {
  return stats_flags(smem, misc) + 4;
}

__device__ __forceinline__ void hist_clear(uint32_t *hist) {
  for (uint32_t b = threadIdx.x; b < kHistSlots; b += blockDim.x) hist[b] = 0u;
}

// Add the LDS histogram to the global one (integer adds: the result does not
// depend on their order) and clear it.  Called by every thread after a barrier.
__device__ __forceinline__ void hist_flush(uint32_t *hist, StatsOut *out) {
  for (uint32_t b = threadIdx.x; b < kHistSlots; b += blockDim.x) {
    const uint32_t v = hist[b];
    if (v) {
      unsigned long long *dst = b == 0 ? reinterpret_cast<unsigned long long *>(&out->below)
                                : b <= kHistBins ? reinterpret_cast<unsigned long long *>(out->hist + (b - 1))
                                                 : reinterpret_cast<unsigned long long *>(&out->above);
      atomicAdd(dst, (unsigned long long)v);
      hist[b] = 0u;
    }
  }
}

// ---- seeding (Section 5.8: the uniform source initialises the pool) ----------------
template <typename T, int NQ, bool SMALL, bool ROT>
__global__ __launch_bounds__(kBlock) void k_seed(SeedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t s = a.streams[blockIdx.x];
  const uint32_t n = a.c.n;
  auto e = make_engine<T, NQ, SMALL, false>(smem, n);
  uint64_t &xs_shared = *misc_word(smem, misc_off<T>(n, false), 0);
  StreamHdr *h = a.c.hdr + s;

  // Initial values from the top 23 bits of successive uniforms:
  // ((v >> 41) - 2^22 + 1/2) * 2^-22, exact in binary32.
  e.poison(e.cur());
  if (e.tid == 0) {
    uint64_t xs = stream_seed(a.seed, s);
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t v = xs_next(xs);
      const double c = __dadd_rn(double(int64_t(v >> 41) - (int64_t(1) << 22)), 0.5);
      e.cur()[i] = T(__dmul_rn(c, 0x1p-22));
    }
    xs_shared = xs;
  }
  __syncthreads();
  uint64_t xs = xs_shared;
  e.load_lds();

  const double nd = double(n);
  double Q = e.sumsq();
  e.scale(__dsqrt_rn(__ddiv_rn(nd, Q)));
  e.write_lds();
  __syncthreads();
  for (uint32_t w = 0; w < a.warmup; ++w) {
    const uint64_t u1 = xs_next(xs);
    const uint64_t u2 = xs_next(xs);
    e.template pass<ROT>(decode_for<ROT>(u1, u2, e.len()), false, 1.0);
    __syncthreads();
  }
  Q = e.sumsq();
  e.scale(__dsqrt_rn(__ddiv_rn(nd, Q)));
  e.write_lds();
  __syncthreads();
  Q = e.sumsq();
  if (e.tid == 0) flag_fault(a.c.err, Q);
  const double last = double(e.last());

  e.store_global(reinterpret_cast<T *>(a.c.arena + h->pool_off));
  if (e.tid == 0) {
    h->xs = xs;
    h->k = 0;
    h->f = 1.0;
    h->xnext = last;
    h->qlast = Q;
    h->n = n;
    h->cursor = uint16_t(a.c.expo ? n / 2 - 1 : n - 1);  // no pool ready
    h->sflags = 0;
  }
}

// ---- generation ---------------------------------------------------------------------
// Work item: continue stream s (pool size n, NQ = n/1024 quadruples per
// thread, or the SMALL layout) for `count` values written from out[obase].
// Pool production (Section 5.5): optional renormalisation every K pools with
// the previous sum of squares, R passes, binary64 sum of squares Q, a
// chi-square sample S from the previous pool's withheld scaled value,
// f = sqrt(S / Q); the n-1 first positions are emitted as T(P[i] * T(f)) and
// the withheld value f * P[n-1] feeds the next sample.  The stored pool is
// never scaled.  Starts and ends without a barrier of its own: the caller
// separates two items on one workgroup by a barrier.
//
// DEFER (no statistics; used without thinning): each pool's scale and
// emission run inside the next pool's first pass (pass_finish), where the
// binary64 chain of the scale overlaps the pass's LDS and ALU latency; the
// last pool is finished after the loop.  Same values, same order of stores.
//
// PAIR: the item is half of a pair (128 threads, make_half_engine) and runs
// the plain loop; nmax is the pool size the LDS is laid out for.
//
// BDI = 128 (not PAIR): the item runs on a workgroup of 128 threads alone
// (NQ = L/128; the same layout and results as 256 threads).
template <typename T, typename O, int NQ, bool SMALL, bool DB, bool NT, bool STATS, bool ROT,
          bool DEFER = false, bool PAIR = false, int BDI = int(kBlock)>
__device__ __forceinline__ void fill_item(const FillArgs &a, unsigned char *smem, uint32_t s,
                                          uint64_t count, uint64_t obase, uint32_t req = 0,
                                          uint32_t nmax = 0) {
  static_assert(!(DEFER && STATS), "the deferred form carries no statistics");
  static_assert(!(PAIR && (STATS || DEFER || SMALL)), "the pair form is the plain loop");
  static_assert(BDI == int(kBlock) || (BDI == 128 && !PAIR && !SMALL && !STATS && !DEFER),
                "128-thread items alone: the plain loop without statistics");
  StreamHdr *h = a.c.hdr + s;
  const uint32_t n = uniform32(h->n);
  count = uniform64(count);
  obase = uniform64(obase);
  const uint32_t half = threadIdx.x >> 7;
  auto e = [&]() {
    if constexpr (PAIR)
      return make_half_engine<T, NQ, DB>(smem, n, nmax, half);
    else if constexpr (BDI == 128)
      return make_half_engine<T, NQ, DB>(smem, n, layout_n_128(n), 0);
    else
      return make_engine<T, NQ, SMALL, DB>(smem, n);
  }();
  StatsAcc sa;
  double t_sum = 0.0, t_sumsq = 0.0, t_lag = 0.0, tprev = 0.0;
  uint64_t pools = 0, t_pairs = 0, x_pools = 0, x_pairs = 0;
  const uint32_t sflags = h->sflags;
  bool prev_seen = (sflags & kSeenByStats) != 0;  // may the next pool pair with the current?
  uint32_t xprev = sflags & kHeldExtreme;
  uint32_t *xflags = nullptr;
  const uint64_t emitted = count;
  if constexpr (STATS) {
    sa.hist = stats_hist(smem, misc_off<T>(n, DB));
    xflags = stats_flags(smem, misc_off<T>(n, DB));
    hist_clear(sa.hist);  // published by the barrier after the pool load
    tprev = h->tprev;
  }
  const Chi2Consts &cc = a.c.cc[__builtin_ctz(n) - 4];
  // values a pool gives: n - 1 normals, or n/2 - 1 exponentials
  const bool expo = __builtin_amdgcn_readfirstlane(a.c.expo) != 0;
  const uint32_t np = expo ? n / 2 - 1 : n - 1;
  uint64_t xs = h->xs;
  uint64_t k = uniform64(h->k);
  const uint64_t k0 = k;
  double f = h->f;
  double xnext = h->xnext;
  double qlast = h->qlast;
  uint32_t cursor = uniform32(h->cursor);
  T *gpool = reinterpret_cast<T *>(a.c.arena + h->pool_off);
  O *out = reinterpret_cast<O *>(a.out);

  e.load_global(gpool);
  // The pair form: both halves run the same number of pool steps (the larger
  // of their pool counts), a half whose item is done taking only the steps'
  // barriers.  Each half publishes its count across the barrier below.
  uint64_t steps = 0;
  if constexpr (PAIR) {  // (the pair form runs without thinning)
    const uint64_t head = cursor < np ? take_of(count, np - cursor) : 0u;
    const uint64_t rest = count - head;
    const uint64_t mine = rest == 0 ? 0 : (rest - 1) / np + 1;
    if (e.tid == 0) *misc_word(smem, misc_off<T>(nmax, DB), 1 + int(half)) = mine;
  }
  e.sync();
  if constexpr (PAIR) {
    const uint64_t c0 = *misc_word(smem, misc_off<T>(nmax, DB), 1);
    const uint64_t c1 = *misc_word(smem, misc_off<T>(nmax, DB), 2);
    steps = c0 > c1 ? c0 : c1;
  }

  // Options as wave-uniform scalars, so that each costs one scalar branch
  // per pool rather than vector selects (the defaults skip their work).
  const bool has_mu = __builtin_amdgcn_readfirstlane(a.c.has_mu) != 0;
  const bool unit_sigma = __builtin_amdgcn_readfirstlane(a.c.unit_sigma) != 0;
  const bool x_current = __builtin_amdgcn_readfirstlane(a.c.x_current) != 0;
  const T muT = T(a.c.mu);
  auto scale_of = [&](double fk) -> T { return unit_sigma ? T(fk) : T(__dmul_rn(fk, a.c.sigma)); };
  // Thinning (stride t > 1): the stream is every t-th value of the underlying
  // sequence, position j of pool q being underlying value q (n-1) + j.  ph is
  // the current pool's phase (q (n-1)) mod t, ph_next the next pool's.
  const uint32_t t = __builtin_amdgcn_readfirstlane(a.c.stride);
  uint32_t ph = 0, ph_next = 0;
  if (t > 1) {
    const uint32_t step = (n - 1) % t;
    ph_next = uint32_t((k % t) * step % t);
    ph = (ph_next + t - step) % t;
  }
  // emit up to `count` of this pool's values from `cursor` in thinned order;
  // returns how many, and moves the cursor past the last one emitted
  auto emit_thinned = [&](uint32_t &cur, const T fT) -> uint32_t {
    const uint32_t r = (ph + cur) % t;
    const uint32_t j0 = cur + (r ? t - r : 0u);
    const uint32_t avail = j0 < n - 1 ? (n - 2 - j0) / t + 1 : 0u;
    const uint32_t take = take_of(count, avail);
    if (take == 0) {
      cur = n - 1;
      return 0u;
    }
    e.template emit_thin<NT, STATS>(out, obase, j0, t, take, fT, &sa, has_mu, muT);
    cur = j0 + (take - 1) * t + 1;
    return take;
  };
  if (cursor < np) {
    const T fT = scale_of(f);
    uint32_t take;
    if (t > 1) {
      take = emit_thinned(cursor, fT);
    } else if (expo) {
      take = take_of(count, np - cursor);
      e.template emit_expo<NT>(out, obase, cursor, cursor + take, fT);
      cursor += take;
    } else {
      take = take_of(count, n - 1 - cursor);
      if (has_mu)
        e.template emit<NT, STATS, true>(out, obase, cursor, cursor + take, fT, &sa, muT);
      else
        e.template emit<NT, STATS, false>(out, obase, cursor, cursor + take, fT, &sa, muT);
      cursor += take;
    }
    obase += take;
    count -= take;
  }

  const double nd = double(n);
  // k mod K, kept as a counter (one 64-bit division per work item, not per pool)
  const uint32_t K = a.c.K;
  uint32_t k_mod = K ? uint32_t(k % K) : 0u;
  const bool rescale = a.c.chi2 != kChi2Off;
  bool deferred = false;
  if constexpr (DEFER) {
    if (t == 1 && !expo) {
      deferred = true;
      // kernel-argument values the chain needs, read before the loop
      const Chi2Consts ccv = cc;
      const uint32_t mode = a.c.chi2;
      const double sigma = a.c.sigma;
      const uint32_t R = a.c.R;
      const uint64_t pools = count == 0 ? 0 : (count - 1) / (n - 1) + 1;
      double pq = 0.0, plast = 0.0;  // Q and element n-1 of the pool awaiting its scale
      bool bad = false;
      T fT = T(0);
      // the scale of the pool awaiting it: register arithmetic, no branch
      auto chain = [&]() {
        const double S = chi2_sample_sel(ccv, mode, x_current ? plast : xnext);
        const double fk = rescale ? __dsqrt_rn(__ddiv_rn(S, pq)) : 1.0;
        f = fk;
        xnext = __dmul_rn(fk, plast);
        fT = unit_sigma ? T(fk) : T(__dmul_rn(fk, sigma));
      };
      auto put = [&](const T (&v)[NQ][4]) { e.put_whole(v, out, obase, fT, has_mu, muT); };
      for (uint64_t j = 0; j < pools; ++j) {
        const bool renorm = k > 0 && K > 0 && k_mod == 0;
        double g = 1.0;
        if (renorm) g = __dsqrt_rn(__ddiv_rn(nd, qlast));
        for (uint32_t r = 0; r < R; ++r) {
          const uint64_t u1 = xs_next(xs);
          const uint64_t u2 = xs_next(xs);
          const PassParams p = decode_for<ROT>(u1, u2, e.len());
          if (r == 0 && j > 0) {
            // pool j-1 is finished here: its n-1 values all go out
            if (renorm)
              e.template pass_finish<ROT, true>(p, g, chain, put);
            else
              e.template pass_finish<ROT, false>(p, g, chain, put);
            obase += n - 1;
            count -= n - 1;
          } else {
            e.template pass<ROT>(p, renorm && r == 0, g);
          }
          if (r + 1 < R) e.sync();
        }
        pq = e.sumsq();
        plast = double(e.last());
        bad |= !(pq > 0.0) || !(pq < __builtin_huge_val());
        qlast = pq;
        k += 1;
        if (K) k_mod = k_mod + 1 == K ? 0u : k_mod + 1;
      }
      if (pools > 0) {
        // the last pool: its scale, then the values the request still wants
        chain();
        const uint32_t take = take_of(count, n - 1);
        if (has_mu)
          e.template emit<NT, false, true>(out, obase, 0, take, fT, &sa, muT);
        else
          e.template emit<NT, false, false>(out, obase, 0, take, fT, &sa, muT);
        cursor = take;
        obase += take;
        count -= take;
      }
      if (bad && e.tid == 0) atomicOr(a.c.err, 1u);
    }
  }
  for (uint64_t step = 0; !deferred && (PAIR ? step < steps : count > 0); ++step) {
    if (PAIR && count == 0) {
      // this half's item is done: the barriers of one pool step (2 per pass
      // with one LDS buffer, 1 with two; the last one is the sum of squares'),
      // plus one per pass in the LDS-poisoning debug build
      const uint32_t per_pass = (DB ? 1u : 2u) + decltype(e)::kPoisonBarriers;
      for (uint32_t b = 0; b < per_pass * a.c.R; ++b) __syncthreads();
      continue;
    }
    const bool renorm = k > 0 && K > 0 && k_mod == 0;
    double g = 1.0;
    if (renorm) g = __dsqrt_rn(__ddiv_rn(nd, qlast));
    // with the previous pool's withheld value as the source (the default), the
    // chi-square sample does not depend on this pool: take it off the chain
    // that follows the sum of squares
    double S = 0.0;
    if (rescale && !x_current) S = chi2_sample(cc, a.c.chi2, xnext);
    for (uint32_t r = 0; r < a.c.R; ++r) {
      const uint64_t u1 = xs_next(xs);
      const uint64_t u2 = xs_next(xs);
      e.template pass<ROT>(decode_for<ROT>(u1, u2, e.len()), renorm && r == 0, g);
      if (r + 1 < a.c.R) e.sync();
    }
    const double Q = e.sumsq();
    const double last = double(e.last());
    double fk = 1.0;
    if (rescale) {
      if (x_current) S = chi2_sample(cc, a.c.chi2, last);
      fk = __dsqrt_rn(__ddiv_rn(S, Q));
    }
    if (e.tid == 0) flag_fault(a.c.err, Q);
    f = fk;
    xnext = __dmul_rn(fk, last);
    qlast = Q;
    if constexpr (STATS) {
      // T = f^2 (Q - P[n-1]^2), the sum of squares of the pool's emitted
      // values, centred on its expected value n - 1
      const double Tk = __dsub_rn(__dmul_rn(__dmul_rn(fk, fk), __dsub_rn(Q, __dmul_rn(last, last))),
                                  double(n - 1));
      t_sum = __dadd_rn(t_sum, Tk);
      t_sumsq = __dadd_rn(t_sumsq, __dmul_rn(Tk, Tk));
      const bool paired = k > 0 && prev_seen;
      if (paired) {
        t_lag = __dadd_rn(t_lag, __dmul_rn(Tk, tprev));
        t_pairs += 1;
      }
      tprev = Tk;
      pools += 1;
      // Section 5.7: does the pool emit a value with |T(P[i] T(f))| >= c_n?
      // Rounding is monotone, so the largest such value is T(max|P[i]| T(f)).
      const T zmax = T(e.max_abs_emitted() * T(fk));
      const uint32_t ek = e.block_any(double(zmax) >= a.c.xthr[__builtin_ctz(n) - 4], xflags);
      x_pools += ek;
      if (paired) x_pairs += ek & xprev;
      xprev = ek;
      prev_seen = true;
    }
    k += 1;
    if (K) k_mod = k_mod + 1 == K ? 0u : k_mod + 1;
    const T fT = scale_of(f);
    uint32_t take;
    if (t > 1) {
      ph = ph_next;
      ph_next = (ph_next + (n - 1) % t) % t;
      cursor = 0;
      take = emit_thinned(cursor, fT);
    } else if (expo) {
      take = take_of(count, np);
      e.template emit_expo<NT>(out, obase, 0, take, fT);
      cursor = take;
    } else {
      take = take_of(count, n - 1);
      if (has_mu)
        e.template emit<NT, STATS, true>(out, obase, 0, take, fT, &sa, muT);
      else
        e.template emit<NT, STATS, false>(out, obase, 0, take, fT, &sa, muT);
      cursor = take;
    }
    obase += take;
    count -= take;
  }

  e.store_global(gpool);
  if (e.tid == 0) {
    h->xs = xs;
    h->k = k;
    h->f = f;
    h->xnext = xnext;
    h->qlast = qlast;
    h->cursor = uint16_t(cursor);
    if constexpr (STATS) {
      h->tprev = tprev;
      if (pools > 0) h->sflags = uint16_t(kSeenByStats | xprev);
    } else if (sflags != 0 && k != k0) {
      h->sflags = 0;  // a pool the statistics did not see
    }
  }
  if constexpr (STATS) {
    // the request's moments: a pairwise tree over the threads, one slot set per
    // moment; then the histogram goes to the global one
    double *slots = stats_slots(smem, misc_off<T>(n, DB));
    const double s1 = e.block_sum(sa.m1, slots);
    const double s2 = e.block_sum(sa.m2, slots + 4);
    const double s3 = e.block_sum(sa.m3, slots + 8);
    const double s4 = e.block_sum(sa.m4, slots + 12);
    if (e.tid == 0) {
      StatsPartial &pp = a.partials[req];
      pp.moment[0] = s1;
      pp.moment[1] = s2;
      pp.moment[2] = s3;
      pp.moment[3] = s4;
      pp.t_sum = t_sum;
      pp.t_sumsq = t_sumsq;
      pp.t_lag = t_lag;
      pp.count = emitted;
      pp.pools = pools;
      pp.t_pairs = t_pairs;
      pp.x_pools = x_pools;
      pp.x_pairs = x_pairs;
    }
    hist_flush(sa.hist, a.stats);
    __syncthreads();  // slots and histogram are reused by the next item
  }
}

// Workgroup b runs work items b*P .. b*P + P-1 one after another (P =
// items_per_wg; all items of the launch share one pool size).  In the affine
// form consecutive items write consecutive output ranges, so a larger P gives
// each workgroup a longer contiguous run of stores.
// BDK: threads per workgroup, 256, or 128 for pools of 1024 to 4096 values
// (NQ = n/512 then; no statistics or rotations).
template <typename T, typename O, int NQ, bool SMALL, bool DB, bool NT, int WPE, bool STATS,
          bool ROT, int BDK = int(kBlock)>
__global__ __launch_bounds__(BDK, WPE) void k_fill(FillArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t per = a.items_per_wg;
  bool ran = false;
  for (uint32_t t = 0; t < per; ++t) {
    const uint32_t j = blockIdx.x * per + t;
    if (j >= a.nitems) break;
    uint32_t s;
    uint64_t count, obase;
    if (a.items) {
      const WorkItem it = a.items[j];
      s = it.stream;
      count = it.count;
      obase = it.out_off;
    } else {
      s = a.affine_s0 + j;
      count = a.count_each;
      obase = uint64_t(j) * a.count_each;
    }
    if (count == 0) {
      if constexpr (STATS)
        if (threadIdx.x == 0) a.partials[j] = StatsPartial{};
      continue;
    }
    if (ran) __syncthreads();  // the previous item's last LDS reads are done
    ran = true;
    const uint32_t req = a.items ? a.items[j].req : j;
    fill_item<T, O, NQ, SMALL, DB, NT, STATS, ROT, false, false, BDK>(a, smem, s, count, obase,
                                                                       req);
  }
}

// The deferred form for latency-bound launches (few streams): one item per
// workgroup, two LDS buffers, no statistics.
template <typename T, typename O, int NQ, bool ROT>
__global__ __launch_bounds__(kBlock) void k_fill_defer(FillArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t j = blockIdx.x;
  if (j >= a.nitems) return;
  uint32_t s;
  uint64_t count, obase;
  if (a.items) {
    const WorkItem it = a.items[j];
    s = it.stream;
    count = it.count;
    obase = it.out_off;
  } else {
    s = a.affine_s0 + j;
    count = a.count_each;
    obase = uint64_t(j) * a.count_each;
  }
  if (count == 0) return;
  fill_item<T, O, NQ, false, true, false, false, ROT, true>(a, smem, s, count, obase);
}

template <typename T, typename O, int NQ, int MAXNQ, bool DB, bool NT, bool STATS, bool ROT,
          bool DEFER = false>
__device__ __forceinline__ void item_as(const FillArgs &a, unsigned char *smem, const WorkItem &it) {
  fill_item<T, O, NQ, false, DB, NT, STATS, ROT, DEFER>(a, smem, it.stream, it.count, it.out_off,
                                                        it.req);
}

// Persistent form: a fixed grid of workgroups pops work items (pool sizes
// 1024 .. 1024*MAXNQ, mixed) from a device counter in the order of the list
// (the host sorts it longest first).  Every workgroup leaves the loop once the
// counter passes the end of the list.
// PAIRS: the list holds entries (a.entries): an item index and a kind
// (kEntry*): one item run by the whole workgroup, or a pair, items i and i+1
// of pool size 1024, run by the two halves at once (128 threads each) in the
// plain loop; with DEFER the items that run alone take the deferred form as
// usual.  (A pair of 2048-value pools would need 136 registers in this
// layout, more than four waves per SIMD allow.)
// With PAIRS the kernel is held to 128 registers (four waves per SIMD, so
// eight streams per compute unit in pairs); combining the two paths would
// otherwise take 143.
template <typename T, typename O, int MAXNQ, bool DB, bool NT, bool STATS, bool ROT,
          bool DEFER = false, bool PAIRS = false>
__global__ __launch_bounds__(kBlock, PAIRS ? 4 : 1) void k_fill_persistent(FillArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // the last 8 bytes of the allocation: the largest pool's spare broadcast
  // word (or the histogram's padding); no item's layout reaches them
  uint64_t &next_item = *reinterpret_cast<uint64_t *>(
      smem + lds_bytes_for<T>(1024 * MAXNQ, DB, STATS) - sizeof(uint64_t));
  for (;;) {
    __syncthreads();  // the previous item's last LDS reads are done
    if (threadIdx.x == 0) next_item = atomicAdd(a.counter, 1u);
    __syncthreads();
    const uint32_t j = uint32_t(next_item);
    if (j >= a.nitems) break;
    // the list is longest first: its head is the critical path, so its waves
    // win instruction issue against the shorter items sharing the SIMD
    if (j < a.prio_items)
      __builtin_amdgcn_s_setprio(3);
    else
      __builtin_amdgcn_s_setprio(0);
    uint32_t idx = j;
    if constexpr (PAIRS) {
      static_assert(!STATS && MAXNQ == 4, "groups: no statistics, pools up to 4096");
      const uint32_t v = a.entries[j];
      idx = v & kEntryIndex;
      const uint32_t kind = v >> kEntryKindShift;
      if (kind == kEntryPair) {
        const WorkItem it = a.items[idx + (threadIdx.x >> 7)];
        fill_item<T, O, 2, false, DB, NT, false, ROT, false, true>(
            a, smem, it.stream, it.count, it.out_off, it.req, 1024 * MAXNQ);
        continue;
      }
    }
    const WorkItem it = a.items[idx];
    if (it.count == 0) {
      if constexpr (STATS)
        if (threadIdx.x == 0) a.partials[it.req] = StatsPartial{};
      continue;
    }
    switch (a.c.hdr[it.stream].n) {
      // deferred form for pools of up to 2048 (the long chains of small pools);
      // larger pools keep the plain loop, whose registers set the occupancy
      case 1024: item_as<T, O, 1, MAXNQ, DB, NT, STATS, ROT, DEFER>(a, smem, it); break;
      case 2048: if constexpr (MAXNQ >= 2) item_as<T, O, 2, MAXNQ, DB, NT, STATS, ROT, DEFER>(a, smem, it); break;
      case 4096: if constexpr (MAXNQ >= 4) item_as<T, O, 4, MAXNQ, DB, NT, STATS, ROT>(a, smem, it); break;
      case 8192: if constexpr (MAXNQ >= 8) item_as<T, O, 8, MAXNQ, DB, NT, STATS, ROT>(a, smem, it); break;
      default: if constexpr (MAXNQ >= 16) item_as<T, O, 16, MAXNQ, DB, NT, STATS, ROT>(a, smem, it); break;
    }
  }
}

// Persistent form on 128-thread workgroups, for lists whose pools hold 1024 or
// 2048 values (no statistics, rotations or deferred emission): each item runs
// alone on 128 threads (NQ = n/512) with the layout of a 2048-value item, so
// the results are those of every other form.  The item word is misc word 3 of
// that layout, which no item uses.
template <typename T, typename O, bool DB, bool NT>
__global__ __launch_bounds__(128) void k_fill_persistent128(FillArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t &next_item =
      *reinterpret_cast<uint64_t *>(smem + lds_bytes_for<T>(2048, DB, false) - sizeof(uint64_t));
  for (;;) {
    __syncthreads();  // the previous item's last LDS reads are done
    if (threadIdx.x == 0) next_item = atomicAdd(a.counter, 1u);
    __syncthreads();
    const uint32_t j = uint32_t(next_item);
    if (j >= a.nitems) break;
    if (j < a.prio_items)
      __builtin_amdgcn_s_setprio(3);
    else
      __builtin_amdgcn_s_setprio(0);
    const WorkItem it = a.items[j];
    if (it.count == 0) continue;
    if (a.c.hdr[it.stream].n == 1024)
      fill_item<T, O, 2, false, DB, NT, false, false, false, false, 128>(a, smem, it.stream,
                                                                         it.count, it.out_off, it.req);
    else
      fill_item<T, O, 4, false, DB, NT, false, false, false, false, 128>(a, smem, it.stream,
                                                                         it.count, it.out_off, it.req);
  }
}

[[maybe_unused]] __global__ void k_reset_counter(uint32_t *ctr) {
  if (threadIdx.x == 0) *ctr = 0u;
}

}  // namespace
}  // namespace wn
