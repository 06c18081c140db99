// gfx950 kernels of the Wallace maximum-entropy normal generator
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
//   * thread tid holds exactly the elements i = tid (mod BD), so the binary64
//     sum of squares in its fixed order (interleaved running sums, then a
//     balanced tree over the BD running sums) needs no data movement before
//     the cross-lane tree;
//   * emission writes, for each (m, c), 64 consecutive output words per wave
//     straight from registers: coalesced stores with no LDS staging.
// There is no MFMA here: the transform is a 4-point stencil, not a dense
// contraction.  The path is bound by HBM writes of the output and the state.
//
// Floating point: the library is built with -ffp-contract=off; binary64 steps
// use the explicit _rn intrinsics so that every operation is one correctly
// rounded IEEE operation in the stated order, matching a scalar CPU
// evaluation bit for bit.

#include "wn_internal.hpp"

namespace wn {
namespace {

constexpr uint32_t kBlock = 256;

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
  uint32_t k;
  uint32_t alpha[4];
  uint32_t gamma[4];
};

__device__ __forceinline__ PassParams decode(uint64_t u1, uint64_t u2, uint32_t L) {
  const uint32_t F[4] = {uint32_t(u1), uint32_t(u1 >> 32), uint32_t(u2), uint32_t(u2 >> 32)};
  PassParams p;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    p.gamma[m] = F[m] & (L - 1);
    p.alpha[m] = 2u * ((F[m] >> 12) & (L / 2 - 1)) + 1u;
  }
  p.k = F[0] >> 30;
  return p;
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

// ---- output casts (round to nearest even) ---------------------------------------
struct Bf16 {
  uint16_t u;
};
struct Half {
  uint16_t u;
};

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return uint16_t((u >> 16) | 0x0040u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
// The binary32 value must exist before the conversion: without the empty asm
// the compiler folds "multiply then convert" into v_fma_mixlo_f16, which rounds
// the exact product to binary16 once instead of rounding to binary32 first.
__device__ __forceinline__ uint16_t f16_bits(float f) {
  asm volatile("" : "+v"(f));
  const _Float16 h = static_cast<_Float16>(f);
  return __builtin_bit_cast(uint16_t, h);
}

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

// ---- the per-workgroup pool engine ------------------------------------------------
// SMALL: pools with L < 256, launched with BD = L threads and NQ = 1.
// DB: two LDS pool buffers; a pass reads one and writes the other, so it needs
// one barrier instead of two (twice the LDS).
//
// Barrier discipline: every LDS pool write is followed by a barrier before the
// pool is read again; sumsq() ends with a barrier that also publishes the pool
// writes before it.  Two sumsq() calls must be separated by a barrier (the
// second one rewrites the partial-sum slots the first one's readers use).
template <typename T, int NQ, bool SMALL, bool DB>
struct Engine {
  T *cur;       // LDS buffer holding the pool
  T *nxt;       // LDS buffer the next pass writes (== cur unless DB)
  double *red;  // LDS, 4 partial sums
  uint32_t L;
  uint32_t tid;
  T y[NQ][4];  // y[c][m] = element m*L + c*BD + tid

  __device__ __forceinline__ uint32_t bd() const { return SMALL ? L : kBlock; }

  __device__ __forceinline__ uint32_t pos(int m, int c) const {
    return uint32_t(m) * L + uint32_t(c) * bd() + tid;
  }

  __device__ __forceinline__ void load_global(const T *__restrict__ g) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const T v = g[pos(m, c)];
        y[c][m] = v;
        cur[pos(m, c)] = v;
      }
  }

  __device__ __forceinline__ void load_lds() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) y[c][m] = cur[pos(m, c)];
  }

  __device__ __forceinline__ void store_global(T *__restrict__ g) const {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) g[pos(m, c)] = y[c][m];
  }

  // write the registers to the buffer holding the pool
  __device__ __forceinline__ void write_lds() {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) cur[pos(m, c)] = y[c][m];
  }

  // y <- T(double(y) * g)
  __device__ __forceinline__ void scale(double g) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) y[c][m] = T(__dmul_rn(double(y[c][m]), g));
  }

  template <int K>
  __device__ __forceinline__ void gather_transform(const PassParams &p, bool renorm, double g) {
    T x[NQ][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint32_t a = p.alpha[m];
      const uint32_t base = __umul24(a, tid) + p.gamma[m];
      const uint32_t step = a * bd();
#pragma unroll
      for (int c = 0; c < NQ; ++c)
        x[c][m] = cur[uint32_t(m) * L + ((base + step * uint32_t(c)) & (L - 1))];
    }
    if (renorm) {
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NQ; ++c) x[c][m] = T(__dmul_rn(double(x[c][m]), g));
    }
#pragma unroll
    for (int c = 0; c < NQ; ++c) quad<K>(x[c][0], x[c][1], x[c][2], x[c][3], y[c]);
  }

  // One pass: gather from the LDS pool, transform, write the new pool.  The
  // caller places a barrier before the next read of the pool.  `renorm`
  // applies the renormalisation scale g to every gathered value first (each
  // element is gathered exactly once per pass, so this equals rescaling the
  // whole pool before the pass).
  __device__ __forceinline__ void pass(const PassParams &p, bool renorm, double g) {
    switch (p.k) {
      case 0: gather_transform<0>(p, renorm, g); break;
      case 1: gather_transform<1>(p, renorm, g); break;
      case 2: gather_transform<2>(p, renorm, g); break;
      default: gather_transform<3>(p, renorm, g); break;
    }
    if (!DB) __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) nxt[pos(m, c)] = y[c][m];
    if (DB) {
      T *t = cur;
      cur = nxt;
      nxt = t;
    }
  }

  // Sum of squares of the pool held in y: running sum over this thread's
  // elements in increasing index order, then a balanced pairwise tree over
  // the BD threads (lanes by xor butterflies, then the waves).  Ends with a
  // barrier; every thread returns the same value.
  __device__ __forceinline__ double sumsq() {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) acc = sq_add(acc, y[c][m]);
    const uint32_t B = bd();
    const uint32_t wl = B < 64 ? B : 64;
    for (uint32_t w = 1; w < wl; w <<= 1) acc = __dadd_rn(acc, __shfl_xor(acc, int(w)));
    if (B > 64 && (tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (B == 128) return __dadd_rn(red[0], red[1]);
    if (B == 256) return __dadd_rn(__dadd_rn(red[0], red[1]), __dadd_rn(red[2], red[3]));
    return acc;
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

  // Emit pool positions [lo, hi) scaled by fT to out[obase + (i - lo)].
  template <bool NT, typename O>
  __device__ __forceinline__ void emit(O *__restrict__ out, uint64_t obase, uint32_t lo,
                                       uint32_t hi, T fT) const {
    if (lo == 0 && hi == 4 * L - 1) {
      // a whole pool: every position but the withheld last one
      O *dst = out + obase + tid;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int c = 0; c < NQ; ++c) {
          const O v = Cast<O>::from(T(y[c][m] * fT));
          if (m < 3 || c < NQ - 1 || tid < bd() - 1)
            put<NT>(dst + (uint32_t(m) * L + uint32_t(c) * bd()), v);
        }
      return;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const uint32_t i = pos(m, c);
        if (i >= lo && i < hi) put<NT>(out + (obase + (i - lo)), Cast<O>::from(T(y[c][m] * fT)));
      }
  }
};

template <typename T, int NQ, bool SMALL, bool DB>
__device__ __forceinline__ Engine<T, NQ, SMALL, DB> make_engine(unsigned char *smem, uint32_t n) {
  Engine<T, NQ, SMALL, DB> e;
  e.cur = reinterpret_cast<T *>(smem);
  e.nxt = DB ? e.cur + n : e.cur;
  e.red = reinterpret_cast<double *>(smem + size_t(n) * sizeof(T) * (DB ? 2 : 1));
  e.L = n / 4;
  e.tid = threadIdx.x;
  return e;
}

__device__ __forceinline__ void flag_fault(uint32_t *err, double Q) {
  if (!(Q > 0.0) || !(Q < __builtin_huge_val())) atomicOr(err, 1u);
}

// ---- seeding (Section 5.8: the uniform source initialises the pool) ----------------
template <typename T, int NQ, bool SMALL>
__global__ __launch_bounds__(kBlock) void k_seed(SeedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint64_t xs_shared;
  const uint32_t s = a.streams[blockIdx.x];
  const uint32_t n = a.c.n;
  auto e = make_engine<T, NQ, SMALL, false>(smem, n);
  StreamHdr *h = a.c.hdr + s;

  // Initial values from the top 23 bits of successive uniforms:
  // ((v >> 41) - 2^22 + 1/2) * 2^-22, exact in binary32.
  if (e.tid == 0) {
    uint64_t xs = stream_seed(a.seed, s);
    for (uint32_t i = 0; i < n; ++i) {
      const uint64_t v = xs_next(xs);
      const double c = __dadd_rn(double(int64_t(v >> 41) - (int64_t(1) << 22)), 0.5);
      e.cur[i] = T(__dmul_rn(c, 0x1p-22));
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
    e.pass(decode(u1, u2, e.L), false, 1.0);
    __syncthreads();
  }
  Q = e.sumsq();
  e.scale(__dsqrt_rn(__ddiv_rn(nd, Q)));
  e.write_lds();
  __syncthreads();
  Q = e.sumsq();
  if (e.tid == 0) flag_fault(a.c.err, Q);
  const double last = double(e.cur[n - 1]);

  e.store_global(reinterpret_cast<T *>(a.c.arena + h->pool_off));
  if (e.tid == 0) {
    h->xs = xs;
    h->k = 0;
    h->f = 1.0;
    h->xnext = last;
    h->qlast = Q;
    h->n = n;
    h->cursor = n - 1;
  }
}

// ---- generation ---------------------------------------------------------------------
// Work item: continue stream s for `count` values written from out[obase].
// Pool production (Section 5.5): optional renormalisation every K pools with
// the previous sum of squares, R passes, binary64 sum of squares Q, a
// chi-square sample S from the previous pool's withheld scaled value,
// f = sqrt(S / Q); the n-1 first positions are emitted as T(P[i] * T(f)) and
// the withheld value f * P[n-1] feeds the next sample.  The stored pool is
// never scaled.
template <typename T, typename O, int NQ, bool SMALL, bool DB, bool NT, int WPE>
__global__ __launch_bounds__(kBlock, WPE) void k_fill(FillArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t j = blockIdx.x;
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

  const uint32_t n = a.c.n;
  auto e = make_engine<T, NQ, SMALL, DB>(smem, n);
  StreamHdr *h = a.c.hdr + s;
  uint64_t xs = h->xs;
  uint64_t k = h->k;
  double f = h->f;
  double xnext = h->xnext;
  double qlast = h->qlast;
  uint32_t cursor = h->cursor;
  T *gpool = reinterpret_cast<T *>(a.c.arena + h->pool_off);
  O *out = reinterpret_cast<O *>(a.out);

  e.load_global(gpool);
  __syncthreads();

  if (cursor < n - 1) {
    const uint32_t take = count < uint64_t(n - 1 - cursor) ? uint32_t(count) : n - 1 - cursor;
    e.template emit<NT>(out, obase, cursor, cursor + take, T(f));
    obase += take;
    count -= take;
    cursor += take;
  }

  const double nd = double(n);
  while (count > 0) {
    const bool renorm = k > 0 && a.c.K > 0 && (k % a.c.K) == 0;
    const double g = renorm ? __dsqrt_rn(__ddiv_rn(nd, qlast)) : 1.0;
    for (uint32_t r = 0; r < a.c.R; ++r) {
      const uint64_t u1 = xs_next(xs);
      const uint64_t u2 = xs_next(xs);
      e.pass(decode(u1, u2, e.L), renorm && r == 0, g);
      if (r + 1 < a.c.R) __syncthreads();
    }
    const double Q = e.sumsq();
    const double last = double(e.cur[n - 1]);
    double fk = 1.0;
    if (a.c.chi2 != kChi2Off) fk = __dsqrt_rn(__ddiv_rn(chi2_sample(a.c.cc, a.c.chi2, xnext), Q));
    if (e.tid == 0) flag_fault(a.c.err, Q);
    f = fk;
    xnext = __dmul_rn(fk, last);
    qlast = Q;
    k += 1;
    const uint32_t take = count < uint64_t(n - 1) ? uint32_t(count) : n - 1;
    e.template emit<NT>(out, obase, 0, take, T(f));
    obase += take;
    count -= take;
    cursor = take;
  }

  e.store_global(gpool);
  if (e.tid == 0) {
    h->xs = xs;
    h->k = k;
    h->f = f;
    h->xnext = xnext;
    h->qlast = qlast;
    h->cursor = cursor;
  }
}

// ---- dispatch ------------------------------------------------------------------------
size_t lds_bytes(uint32_t n, bool pool_f64, bool db) {
  return size_t(n) * (pool_f64 ? 8 : 4) * (db ? 2 : 1) + 4 * sizeof(double);
}

template <typename Kern>
hipError_t prepare(Kern kern, size_t lds) {
  if (lds > 65536)
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  return hipSuccess;
}

template <typename T, int NQ, bool SMALL>
hipError_t seed_t(const SeedArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes(a.c.n, sizeof(T) == 8, false);
  auto kern = k_seed<T, NQ, SMALL>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : kBlock;
  hipLaunchKernelGGL(kern, dim3(a.nstreams), dim3(block), lds, st, a);
  return hipGetLastError();
}

template <typename T, typename O, int NQ, bool SMALL, bool DB, bool NT, int WPE = 1>
hipError_t fill_t(const FillArgs &a, hipStream_t st) {
  const size_t lds = lds_bytes(a.c.n, sizeof(T) == 8, DB);
  auto kern = k_fill<T, O, NQ, SMALL, DB, NT, WPE>;
  hipError_t e = prepare(kern, lds);
  if (e != hipSuccess) return e;
  const uint32_t block = SMALL ? a.c.n / 4 : kBlock;
  hipLaunchKernelGGL(kern, dim3(a.nitems), dim3(block), lds, st, a);
  return hipGetLastError();
}

// Non-semantic variants (identical results): bit 0 double-buffered LDS,
// bit 1 nontemporal output stores, bit 2 at most 64 VGPRs (8 waves per SIMD).  Binary32 pools of 1024..8192 values have
// all four; every other shape runs variant 0.
template <typename T, typename O, int NQ>
hipError_t fill_v(const FillArgs &a, hipStream_t st) {
  if constexpr (sizeof(T) == 4 && NQ <= 8) {
    switch (a.variant & 7u) {
      case 1: return fill_t<T, O, NQ, false, true, false>(a, st);
      case 2: return fill_t<T, O, NQ, false, false, true>(a, st);
      case 3: return fill_t<T, O, NQ, false, true, true>(a, st);
      case 4: return fill_t<T, O, NQ, false, false, false, 8>(a, st);
      case 5: return fill_t<T, O, NQ, false, true, false, 8>(a, st);
      default: break;
    }
  }
  return fill_t<T, O, NQ, false, false, false>(a, st);
}

template <typename T>
hipError_t seed_n(const SeedArgs &a, hipStream_t st) {
  switch (a.c.n) {
    case 1024: return seed_t<T, 1, false>(a, st);
    case 2048: return seed_t<T, 2, false>(a, st);
    case 4096: return seed_t<T, 4, false>(a, st);
    case 8192: return seed_t<T, 8, false>(a, st);
    case 16384: return seed_t<T, 16, false>(a, st);
    default: return seed_t<T, 1, true>(a, st);
  }
}

template <typename T, typename O>
hipError_t fill_n(const FillArgs &a, hipStream_t st) {
  switch (a.c.n) {
    case 1024: return fill_v<T, O, 1>(a, st);
    case 2048: return fill_v<T, O, 2>(a, st);
    case 4096: return fill_v<T, O, 4>(a, st);
    case 8192: return fill_v<T, O, 8>(a, st);
    case 16384: return fill_v<T, O, 16>(a, st);
    default: return fill_t<T, O, 1, true, false, false>(a, st);
  }
}

}  // namespace

hipError_t launch_seed(const SeedArgs &a, bool pool_f64, hipStream_t s) {
  if (a.nstreams == 0) return hipSuccess;
  return pool_f64 ? seed_n<double>(a, s) : seed_n<float>(a, s);
}

hipError_t launch_fill(const FillArgs &a, bool pool_f64, uint32_t out_dtype, hipStream_t s) {
  if (a.nitems == 0) return hipSuccess;
  if (pool_f64) {
    switch (out_dtype) {
      case kOutF64: return fill_n<double, double>(a, s);
      case kOutF32: return fill_n<double, float>(a, s);
      case kOutBF16: return fill_n<double, Bf16>(a, s);
      default: return fill_n<double, Half>(a, s);
    }
  }
  switch (out_dtype) {
    case kOutF32: return fill_n<float, float>(a, s);
    case kOutBF16: return fill_n<float, Bf16>(a, s);
    case kOutF16: return fill_n<float, Half>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wn
