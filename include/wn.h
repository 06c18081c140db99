/*
 * wn.h -- C ABI of the MI355X (gfx950) Wallace maximum-entropy normal
 * generator.
 *
 * Method: R. P. Brent, "Some Comments on C. S. Wallace's Random Number
 * Generators", Section 5 (5.1-5.8).  A pool of n normal variates is renewed by
 * passes of 4x4 orthogonal transforms (Section 5.3, the matrix A1 and its
 * sign variants) applied to quadruples chosen through affine row maps
 * (Section 5.4); after R passes the pool's sum of squares drives a scale factor
 * taken from an approximate chi-square sample (Section 5.5), n-1 scaled values
 * are returned and the last one is withheld for the next pool's sample.
 * The uniform source (Sections 3 and 5.8) is xorshift64, two draws per pass.
 *
 * All entry points are extern "C", take plain pointers and sizes, and never
 * throw or abort.  Every call returns a wn_status; wn_last_error() gives a
 * message for the calling thread's last failure.  Validation happens before
 * anything is enqueued: on any error nothing is enqueued and the generator's
 * state is unchanged.
 *
 * Asynchrony: wn_seed and wn_fill enqueue work on the given HIP stream (NULL =
 * the default stream) and return at once.  Successive calls on one generator
 * are ordered even across different streams (each call waits for the previous
 * call's completion event).  A wn_gen is not thread-safe.
 */
#ifndef WN_H
#define WN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wn_gen wn_gen; /* opaque; owned by the library */

typedef enum {
  WN_OK = 0,
  WN_EINVAL = 1,  /* bad argument or configuration */
  WN_ENOMEM = 2,  /* device or host allocation failed */
  WN_EDEVICE = 3, /* no usable device, a HIP call failed, or a fault reported by a kernel */
  WN_ESTATE = 4,  /* fill before seed */
  WN_ENOTSUP = 5  /* valid but unsupported combination */
} wn_status;

typedef enum { WN_F64 = 0, WN_F32 = 1, WN_BF16 = 2, WN_F16 = 3 } wn_dtype;

/* Chi-square approximation used for the rescale (Section 5.5).  CUBIC is the
 * A(x^2-1) + sqrt(2(nu-A^2)) x + nu form with A^3 - 3 nu A + 2 nu = 0; OFF keeps
 * the pool's constant sum of squares (the defect the rescale removes); FISHER
 * is 2 chi2 ~ (x + sqrt(2 nu - 1))^2; WH is the Wilson-Hilferty cube. */
typedef enum { WN_CHI2_CUBIC = 0, WN_CHI2_OFF = 1, WN_CHI2_FISHER = 2, WN_CHI2_WH = 3 } wn_chi2;

/* Where the chi-square sample of pool k takes its normal deviate x (Section
 * 5.5): PREVIOUS is the withheld, scaled last value of pool k-1 (fastnorm2,
 * the default); CURRENT is the last value of pool k itself (fastnorm's choice,
 * which couples the scale to the emitted sum of squares; kept as a control). */
typedef enum { WN_X_PREVIOUS = 0, WN_X_CURRENT = 1 } wn_chi2_source;

/* The orthogonal transform of a pass.  A4: the 4x4 matrices A1 D_k of
 * Section 5.3 (seven additions, one halving).  ROTATION: plane rotations
 * R(theta) with cos = (1-t^2)/(1+t^2), sin = 2t/(1+t^2) and t fixed per pass
 * (Section 5.3, the rann4 form).  A rotation pass treats the pool as two
 * rows of n/2, reads row r through q -> (alpha_r q + gamma_r) mod n/2 with odd
 * alpha_r (Section 5.4), draws t in [0, 1) from 24 bits and random signs for
 * cos and sin (Section 5.2), and writes (c a + s b, c b - s a) to position q
 * of the two rows.  Seeding runs 2 log2(n) + 4 warm-up passes instead of
 * log2(n) + 4: a pair-join grows dependency sets half as fast. */
typedef enum { WN_TRANSFORM_A4 = 0, WN_TRANSFORM_ROTATION = 1 } wn_transform;

/* The law of the values returned.  Section 5 names the exponential (E x = 1,
 * x >= 0) beside the normal as a maximum-entropy law but gives no transform
 * for it.  WN_EXPONENTIAL returns, for each pool, position j = m*(n/4) + q
 * (m = 0, 1; q a column of the pool's 4 rows of n/4) as ((a*a) + (b*b)) * 1/2
 * in the pool type, where a and b are the scaled normal values of rows m and
 * m+2 of column q: (a^2 + b^2)/2 is exactly Exp(1) for independent N(0,1) a
 * and b (chi-square with two degrees of freedom, halved).  The pairs are
 * disjoint and leave out only the withheld value and its partner, so a pool
 * gives n/2 - 1 values, and with the chi-square rescale their sum varies from
 * pool to pool like the maximum-entropy argument asks (Section 5.5).  Counts
 * and cursors are in values of the chosen law.  With WN_EXPONENTIAL, mean and
 * stddev must keep their defaults, emit_stride must be 1, and wn_fill_stats
 * (whose statistics are those of normal values) is not offered. */
typedef enum { WN_NORMAL = 0, WN_EXPONENTIAL = 1 } wn_variate;

typedef struct {
  uint32_t struct_size;       /* sizeof(wn_config), or WN_CONFIG_V1_SIZE (fields up to device)
                                 or WN_CONFIG_V2_SIZE (fields up to stddev) */
  uint32_t num_streams;       /* 1 .. 2^24; stream ids are 0 .. num_streams-1 */
  const uint32_t *pool_n;     /* host array [num_streams] of pool sizes, or NULL */
  uint32_t default_pool_n;    /* pool size when pool_n == NULL */
  uint32_t passes_per_output; /* R >= 1 passes between emitted pools (Section 5.7) */
  wn_dtype pool_dtype;        /* WN_F32 or WN_F64 */
  wn_chi2 chi2;               /* rescale mode */
  uint32_t renorm_period;     /* K: renormalise every K pools (0 = never) */
  int device;                 /* HIP device ordinal */
  /* version 2 */
  wn_chi2_source chi2_source; /* default WN_X_PREVIOUS */
  wn_transform transform;     /* default WN_TRANSFORM_A4 */
  double mean;                /* mu added to every output (0: none) */
  double stddev;              /* sigma > 0 folded into the scale (1: none) */
  /* version 3 */
  uint32_t emit_stride;       /* t in 1..16 (0 means 1): each stream returns every t-th value
                                 of its underlying sequence, starting with the first; the
                                 option of Section 5.7 that keeps only some of the values.  Pool
                                 statistics describe the underlying pools. */
  wn_variate variate;         /* WN_NORMAL (0, the default) or WN_EXPONENTIAL */
} wn_config;
#define WN_CONFIG_V1_SIZE 40u
#define WN_CONFIG_V2_SIZE 64u
/* Pool sizes are powers of two in [16, 16384].  The library copies the
 * configuration (and pool_n) during wn_create.  A shorter struct (size
 * WN_CONFIG_V1_SIZE or WN_CONFIG_V2_SIZE) gets the defaults of the fields it
 * lacks.  With mean mu and stddev
 * sigma, value i of pool k is T(P[i] * T(f_k * sigma)), plus T(mu) in the pool
 * type when mu != 0 (Section 5.5: sigma costs nothing, being folded into the
 * scale); sigma = 1, mu = 0 leave the generator's bits unchanged. */

/* Per-stream state as returned by wn_get_stream. */
typedef struct {
  uint64_t xs;     /* xorshift64 state */
  uint64_t k;      /* pools produced since seeding */
  uint32_t n;      /* pool size */
  uint32_t cursor; /* next pool position to emit; n-1 means the pool is used up */
  double f;        /* scale factor of the current pool */
  double xnext;    /* withheld, scaled value feeding the next chi-square sample */
  double qlast;    /* binary64 sum of squares of the current pool */
} wn_stream_info;

/* Launch choices that never change results (bit-exact across all settings);
 * an autotuner may pick them per workload. */
typedef struct {
  uint32_t struct_size;        /* sizeof(wn_tuning) */
  uint32_t lds_double_buffer;  /* 1: two LDS pool buffers, one barrier per pass */
  uint32_t nontemporal_stores; /* 1: output stores bypass cache retention */
  uint32_t waves_per_simd;     /* 0, or 5, 6 or 8: cap registers so that this many waves fit
                                  per SIMD (not with nontemporal; one-size launches only) */
  uint32_t wgs_per_cu;         /* persistent launches: workgroups per compute unit
                                  (0 = as many as can be resident), <= 16 */
  uint32_t use_graph;          /* 1: persistent launches replay a captured HIP graph */
  uint32_t long_priority_pct;  /* persistent launches: 0 = off; else the items whose estimated
                                  work (pools x (pool size + 4096)) is at least this percentage of the
                                  longest item's run at raised wave priority, so that the
                                  longest streams (the critical path) keep their pace while
                                  they share compute units; <= 100 (default 25) */
  uint32_t streams_per_wg;     /* one-size launches of consecutive streams with equal counts:
                                  each workgroup runs this many streams one after another
                                  (longer contiguous output runs); 1..16, default 1 */
  uint32_t defer_emission;     /* without statistics or thinning: each pool's scale and
                                  emission run inside the next pool's first pass, overlapping
                                  the pass's latency (a shorter chain of pools per stream; same
                                  results).  Bit 0: one-size launches of at most one stream per
                                  compute unit with pools of 1024 or 2048 values; bit 1: the
                                  items of 1024 and 2048 values of persistent launches whose
                                  pools are at most 4096.  0..3, default 1 */
  uint32_t group_items;        /* persistent launches without statistics, thinning or rotations,
                                  pools of at most 4096: 1 = the items of 1024 values outside the
                                  long-item head run in pairs, one per half of the workgroup
                                  (128 threads each), neighbours in length, in the plain loop
                                  (same results); default 0 */
  uint32_t threads_per_stream; /* without statistics, rotations, thinning or exponential
                                  variates: 128 or 256 threads per stream (0 = 256) in one-size
                                  launches of pools of 1024 to 4096 values and in persistent
                                  launches whose pools hold at most 2048; the same element
                                  layout m*L + c*threads + tid, column sums and tree (same
                                  results) */
} wn_tuning;

/* Validate cfg, select the device, allocate the per-stream state in device
 * memory (pools of n values, Section 5.1, and 64-byte headers) and compute the
 * chi-square constants of Section 5.5 on the host.  *out_gen receives the
 * generator (NULL on failure).
 * Errors: WN_EINVAL (cfg), WN_EDEVICE (no device / bad ordinal), WN_ENOMEM
 * (device or host allocation failed, e.g. a state arena larger than the
 * device memory; nothing stays allocated then). */
wn_status wn_create(const wn_config *cfg, wn_gen **out_gen);

/* Seed every stream: stream s starts from xorshift64 state = output s+1 of
 * SplitMix64 from `seed`, fills its pool from uniforms, renormalises, runs
 * log2(n)+4 warm-up passes and renormalises again (Section 5.8: the uniform
 * source serves for initialisation).  Enqueued on hip_stream. */
wn_status wn_seed(wn_gen *g, uint64_t seed, void *hip_stream);

/* Generate (Sections 5.1-5.5: R passes of the transforms per pool, the
 * chi-square rescale, n-1 values per pool returned and one withheld):
 * request j asks stream streams[j] for counts[j] values; outputs are
 * concatenated in request order into `out`, device memory owned by the caller
 * of at least sum(counts) elements of out_dtype.  streams/counts are host
 * arrays, read before the call returns.  Streams continue where the previous
 * call stopped: fill(s, a) then fill(s, b) equals fill(s, a + b) bit for bit,
 * and results never depend on batching, order or launch shape.
 * Requests of consecutive streams streams[j] = streams[0] + j with one count
 * and one pool size enqueue only kernels and event operations: such a call can
 * be captured into a HIP graph, and each replay continues the streams as a
 * call would (other request forms upload a work list and may wait on host
 * staging, so they are not for capture).
 * Errors: WN_EINVAL (null pointer with a non-zero count, stream id out of
 * range, a stream listed twice, more than 2^56 values in one call), WN_ESTATE
 * (not seeded), WN_ENOTSUP (WN_F64 output from a binary32 pool), WN_EDEVICE
 * (HIP failure). */
wn_status wn_fill(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                  void *out, wn_dtype out_dtype, void *hip_stream);

/* Statistics of the values one wn_fill_stats call emits (device memory,
 * written by the call).  Sums are binary64 in a fixed order that depends only
 * on the request (not on scheduling), so repeated runs give identical bits.
 * y is each value as stored in the output type.  For every pool k produced,
 * D_k = f_k^2 (Q_k - P_k[n-1]^2) - (n - 1) is the sum of squares of its n-1
 * emitted values (Section 5.5) minus its expected value; successive pools of a
 * stream form the lag pairs used to detect pool-to-pool correlation (Sections
 * 5.6, 5.7), also across calls, as long as both pools were produced by
 * wn_fill_stats (a wn_fill that produces a pool starts a new chain).  Centring keeps the lag-1 correlation
 * (t_lag/t_pairs - (t_sum/pools)^2) / variance well conditioned. */
typedef struct {
  uint64_t count;        /* values emitted */
  double moment[4];      /* sum of y, y^2, y^3, y^4 */
  uint64_t below, above; /* values with y < -8, y >= 8 */
  uint64_t pools;        /* pools produced */
  double t_sum, t_sumsq; /* sum of D_k and of D_k^2 over the pools produced */
  uint64_t t_pairs;      /* pools produced that have a predecessor in their stream */
  double t_lag;          /* sum of D_k * D_{k-1} over those pools */
  uint64_t hist[4096];   /* count of values with floor(256 y) + 2048 = bin, y in [-8, 8) */
  /* Adjacent-pool clustering of rare values (Section 5.7).  A pool holds an
   * extreme value when one of its n-1 emitted positions has
   * |T(P[i] T(f))| >= c_n (the standardised value in the pool type, before
   * mean and stddev; c_n from wn_extreme_threshold).  Under independence
   * x_pairs / t_pairs is about (x_pools / pools)^2; a finite pool makes it
   * larger, less so with more passes per emitted pool. */
  uint64_t x_pools;      /* pools produced that hold an extreme value */
  uint64_t x_pairs;      /* of the t_pairs pools, those that hold one after a pool that did */
} wn_stats;

/* The extreme-value threshold c_n of wn_stats for pools of n values: the
 * smallest multiple of 2^-8 with erfc(c_n / sqrt 2) <= 0.1 / n, so that about
 * one pool in ten holds such a value.  Host only; NaN for an unsupported n. */
double wn_extreme_threshold(uint32_t n);

/* The chi-square constants the generator uses for pools of n values (Section
 * 5.5; host only, no device needed).  out (6 doubles, caller-owned) receives
 * nu = n; A, the small root of A^3 - 3 nu A + 2 nu = 0 (eight Newton steps
 * from 2/3); b = sqrt(2 (nu - A^2)); the Fisher root sqrt(2 nu - 1); and the
 * Wilson-Hilferty scale sqrt(2 / (9 nu)) and shift 1 - 2 / (9 nu).
 * Errors: WN_EINVAL for a NULL out or a pool size the generator does not take
 * (out is then untouched). */
wn_status wn_chi2_constants(uint32_t n, double *out);

/* wn_fill plus fused statistics of the emitted values into `stats`
 * (caller-owned device memory, 8-byte aligned, sizeof(wn_stats); overwritten).
 * Same semantics and outputs as wn_fill; every count must be below 2^32.
 * Errors: as wn_fill; WN_EINVAL also for a NULL or misaligned stats pointer or
 * a count of 2^32 or more. */
wn_status wn_fill_stats(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                        void *out, wn_dtype out_dtype, wn_stats *stats, void *hip_stream);

/* wn_fill_stats for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): it
 * calls no hipMalloc, hipFree or other allocating routine.  Its per-request
 * partial sums live in one statically allocated device array of
 * WN_NOALLOC_MAX_REQUESTS entries of 96 bytes (6 MiB), which every device the
 * library runs on holds until the process ends; wn_create looks up its
 * address.  Results (outputs and statistics) are those of wn_fill_stats.
 * Restriction: the requests must take the form that needs no work list,
 * consecutive stream ids streams[j] = streams[0] + j with one count and one
 * pool size (one request always qualifies).  All calls on one device share the
 * array: calls that overlap on one device (different generators on different
 * streams) race; calls on one generator are ordered as usual.
 * Errors: as wn_fill_stats; WN_EINVAL also for nreq > WN_NOALLOC_MAX_REQUESTS,
 * WN_ENOTSUP for any other request form. */
#define WN_NOALLOC_MAX_REQUESTS 65536u
wn_status wn_fill_stats_noalloc(wn_gen *g, uint32_t nreq, const uint32_t *streams,
                                const uint64_t *counts, void *out, wn_dtype out_dtype,
                                wn_stats *stats, void *hip_stream);

/* The statistics battery (Sections 5.5-5.7) on one call's (or several
 * chained calls') wn_stats, host copy, for pools of pool_n values.  Each
 * statistic is in standard errors of N independent normal values: z[WN_Q_MEAN],
 * [WN_Q_VAR], [WN_Q_SKEW], [WN_Q_KURT] the first four moments; [WN_Q_HIST]
 * the histogram's chi-square against the normal law ((chi2 - dof) /
 * sqrt(2 dof); cells expecting fewer than 5 values merged with the tails);
 * [WN_Q_POOL_MEAN], [WN_Q_POOL_VAR] the pool sums D_k against chi-square with
 * n - 1 degrees of freedom; [WN_Q_POOL_LAG] the correlation of successive pool
 * sums times sqrt(pairs); [WN_Q_EXTREME_PAIRS] adjacent pools both holding an
 * extreme value against independence (Section 5.7; variance t_pairs p^2
 * (1 + 2p - 3p^2) for overlapping pairs).  passed = 1 when every |z| <= z_max,
 * the histogram and the clustering one-sided (only a worse fit than chance,
 * and only an excess of adjacent extreme pools, fail); failed_mask bit i marks
 * z[i].
 * A statistic that cannot be formed (no pairs) is 0.  Host only.
 * Errors: WN_EINVAL (NULL pointer, bad pool size, z_max <= 0, fewer than two
 * values or pools). */
enum {
  WN_Q_MEAN = 0, WN_Q_VAR, WN_Q_SKEW, WN_Q_KURT, WN_Q_HIST, WN_Q_POOL_MEAN, WN_Q_POOL_VAR,
  WN_Q_POOL_LAG, WN_Q_EXTREME_PAIRS, WN_QUALITY_NZ
};
typedef struct {
  double z[WN_QUALITY_NZ];
  uint32_t passed;
  uint32_t failed_mask;
} wn_quality;
wn_status wn_quality_check(const wn_stats *stats, uint32_t pool_n, double z_max, wn_quality *q);

/* Choose the semantic parameters, pool size n and passes per emitted pool R,
 * from the candidates that pass the statistics battery: Section 5.7 gives a
 * larger pool and discarded pools (R passes per emitted pool) as the remedies
 * for finite-pool effects, at a cost in speed.  For each candidate (n, R) (R
 * only, when base->pool_n gives per-stream sizes) a temporary generator with
 * base's other fields is seeded with `seed`; calib_values values per pool
 * size are drawn with wn_fill_stats (in calls that fit `out`) and judged by
 * wn_quality_check at z_max; each passing candidate then times the caller's
 * request (streams, counts, out_dtype; one untimed call, three timed back to
 * back on hip_stream).  *chosen receives base with the fastest passing (n, R):
 * create the generator from it, so that its values follow from that stated
 * configuration.  report[0 .. min(*nreport, report_cap)) receives every
 * candidate measured.  Synchronous; allocates temporary generators.
 * Errors: WN_EINVAL (arguments), WN_ENOTSUP (no candidate passed; *chosen
 * unchanged), and any error of the calls it makes. */
typedef struct {
  uint32_t struct_size;     /* sizeof(wn_quality_tuning) */
  uint32_t pool_sizes[8];   /* candidate pool sizes, 0-terminated (none: 1024, 2048, 4096) */
  uint32_t passes[8];       /* candidate R, 0-terminated (none: 1, 2, 3) */
  uint64_t calib_values;    /* values per candidate and pool size for the battery (0: 2^30) */
  double z_max;             /* every statistic within z_max standard errors (0: 5) */
} wn_quality_tuning;
typedef struct {
  uint32_t pool_n;          /* 0: the per-stream sizes of base */
  uint32_t R;
  uint32_t passed;          /* the battery passed for every pool size */
  uint32_t failed_mask;     /* union of wn_quality.failed_mask */
  double worst_z;           /* largest |z| (histogram and clustering one-sided) */
  float ms;                 /* time of the caller's request (0 if the candidate failed) */
  uint32_t reserved;
} wn_tune_candidate;
wn_status wn_tune_config(const wn_config *base, const wn_quality_tuning *opts, uint32_t nreq,
                         const uint32_t *streams, const uint64_t *counts, void *out,
                         wn_dtype out_dtype, uint64_t seed, void *hip_stream, wn_config *chosen,
                         wn_tune_candidate *report, uint32_t report_cap, uint32_t *nreport);

/* Wait for the generator's outstanding work and report a fault a kernel
 * flagged since the last check (a non-finite or zero sum of squares):
 * WN_EDEVICE with a message, else WN_OK. */
wn_status wn_sync(wn_gen *g);

/* Copy stream s's state to the host (synchronous).  pool_out (nullable)
 * receives n values of the pool type. */
wn_status wn_get_stream(wn_gen *g, uint32_t s, wn_stream_info *info, void *pool_out);

/* Set or read the generator's launch choices.  wn_set_tuning validates the
 * struct (WN_EINVAL on a bad size, a flag other than 0/1, waves_per_simd other
 * than 0/5/6/8 or set with nontemporal_stores, wgs_per_cu > 16,
 * long_priority_pct > 100, streams_per_wg outside 1..16, defer_emission > 3 or
 * group_items > 1)
 * and applies to later calls.  Binary32 pools of
 * 1024..8192 values have every choice; other shapes, and the plane-rotation
 * family (one launch variant), ignore them.  Defaults: the choices measured
 * fastest for binary32 pools on MI355X. */
wn_status wn_set_tuning(wn_gen *g, const wn_tuning *t);
wn_status wn_get_tuning(wn_gen *g, wn_tuning *t);

/* Autotune the launch choices for one request shape.  A measurement of a
 * candidate (LDS buffering, store kind, streams per workgroup, deferred
 * emission; for persistent launches grid size, long-item priority and pairs) runs the
 * request once untimed and three times back to back, timed with HIP events on
 * hip_stream, then restores the generator's state.  Every candidate is measured
 * twice (the better counts), the three fastest five more times each in turn,
 * and the one with the lowest median is kept.  The generator's state is unchanged on
 * return; `out` (same contract as wn_fill) is used as scratch and holds no
 * defined values afterwards.  *best (nullable) receives the choice, which is
 * also applied.  Synchronous.  Allocates a temporary copy of the state.
 * Errors: as wn_fill, plus WN_ENOMEM. */
wn_status wn_autotune(wn_gen *g, uint32_t nreq, const uint32_t *streams, const uint64_t *counts,
                      void *out, wn_dtype out_dtype, void *hip_stream, wn_tuning *best);

/* Checkpoints: the complete state of every stream (pools, uniform states,
 * scales, cursors) as a host byte buffer of wn_state_size(g) bytes.
 * wn_save_state copies it out after the generator's queued work; wn_load_state
 * restores it (the generator must have the same configuration; it counts as
 * seeded afterwards).  Restoring a saved state and repeating the same calls
 * reproduces their outputs bit for bit.  Both are synchronous.
 * Errors: WN_EINVAL (NULL buffer, wrong size, a state saved under another
 * configuration, or a stream header whose pool size, pool offset, cursor or
 * flags do not fit this generator; nothing is loaded then), WN_ESTATE (save
 * before seed), WN_EDEVICE. */
size_t wn_state_size(const wn_gen *g);
wn_status wn_save_state(wn_gen *g, void *host_buf, size_t bytes);
wn_status wn_load_state(wn_gen *g, const void *host_buf, size_t bytes);

/* Free everything the generator owns.  NULL-safe.  Waits for its work. */
void wn_destroy(wn_gen *g);

/* Message for the calling thread's last failed call ("" if none). */
const char *wn_last_error(void);

/* Library version, as major*10000 + minor*100 + patch. */
uint32_t wn_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WN_H */
