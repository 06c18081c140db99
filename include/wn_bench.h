/*
 * wn_bench.h -- measurement kernels shipped beside the generator in libwn.so.
 *
 * None of these is part of the generator.  They give the benchmark its
 * reference points on the same GPU:
 *   - wn_bench_store: the HBM write ceiling (a kernel that only writes);
 *   - wn_bench_traffic: the memory traffic of one generator fill without any
 *     arithmetic (read each stream's pool and header, write the outputs as
 *     one coalesced run per stream, write the pool and header back) -- the
 *     practical ceiling of the generator for that workload;
 *   - wn_bench_box_muller: a conventional normal generator for comparison
 *     (Section 4 of Brent's paper contrasts such transformation methods with
 *     Wallace's): the Box-Muller transform of Philox4x32-10 counter-based
 *     uniforms (Salmon, Moraes, Dror, Shaw, SC'11).
 * All are asynchronous on hip_stream and return a wn_status (wn.h).
 */
#ifndef WN_BENCH_H
#define WN_BENCH_H

#include <stdint.h>

#include "wn.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Write `bytes` (a multiple of 16) of zeros to device memory `dst` (16-byte
 * aligned).  width_dwords selects the store width per lane: 1 (dword) or 4
 * (dwordx4), in a grid-stride loop; adding 0x100 makes the stores
 * nontemporal; 1 | 0x200 writes dwords in runs of 256 KiB, each run by one
 * workgroup of a persistent grid of four workgroups per compute unit (the
 * fastest store pattern measured on MI355X).
 * Errors: WN_EINVAL (NULL dst, bytes not a multiple of 16, bad width),
 * WN_EDEVICE (launch failure). */
wn_status wn_bench_store(void *dst, uint64_t bytes, uint32_t width_dwords, void *hip_stream);

/* A plain streaming copy of a fill's bytes: for each of num_streams work
 * items (one workgroup each), read pool_n binary32 values and a 64-byte header
 * from `state` (num_streams * (pool_n*4 + 64) bytes, caller-owned), write
 * per_stream binary32 values to out (caller-owned, num_streams * per_stream
 * values) as consecutive coalesced words (each wave 64 words per
 * instruction), and write the pool and header back.  The bytes of the
 * generator's fill of that request with no arithmetic: its practical ceiling.
 * pool_n is a power of two in [1024, 16384].
 * Errors: WN_EINVAL (NULL pointers, bad pool_n), WN_EDEVICE. */
wn_status wn_bench_traffic(void *state, void *out, uint32_t num_streams, uint32_t pool_n,
                           uint64_t per_stream, void *hip_stream);

/* Box-Muller over Philox4x32-10: `count` (a multiple of 4) normals to out
 * (binary32 when out_dtype == WN_F32, binary64 when WN_F64).  Counter i/4 and
 * key (seed low, seed high) give four uniforms u = (x + 1/2) 2^-32, paired
 * into two (radius, angle) draws.  fast != 0 uses the hardware approximations
 * of log and sin/cos instead of the accurate library functions (binary32 only).
 * Errors: WN_EINVAL (NULL out, count not a multiple of 4, bad dtype),
 * WN_EDEVICE. */
wn_status wn_bench_box_muller(void *out, uint64_t count, wn_dtype out_dtype, uint64_t seed,
                              int fast, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* WN_BENCH_H */
