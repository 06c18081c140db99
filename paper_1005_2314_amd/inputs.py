"""Seeded synthetic workloads (shapes of the generator's benchmark configs).

This module holds no arithmetic of the method: only the request shapes
(stream ids, counts, pool sizes) that both the GPU path and the CPU oracle are
given.  Every draw is seeded.
"""
import numpy as np


def plain_f64():
    """One stream, pool 1024 binary64, one pass per pool, 2^20 outputs (binary64)."""
    return dict(num_streams=1, pool_n=1024, R=1, pool="f64", out="f64", seed=1,
                streams=np.array([0], np.uint32), counts=np.array([1 << 20], np.uint64))


def batched_f32(num_streams=65536, per_stream=1 << 14):
    """65536 independent streams, pool 4096 binary32, two passes per pool,
    2^14 outputs per stream (2^30 total), binary32 output."""
    return dict(num_streams=num_streams, pool_n=4096, R=2, pool="f32", out="f32", seed=1,
                streams=np.arange(num_streams, dtype=np.uint32),
                counts=np.full(num_streams, per_stream, np.uint64))


def uneven(num_streams=10000, seed=2026):
    """10000 streams, counts floor(2^(10 + 12 U)) with U uniform on [0, 1) (log-uniform on
    [2^10, 2^22)), pool sizes uniform over {1024, 2048, 4096}; binary32 pools."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(num_streams)
    sizes = np.array([1024, 2048, 4096], np.uint32)[rng.integers(0, 3, num_streams)]
    counts = np.floor(2.0 ** (10 + 12 * u)).astype(np.uint64)
    return dict(num_streams=num_streams, pool_n=sizes, R=2, pool="f32", out="f32", seed=1,
                streams=np.arange(num_streams, dtype=np.uint32), counts=counts)


def precision(num_streams=16384, per_stream=1 << 16):
    """16384 streams x 2^16 outputs, pool 4096, two passes per pool."""
    return dict(num_streams=num_streams, pool_n=4096, R=2, seed=1,
                streams=np.arange(num_streams, dtype=np.uint32),
                counts=np.full(num_streams, per_stream, np.uint64))


def throughput_quality(num_streams=262144, per_stream=1 << 18, chunks=4):
    """262144 streams x 2^18 outputs (2^36 total), pool 4096, two passes, filled in
    `chunks` equal calls per stream."""
    return dict(num_streams=num_streams, pool_n=4096, R=2, pool="f32", out="f32", seed=1,
                streams=np.arange(num_streams, dtype=np.uint32),
                counts=np.full(num_streams, per_stream // chunks, np.uint64), chunks=chunks)


def sample_streams(num_streams, k, seed=11):
    """k distinct stream ids spread over [0, num_streams): the ends plus seeded picks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    picks = set([0, num_streams - 1])
    while len(picks) < min(k, num_streams):
        picks.add(int(rng.integers(0, num_streams)))
    return np.array(sorted(picks), np.uint32)
