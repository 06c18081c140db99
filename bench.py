"""Benchmark of batched binary32 Wallace generation on one MI355X.

A step is one wn_fill over the whole workload: 65536 independent streams, each
with a 4096-value binary32 pool, two passes per emitted pool, 2^14 values per
stream (2^30 binary32 normals, 4 GiB written).  Streams are seeded before the
timed region (seeding is timed separately) and continue across steps.

Prints one JSON line with throughput, the roofline of the generation kernel
(HIP events on the launch stream), and the CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def workload_bytes(w, out_bytes_per_value):
    """Algorithmic HBM bytes of one fill: outputs written plus each stream's state
    (pool and 64-byte header) read once and written once."""
    n_streams = int(w["num_streams"])
    values = int(w["counts"].sum())
    state = n_streams * (2 * (w["pool_n"] * 4) + 2 * 64)
    return values * out_bytes_per_value, state


def cpu_baseline(w, target_seconds):
    """The oracle, untuned, on all host cores, over a bounded sample of streams:
    one untimed call (it seeds the sampled streams), then one timed call of the
    same per-stream count, as the GPU steps continue their streams."""
    import numpy as np

    from oracle import oracle as O
    per = int(w["counts"][0])
    threads = O.max_threads()
    m = 16 * threads
    probe = O.Generator(m, pool_n=w["pool_n"], R=w["R"], pool_dtype="f32")
    probe.seed(w["seed"])
    probe.fill(np.arange(m), [per] * m)
    t0 = time.perf_counter()
    probe.fill(np.arange(m), [per] * m)
    rate = m * per / (time.perf_counter() - t0)
    del probe
    k = int(max(threads, min(w["num_streams"], rate * target_seconds / per)))
    k = max(threads, (k // threads) * threads)
    g = O.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"], pool_dtype="f32")
    g.seed(w["seed"])
    streams = np.arange(k, dtype=np.uint32)
    g.fill(streams, [per] * k)
    t0 = time.perf_counter()
    g.fill(streams, [per] * k)
    dt = time.perf_counter() - t0
    return {"value": k * per / dt, "unit": "normals/s", "cores": threads, "kind": "oracle",
            "sample": f"streams 0..{k - 1} of {w['num_streams']} (pool 4096 f32, R=2), "
                      f"one continuing call of {per} values each after an untimed call; "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (streams shard "
              "across GPUs with no exchange, but this build measures one GPU)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1005_2314_amd import build as libbuild
    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    from paper_1005_2314_amd import inputs
    from paper_1005_2314_amd import wn as W

    w = inputs.batched_f32()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"], pool_dtype=W.WN_F32)
    total = int(w["counts"].sum())
    out = torch.empty(total, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    g.seed(w["seed"])
    torch.cuda.synchronize()
    seed_s = time.perf_counter() - t0

    for _ in range(args.warmup):
        g.fill_into(out, w["streams"], w["counts"], stream)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        g.fill_into(out, w["streams"], w["counts"], stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.sync()
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_ms = sum(kern_ms) / len(kern_ms)

    out_b, state_b = workload_bytes(w, 4)
    alg_bytes = out_b + state_b
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    rec = {
        "metric": "normals/s, batched binary32 Wallace generation",
        "value": total * args.steps / wall,
        "unit": "normals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_f32: 65536 streams x 2^14 normals, pool 4096 binary32, "
                               "2 passes per pool, chi-square rescale, binary32 output",
                   "streams": w["num_streams"], "per_stream": int(w["counts"][0]),
                   "pool_n": w["pool_n"], "passes": w["R"], "seed_ms": seed_s * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_fill<float,float,4>", "kernel_ms": avg_ms,
                     "bytes_per_launch": alg_bytes, "output_bytes": out_b,
                     "state_bytes": state_b,
                     "output_write_frac": out_b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
