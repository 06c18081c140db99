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
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall time of the timed oracle baseline calls")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the other workload configurations")
    return ap.parse_args()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_fill_batched_f32_hbm_traffic.md")
FILL_SOURCES = [os.path.join(ROOT, "paper_1005_2314_amd", "csrc", f)
                for f in ("wn_device.hpp", "wn_launch.hpp", "wn_launch_f32_f32.hip",
                          "wn_internal.hpp")]


def measured_traffic():
    """HBM bytes per launch of the generation kernel from the committed
    FETCH_SIZE/WRITE_SIZE profile, or None when the kernel sources have changed
    since the counters were taken."""
    import hashlib
    try:
        fields = dict(line.split(": ", 1) for line in open(TRAFFIC_PROFILE).read().splitlines()
                      if ": " in line and line.split(": ", 1)[0].isidentifier())
        h = hashlib.sha256()
        for f in FILL_SOURCES:
            h.update(open(f, "rb").read())
        if h.hexdigest() != fields.get("source_sha256", "").strip():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def workload_bytes(w, out_bytes_per_value):
    """Algorithmic HBM bytes of one fill: outputs written plus each stream's state
    (pool and 64-byte header) read once and written once."""
    n_streams = int(w["num_streams"])
    values = int(w["counts"].sum())
    state = n_streams * (2 * (w["pool_n"] * 4) + 2 * 64)
    return values * out_bytes_per_value, state


def cpu_baseline(w, target_seconds):
    """The oracle, untuned, on all host cores (OpenMP over streams), over a bounded
    sample of the workload's streams: one untimed call seeds them, then continuing
    calls of the same per-stream count are timed until `target_seconds` of wall
    time have passed, as the GPU steps continue their streams."""
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
    # at most the whole workload, at least one call of about a second
    k = int(min(w["num_streams"], max(m, rate * 1.0 / per)))
    g = O.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"], pool_dtype="f32")
    g.seed(w["seed"])
    streams = np.arange(k, dtype=np.uint32)
    g.fill(streams, [per] * k)
    calls = 0
    t0 = time.perf_counter()
    while True:
        g.fill(streams, [per] * k)
        calls += 1
        dt = time.perf_counter() - t0
        if dt >= target_seconds:
            break
    # the same on one core: 16 of the streams, about two seconds
    k1 = min(k, 16)
    g.fill(streams[:k1], [per] * k1, threads=1)
    calls1 = 0
    t1 = time.perf_counter()
    while True:
        g.fill(streams[:k1], [per] * k1, threads=1)
        calls1 += 1
        dt1 = time.perf_counter() - t1
        if dt1 >= 2.0:
            break
    g.fill(streams[:0], [], threads=threads)  # the oracle's thread count back to all cores
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": calls * k * per / dt, "unit": "normals/s", "cores": threads,
            "kind": "oracle", "cpu": cpu,
            "sample": f"streams 0..{k - 1} of {w['num_streams']} (pool 4096 f32, R=2): "
                      f"{calls} continuing calls of {per} values per stream after an untimed "
                      f"seeding call, {dt:.1f} s wall on {threads} threads",
            "one_core": {"value": calls1 * k1 * per / dt1, "unit": "normals/s",
                         "sample": f"streams 0..{k1 - 1}: {calls1} continuing calls of {per} "
                                   f"values per stream, {dt1:.1f} s wall on 1 thread"}}


def time_launch(fn, stream, reps=3, warmup=1):
    """Median duration (ms) of fn() enqueued on `stream`, by HIP events on that stream."""
    import torch
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return sorted(ts)[len(ts) // 2]


def comparators(W, w, out, stream):
    """Reference points on the same GPU: HBM write ceilings, the generator's traffic
    with no arithmetic, the plain single-stream binary64 form, Box-Muller."""
    import ctypes as C

    import torch

    from paper_1005_2314_amd import inputs
    res = {}
    total = out.numel()
    st = C.c_void_p(stream.cuda_stream)
    optr = C.c_void_p(out.data_ptr())
    for name, code in (("store_ceiling_dwordx1", 1), ("store_ceiling_dwordx4", 4),
                       ("store_ceiling_runs_256KiB", 1 | 0x200)):
        ms = time_launch(lambda: W.wn_bench_store(optr, total * 4, code, st), stream)
        res[name] = {"ms": ms, "GB_per_s": total * 4 / ms / 1e6}
    n = w["pool_n"]
    state = torch.zeros(w["num_streams"] * (n * 4 + 64), dtype=torch.uint8, device=out.device)
    sptr = C.c_void_p(state.data_ptr())
    ms = time_launch(lambda: W.wn_bench_traffic(sptr, optr, w["num_streams"], n,
                                                int(w["counts"][0]), st), stream)
    out_b, state_b = workload_bytes(w, 4)
    res["traffic_ceiling"] = {"ms": ms, "GB_per_s": (out_b + state_b) / ms / 1e6,
                              "normals_per_s": total / ms * 1e3,
                              "what": "a plain streaming copy of the fill's bytes (pools and "
                                      "headers read and written, outputs written), no arithmetic"}
    del state
    for fast in (0, 1):
        ms = time_launch(lambda: W.wn_bench_box_muller(optr, total, W.WN_F32, 1, fast, st), stream)
        res["box_muller_philox_f32" + ("_fast" if fast else "")] = {
            "ms": ms, "normals_per_s": total / ms * 1e3, "GB_per_s": total * 4 / ms / 1e6}
    p = inputs.plain_f64()
    g = W.Generator(1, pool_n=p["pool_n"], R=p["R"], pool_dtype=W.WN_F64)
    g.seed(p["seed"])
    o64 = torch.empty(int(p["counts"][0]), dtype=torch.float64, device=out.device)
    ms = time_launch(lambda: g.fill_into(o64, p["streams"], p["counts"], stream), stream)
    res["plain_f64_single_stream"] = {"ms": ms, "normals_per_s": o64.numel() / ms * 1e3,
                                      "what": "1 stream, pool 1024 binary64, R=1, 2^20 binary64"}
    g.close()
    return res


def other_workloads(W, stream):
    """The other workload configurations, each timed in the launch form it runs in
    (steady state: untimed calls first, then the mean of back-to-back calls)."""
    import numpy as np
    import torch

    from paper_1005_2314_amd import inputs
    res = {}

    def steady(fn, reps=3):
        """Mean duration (ms) of `reps` calls back to back, after untimed calls
        that keep the GPU busy for about 50 ms (clocks settle after an idle
        host phase)."""
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        fn()
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        for _ in range(min(200, int(50.0 / max(a.elapsed_time(b), 0.05)))):
            fn()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / reps

    # plain single-stream binary64 form (one pool-1024 stream, one pass per pool)
    p = inputs.plain_f64()
    g = W.Generator(1, pool_n=p["pool_n"], R=p["R"], pool_dtype=W.WN_F64)
    g.seed(p["seed"])
    o = torch.empty(int(p["counts"][0]), dtype=torch.float64, device="cuda")
    ms = steady(lambda: g.fill_into(o, p["streams"], p["counts"], stream))
    res["plain_f64"] = {"config": "1 stream, pool 1024 binary64, R=1, 2^20 binary64 out",
                        "ms": ms, "normals_per_s": o.numel() / ms * 1e3}
    g.close()
    del o

    # uneven batch: one persistent launch replayed from a HIP graph; R from the
    # quality-constrained tuner (candidates 1, 2, 3 at 2^30 calibration values per
    # pool size), then the launch choices by the autotuner
    u = inputs.uneven()
    total = int(u["counts"].sum())
    o = torch.empty(total, dtype=torch.float32, device="cuda")
    base, keep = W.make_config(u["num_streams"], u["pool_n"], R=u["R"])
    chosen, report = W.tune_config(base, o, u["streams"], u["counts"], seed=u["seed"],
                                   passes=(1, 2, 3))
    R = chosen.passes_per_output
    entry = {"config": "10000 streams, log-uniform counts in [2^10, 2^22), pools 1024/2048/4096 "
                       "binary32, one persistent graph-replayed launch",
             "total_normals": total, "passes_chosen": R,
             "candidates": [{"R": c.R, "passed": bool(c.passed), "worst_z": c.worst_z,
                             "ms": c.ms} for c in report]}
    for r in sorted({R, 2}):
        g = W.Generator(u["num_streams"], pool_n=u["pool_n"], R=r)
        g.seed(u["seed"])
        t = g.autotune(o, u["streams"], u["counts"], stream)
        ms = steady(lambda: g.fill_into(o, u["streams"], u["counts"], stream))
        entry[f"R{r}"] = {"ms": ms, "normals_per_s": total / ms * 1e3,
                          "tuning": {"wgs_per_cu": t.wgs_per_cu, "group_items": t.group_items,
                                     "lds_double_buffer": t.lds_double_buffer,
                                     "long_priority_pct": t.long_priority_pct,
                                     "defer_emission": t.defer_emission}}
        g.close()
    entry["ms"] = entry[f"R{R}"]["ms"]
    entry["normals_per_s"] = entry[f"R{R}"]["normals_per_s"]
    res["uneven"] = entry
    del o, keep

    # precision workload: binary32 pools, 16-bit outputs
    q = inputs.precision()
    g = W.Generator(q["num_streams"], pool_n=q["pool_n"], R=q["R"])
    g.seed(q["seed"])
    entry = {"config": "16384 streams x 2^16, pool 4096 binary32 (and binary64: f64_pool_*), R=2; "
                       "launch choices by the autotuner per output type"}
    for dt, name in ((W.WN_BF16, "bf16"), (W.WN_F16, "f16"), (W.WN_F32, "f32")):
        o = torch.empty(int(q["counts"].sum()), dtype=W.torch_dtype(dt), device="cuda")
        t = g.autotune(o, q["streams"], q["counts"], stream)
        ms = steady(lambda: g.fill_into(o, q["streams"], q["counts"], stream))
        entry[f"{name}_out"] = {"ms": ms, "normals_per_s": o.numel() / ms * 1e3,
                                "tuning": {"lds_double_buffer": t.lds_double_buffer,
                                           "nontemporal_stores": t.nontemporal_stores,
                                           "waves_per_simd": t.waves_per_simd,
                                           "streams_per_wg": t.streams_per_wg}}
        del o
    g.close()
    # the same workload from binary64 pools
    g = W.Generator(q["num_streams"], pool_n=q["pool_n"], R=q["R"], pool_dtype=W.WN_F64)
    g.seed(q["seed"])
    for dt, name in ((W.WN_F64, "f64"), (W.WN_F32, "f32"), (W.WN_BF16, "bf16")):
        o = torch.empty(int(q["counts"].sum()), dtype=W.torch_dtype(dt), device="cuda")
        t = g.autotune(o, q["streams"], q["counts"], stream)
        ms = steady(lambda: g.fill_into(o, q["streams"], q["counts"], stream))
        entry[f"f64_pool_{name}_out"] = {"ms": ms, "normals_per_s": o.numel() / ms * 1e3,
                                         "tuning": {"lds_double_buffer": t.lds_double_buffer,
                                                    "threads_per_stream": t.threads_per_stream}}
        del o
    res["precision"] = entry
    g.close()

    # one chunk of the quality workload with fused statistics (and without)
    c = inputs.throughput_quality()
    g = W.Generator(c["num_streams"], pool_n=c["pool_n"], R=c["R"])
    g.seed(c["seed"])
    o = torch.empty(int(c["counts"].sum()), dtype=torch.float32, device="cuda")
    buf = g.stats_buffer()
    ms = steady(lambda: g.fill_stats_into(o, c["streams"], c["counts"], buf, stream), reps=2)
    ms0 = steady(lambda: g.fill_into(o, c["streams"], c["counts"], stream), reps=2)
    res["quality_chunk"] = {"config": "262144 streams x 2^16 (one of 4 chunks), pool 4096 "
                                      "binary32, R=2, fused statistics",
                            "ms_with_stats": ms, "normals_per_s_with_stats": o.numel() / ms * 1e3,
                            "ms_without_stats": ms0,
                            "normals_per_s_without_stats": o.numel() / ms0 * 1e3}
    g.close()
    del o
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (streams would "
              "shard across GPUs with no exchange, but only the one-GPU path exists)",
              file=sys.stderr)
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

    # the library's autotuner picks the launch variant for this request shape
    # (it restores the streams' state afterwards); outside the timed region
    tuned = g.autotune(out, w["streams"], w["counts"], stream)
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
        "metric": "normals/s and % HBM-write roofline, batched FP32 vs plain FP64 form",
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
                   "pool_n": w["pool_n"], "passes": w["R"], "seed_ms": seed_s * 1e3,
                   "tuning": {"lds_double_buffer": tuned.lds_double_buffer,
                              "nontemporal_stores": tuned.nontemporal_stores,
                              "waves_per_simd": tuned.waves_per_simd,
                              "streams_per_wg": tuned.streams_per_wg}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "k_fill (pool 4096 binary32, binary32 output)", "kernel_ms": avg_ms,
                     "bytes_per_launch": alg_bytes, "output_bytes": out_b,
                     "state_bytes": state_b,
                     "output_write_frac": out_b / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     # every call reads and writes each stream's pool: a third of the
                     # bytes here, so 70% of 8 TB/s in output writes alone would need
                     # output_write_frac * 8 TB/s * bytes_per_launch / output_bytes in all
                     "state_io_frac": state_b / alg_bytes},
    }
    if not args.no_comparators:
        rec["comparators"] = comparators(W, w, out, stream)
        ceil = rec["comparators"]["traffic_ceiling"]["ms"]
        rec["roofline"]["frac_of_traffic_ceiling"] = ceil / avg_ms
        # the metric's comparisons in one place: output writes as a share of the
        # 8 TB/s peak, and throughput against the plain single-stream binary64
        # form and both Box-Muller forms on the same GPU
        cmp = rec["comparators"]
        rec["headline"] = {
            "hbm_write_roofline_pct": 100.0 * rec["roofline"]["output_write_frac"],
            "hbm_roofline_pct_all_bytes": 100.0 * rec["roofline"]["frac"],
            "x_plain_f64_form": rec["value"] / cmp["plain_f64_single_stream"]["normals_per_s"],
            "x_box_muller_accurate": rec["value"] / cmp["box_muller_philox_f32"]["normals_per_s"],
            "x_box_muller_fast": rec["value"] / cmp["box_muller_philox_f32_fast"]["normals_per_s"]}
    if not args.no_workloads:
        del out
        torch.cuda.empty_cache()
        rec["workloads"] = other_workloads(W, stream)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
