"""Measure every workload configuration on the GPU and print one JSON object.

    python -m paper_1005_2314_amd.report [--skip NAME ...]

Workloads (shapes in paper_1005_2314_amd.inputs):
  plain       one stream, pool 1024 binary64, one pass per pool, 2^20 binary64
  batched     65536 streams x 2^14, pool 4096 binary32, two passes
  uneven      10000 streams, log-uniform counts, pools 1024/2048/4096, one
              persistent launch, default and autotuned launch choices
  precision   16384 streams x 2^16, pool 4096, two passes: binary32 and binary64
              pools, binary32/bf16/f16 outputs (timings; the errors against
              the binary64 reference are measured by the GPU tests)
  quality     262144 streams x 2^18 (2^36 values), pool 4096 binary32, two
              passes, in 4 chunks with fused statistics

Timings use HIP events on the launch stream (median of repeats).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _time(fn, stream, reps=3, warmup=2):
    """Mean duration (ms) of fn() over `reps` calls enqueued back to back on
    `stream` after untimed ones (steady state, as continuing calls run): `warmup`
    calls, then as many as keep the GPU busy for about 50 ms more, since the
    first calls after an idle host phase run slower while the clocks settle."""
    import torch
    for _ in range(warmup):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
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


def plain(W, inputs, stream):
    import torch
    w = inputs.plain_f64()
    g = W.Generator(1, pool_n=w["pool_n"], R=w["R"], pool_dtype=W.WN_F64)
    g.seed(w["seed"])
    out = torch.empty(int(w["counts"][0]), dtype=torch.float64, device="cuda")
    ms = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream)
    g.close()
    return {"ms": ms, "normals_per_s": out.numel() / ms * 1e3}


def batched(W, inputs, stream):
    import torch
    w = inputs.batched_f32()
    g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"])
    t0 = time.perf_counter()
    g.seed(w["seed"])
    torch.cuda.synchronize()
    seed_ms = (time.perf_counter() - t0) * 1e3
    out = torch.empty(int(w["counts"].sum()), dtype=torch.float32, device="cuda")
    ms_default = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream, reps=5)
    t = g.autotune(out, w["streams"], w["counts"], stream)
    ms = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream, reps=5)
    res = {"ms": ms, "normals_per_s": out.numel() / ms * 1e3, "seed_ms": seed_ms,
           "ms_default_tuning": ms_default,
           "tuning": {"lds_double_buffer": t.lds_double_buffer,
                      "waves_per_simd": t.waves_per_simd}}
    for dt, name in ((W.WN_BF16, "bf16"), (W.WN_F16, "f16")):
        o16 = torch.empty(out.numel(), dtype=W.torch_dtype(dt), device="cuda")
        m = _time(lambda: g.fill_into(o16, w["streams"], w["counts"], stream), stream, reps=5)
        res[f"{name}_out"] = {"ms": m, "normals_per_s": out.numel() / m * 1e3}
        del o16
    g.close()
    return res


def uneven(W, inputs, stream):
    import numpy as np
    import torch
    w = inputs.uneven()
    g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"])
    g.seed(w["seed"])
    total = int(w["counts"].sum())
    out = torch.empty(total, dtype=torch.float32, device="cuda")
    ms_default = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream)
    t = g.autotune(out, w["streams"], w["counts"], stream)
    ms_tuned = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream)
    # the chain of one stream alone: the longest request of each pool size (a
    # small pool costs more per value, so the longest request is not always the
    # longest chain)
    chains = []
    for n in np.unique(w["pool_n"]):
        idx = np.nonzero(w["pool_n"] == n)[0]
        j = int(idx[np.argmax(w["counts"][idx])])
        one = torch.empty(int(w["counts"][j]), dtype=torch.float32, device="cuda")
        ms_one = _time(lambda: g.fill_into(one, [j], [int(w["counts"][j])], stream), stream)
        chains.append({"stream": j, "pool_n": int(n), "count": int(w["counts"][j]),
                       "ms_alone": ms_one})
        del one
    g.close()
    return {"total_normals": total, "ms_default": ms_default, "ms_tuned": ms_tuned,
            "normals_per_s_tuned": total / ms_tuned * 1e3,
            "tuning": {"lds_double_buffer": t.lds_double_buffer,
                       "nontemporal_stores": t.nontemporal_stores,
                       "wgs_per_cu": t.wgs_per_cu, "use_graph": t.use_graph,
                       "long_priority_pct": t.long_priority_pct,
                       "defer_emission": t.defer_emission},
            "longest_chain_ms": max(c["ms_alone"] for c in chains),
            "longest_streams": chains}


def precision(W, inputs, stream):
    """Full-size timings of every pool/output type pair (the errors against the
    binary64 reference are measured by the GPU test suite)."""
    import torch
    w = inputs.precision()
    res = {}
    for pool in ("f32", "f64"):
        g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"],
                        pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32)
        g.seed(w["seed"])
        for odt, oname in ((W.WN_F32, "f32"), (W.WN_BF16, "bf16"), (W.WN_F16, "f16")):
            out = torch.empty(int(w["counts"].sum()), dtype=W.torch_dtype(odt), device="cuda")
            ms = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream)
            res[f"pool_{pool}_out_{oname}"] = {"ms": ms, "normals_per_s": out.numel() / ms * 1e3}
            del out
        g.close()
    return res


def quality(W, inputs, stream):
    import numpy as np
    import torch
    from scipy import special
    w = inputs.throughput_quality()
    g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"])
    g.seed(w["seed"])
    per = int(w["counts"][0])
    out = torch.empty(w["num_streams"] * per, dtype=torch.float32, device="cuda")
    bufs = [g.stats_buffer() for _ in range(w["chunks"])]
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for c in range(w["chunks"]):
        g.fill_stats_into(out, w["streams"], w["counts"], bufs[c], stream)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b)
    # the same chunks without statistics, for the cost of fusing them
    t_plain = _time(lambda: g.fill_into(out, w["streams"], w["counts"], stream), stream, reps=3)
    sts = [g.read_stats(x) for x in bufs]
    N = sum(s.count for s in sts)
    mom = [sum(s.moment[k] for s in sts) / N for k in range(4)]
    var = mom[1] - mom[0] ** 2
    kurt = (mom[3] - 4 * mom[0] * mom[2] + 6 * mom[0] ** 2 * mom[1] - 3 * mom[0] ** 4) / var ** 2
    hist = sum(np.ctypeslib.as_array(s.hist).astype(np.float64) for s in sts)
    edges = (np.arange(4097) - 2048) / 256.0
    p = np.diff(0.5 * special.erfc(-edges / math.sqrt(2)))
    expct = p * N
    keep = expct > 50
    chi2 = float(np.sum((hist[keep] - expct[keep]) ** 2 / expct[keep]))
    P = sum(s.pools for s in sts)
    tm = sum(s.t_sum for s in sts) / P
    tv = sum(s.t_sumsq for s in sts) / P - tm * tm
    pairs = sum(s.t_pairs for s in sts)
    corr = (sum(s.t_lag for s in sts) / pairs - tm * tm) / tv
    xpools = sum(s.x_pools for s in sts)
    xpairs = sum(s.x_pairs for s in sts)
    xrate = xpools / P
    xexp = pairs * xrate * xrate
    g.close()
    return {"normals": N, "ms_with_stats": ms, "normals_per_s_with_stats": N / ms * 1e3,
            "ms_per_chunk_without_stats": t_plain,
            "normals_per_s_without_stats": out.numel() / t_plain * 1e3,
            "mean": mom[0], "variance": var, "kurtosis": kurt,
            "skew": (mom[2] - 3 * mom[0] * mom[1] + 2 * mom[0] ** 3) / var ** 1.5,
            "hist_chi2": chi2, "hist_dof": int(np.count_nonzero(keep)) - 1,
            "pool_sum_mean_minus_nu": tm, "pool_sum_var_over_2nu": tv / (2 * (w["pool_n"] - 1)),
            "successive_pool_corr": corr, "pool_pairs": pairs,
            "extreme_threshold": W.extreme_threshold(w["pool_n"]), "extreme_pool_rate": xrate,
            "extreme_adjacent_pairs": xpairs, "extreme_adjacent_expected": xexp,
            "extreme_adjacent_z": (xpairs - xexp) / math.sqrt(xexp),
            "below": sum(s.below for s in sts), "above": sum(s.above for s in sts)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--skip", nargs="*", default=[])
    args = ap.parse_args()
    import torch

    from paper_1005_2314_amd import build as libbuild
    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    from paper_1005_2314_amd import inputs
    from paper_1005_2314_amd import wn as W
    stream = torch.cuda.current_stream()
    out = {"device": torch.cuda.get_device_name(0)}
    for name, fn in (("plain", plain), ("batched", batched), ("uneven", uneven),
                     ("precision", precision), ("quality", quality)):
        if name in args.skip:
            continue
        print(f"[report] {name} ...", file=sys.stderr, flush=True)
        out[name] = fn(W, inputs, stream)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
