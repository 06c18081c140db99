"""Precision sweep: binary32 and binary64 pools, binary32/bf16/f16 outputs,
on sampled streams of the full precision workload (16384 streams x 2^16,
pool 4096, two passes, in the launch the workload runs): bit for bit against
the oracle of the same pool type, and within stated bounds of the binary64
oracle.

Bounds: a binary64 pool cast to the output type is the reference rounded once
more (bf16/f16 through binary32: at most one ulp of the output type); a
binary32 pool adds the binary32 rounding walk of the passes, bounded as in the
oracle's own test (8 sqrt(P) 2^-24 on values of unit size, P = passes since
seeding: the walk's standard deviation is below sqrt(P) 2^-24, and the largest
of the 4e5 values compared stays under 8.3 standard deviations except with
probability 1e-9), plus the output rounding.  The measured errors are written to
precision.json in the directory named by WN_REPORT_DIR, when it is set.
"""
import json
import math
import os

import numpy as np
import pytest

from gpu_util import WN_TO_ORC, assert_bits_equal, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import inputs
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu



def _widen(raw, oname):
    if oname == "bf16":
        return (raw.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if oname == "f16":
        return raw.view(np.float16).astype(np.float64)
    return raw.view({"f32": np.float32, "f64": np.float64}[oname]).astype(np.float64)


def _ulp(ref, oname):
    a = np.abs(ref)
    if oname == "f32":
        return np.spacing(a.astype(np.float32)).astype(np.float64)
    if oname == "f16":
        return np.spacing(a.astype(np.float16)).astype(np.float64)
    e = np.floor(np.log2(np.maximum(a, 2.0**-126)))
    return 2.0 ** (e - 7)  # bf16: 8 significant bits


def _moments(v):
    d = v - v.mean()
    var = float(np.mean(d * d))
    return [float(v.mean()), var, float(np.mean(d**3)) / var**1.5, float(np.mean(d**4)) / var**2]


def test_precision_sweep_against_binary64_oracle():
    import torch
    w = inputs.precision()
    sample = inputs.sample_streams(w["num_streams"], 6)
    per = int(w["counts"][0])
    ref = O.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"], pool_dtype="f64")
    ref.seed(w["seed"])
    y64 = ref.fill(sample, [per] * len(sample), O.F64)
    passes = int(math.log2(w["pool_n"])) + 4 + w["R"] * (per // (w["pool_n"] - 1) + 1)
    walk = 8.0 * math.sqrt(passes) * 2.0**-24
    report = {}
    for pool in ("f32", "f64"):
        g = W.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"],
                        pool_dtype=W.WN_F64 if pool == "f64" else W.WN_F32)
        same = O.Generator(w["num_streams"], pool_n=w["pool_n"], R=w["R"], pool_dtype=pool)
        for odt, oname in ((W.WN_F32, "f32"), (W.WN_BF16, "bf16"), (W.WN_F16, "f16")):
            print(f"precision: pool {pool} -> {oname}, full workload", flush=True)
            g.seed(w["seed"])
            out = g.fill(w["streams"], w["counts"], odt)
            torch.cuda.synchronize()
            got = torch.cat([out[int(s) * per:(int(s) + 1) * per] for s in sample])
            raw = to_numpy_bits(got)
            # bit for bit against the oracle of the same pool type
            same.seed(w["seed"])
            want = same.fill(sample, [per] * len(sample), WN_TO_ORC[odt])
            assert_bits_equal(raw, want.view(raw.dtype), f"pool {pool} -> {oname}")
            y = _widen(raw, oname)
            err = np.abs(y - y64)
            ulp = _ulp(y64, oname)
            if pool == "f64":
                bound = ulp  # one extra rounding (two for the 16-bit types, each <= 1/2 ulp)
            else:
                bound = ulp + walk
            assert np.all(err <= bound), (pool, oname, float(np.max(err / bound)))
            mg, mr = _moments(y), _moments(y64)
            report[f"pool_{pool}_out_{oname}"] = {
                "max_abs_err": float(err.max()), "max_ulp_err": float(np.max(err / ulp)),
                "moment_abs_err": [abs(a - b) for a, b in zip(mg, mr)],
                "sample": f"{len(sample)} streams x {per}"}
            del out
        g.close()
    outdir = os.environ.get("WN_REPORT_DIR", "")
    if outdir and os.path.isdir(outdir):
        with open(os.path.join(outdir, "precision.json"), "w") as fh:
            json.dump(report, fh, indent=1)
