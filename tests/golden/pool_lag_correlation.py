"""Writes pool_lag_correlation.txt: the oracle's lag-1 correlation of successive
pool sums at n = 4096, R = 2 (the quality workload's configuration).

For each pool k of a stream, D_k = f_k^2 (Q_k - P_k[n-1]^2) - (n - 1) is the sum of
squares of its n - 1 emitted values minus its expected value (Section 5.5); the
statistic is corr(D_k, D_{k+1}) over all successive pairs within streams, the
quantity the GPU statistics report as t_lag.  Calls only oracle/; run as
    python tests/golden/pool_lag_correlation.py [streams] [values per stream] [seed] [calls]
(defaults 4096 streams x 4096 pools, seed 20261203, about 1.7e7 pools: two minutes on 8
cores; only the default run writes the file).  With 262144 streams x 2^18 values, seed 1
and 4 calls it computes the statistic of exactly the streams of the quality workload
(2^36 values in four chunks), which the GPU's fused statistics report for that workload.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from oracle import oracle as O  # noqa: E402


def main():
    n, R = 4096, 2
    ns = int(sys.argv[1]) if len(sys.argv) > 1 else 4096
    values = int(sys.argv[2]) if len(sys.argv) > 2 else 4096 * (n - 1)
    seed = int(sys.argv[3]) if len(sys.argv) > 3 else 20261203
    calls = int(sys.argv[4]) if len(sys.argv) > 4 else 256
    default = len(sys.argv) == 1
    pools = -(-values // (n - 1))  # pools produced per stream
    s1 = s2 = lag = 0.0
    npairs = npools = 0
    group = 256
    for s0 in range(0, ns, group):
        streams = np.arange(s0, min(ns, s0 + group), dtype=np.uint32)
        g = O.Generator(ns, pool_n=n, R=R, trace=True)
        g.seed(seed)
        for c in range(calls):  # values split over the calls (bf16 output, discarded)
            part = values // calls + (1 if c < values % calls else 0)
            g.fill(streams, [part] * len(streams), O.BF16)
        for s in streams:
            d = g.trace(int(s), pools + 8)[:, 4] - (n - 1)
            s1 += float(d.sum())
            s2 += float((d * d).sum())
            lag += float((d[1:] * d[:-1]).sum())
            npools += d.size
            npairs += d.size - 1
        del g
    mean = s1 / npools
    var = s2 / npools - mean * mean
    r = (lag / npairs - mean * mean) / var
    se = 1.0 / np.sqrt(npairs)
    text = (f"# oracle, n = {n}, R = {R}, seed {seed}: {ns} streams x {values} values "
            f"({pools} pools) in {calls} calls\n"
            f"pairs: {npairs}\n"
            f"mean_D: {mean:.6f}\n"
            f"var_D_over_2(n-1): {var / (2 * (n - 1)):.6f}\n"
            f"lag1_correlation: {r:.6e}\n"
            f"standard_error: {se:.3e}\n")
    if default:
        with open(os.path.join(HERE, "pool_lag_correlation.txt"), "w") as fh:
            fh.write(text)
    print(text, end="")


if __name__ == "__main__":
    main()
