"""Seeded property sweep of the oracle (CPU): for random configurations
(pool sizes, one or mixed, pool type, passes, renormalisation period,
chi-square mode and source, transform family, variate, thinning, location and
scale), a stream's values do not depend on how its requests are split into
calls, on which other streams share a call, or on request order; and a
thinned stream is every t-th value of the same stream unthinned."""
import numpy as np
import pytest

from oracle import oracle as O

SIZES = [16, 64, 256, 1024, 2048]


def config(seed):
    rng = np.random.default_rng(seed)
    ns = int(rng.integers(2, 7))
    sizes = (rng.choice(SIZES, size=ns) if rng.random() < 0.5
             else np.full(ns, rng.choice(SIZES))).astype(np.uint32)
    variate = int(rng.random() < 0.25)
    kw = dict(R=int(rng.choice([1, 2, 3])), K=int(rng.choice([0, 1, 3, 16])),
              chi2=int(rng.choice([0, 1, 2, 3])), x_current=bool(rng.random() < 0.2),
              transform=int(rng.random() < 0.3), variate=variate,
              pool_dtype="f64" if rng.random() < 0.3 else "f32")
    if not variate and rng.random() < 0.3:
        kw["mean"], kw["stddev"] = 0.5, 2.0
    return rng, ns, sizes, kw


def make(ns, sizes, kw, seed, **extra):
    g = O.Generator(ns, pool_n=sizes, **kw, **extra)
    g.seed(seed)
    return g


@pytest.mark.parametrize("case", range(40))
def test_calls_batching_and_order_do_not_change_a_stream(case):
    rng, ns, sizes, kw = config(300 + case)
    total = [int(rng.integers(0, 4 * int(n))) for n in sizes]
    whole = make(ns, sizes, kw, case)
    want = {}
    for s in range(ns):  # one stream per call, all of it at once
        want[s] = whole.fill([s], [total[s]], O.F32)
    split = make(ns, sizes, kw, case)
    got = {s: [] for s in range(ns)}
    left = list(total)
    while any(left):
        order = rng.permutation(ns)
        streams, counts = [], []
        for s in order:
            if left[s] and rng.random() < 0.7:
                c = int(rng.integers(1, left[s] + 1))
                streams.append(int(s))
                counts.append(c)
                left[s] -= c
        if not streams:
            continue
        y = split.fill(streams, counts, O.F32)
        at = 0
        for s, c in zip(streams, counts):
            got[s].append(y[at:at + c])
            at += c
    for s in range(ns):
        g = np.concatenate(got[s]) if got[s] else np.zeros(0, np.float32)
        np.testing.assert_array_equal(g.view(np.uint32), want[s].view(np.uint32), err_msg=f"stream {s}")


@pytest.mark.parametrize("case", range(20))
def test_thinning_takes_every_t_th_value(case):
    rng, ns, sizes, kw = config(600 + case)
    kw["variate"] = 0
    t = int(rng.choice([2, 3, 5, 7, 16]))
    per = [int(rng.integers(0, 3 * int(n))) for n in sizes]
    plain = make(ns, sizes, kw, case)
    thin = make(ns, sizes, kw, case, emit_stride=t)
    for s in range(ns):
        full = plain.fill([s], [per[s] * t], O.F32)
        part = thin.fill([s], [per[s]], O.F32)
        np.testing.assert_array_equal(part.view(np.uint32), full[::t].view(np.uint32),
                                      err_msg=f"stream {s}, t={t}")
