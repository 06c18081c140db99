"""The quality-constrained choice of pool size and passes (wn_tune_config):
the chosen (n, R) is among the candidates that passed the statistics battery
and is the fastest of them; a candidate the paper predicts to fail (a 64-value
pool with one pass per pool clusters extreme values, Section 5.7) fails; and a
generator created from the returned configuration gives the oracle's bits for
that (n, R)."""
import numpy as np
import pytest

from gpu_util import assert_bits_equal, bits, to_numpy_bits
from oracle import oracle as O
from paper_1005_2314_amd import wn as W

pytestmark = pytest.mark.gpu

Q = {name: i for i, name in enumerate(W.WN_QUALITY_NAMES)}


def test_chosen_configuration_passes_and_matches_oracle():
    import torch
    ns, per = 2048, 1 << 12
    base, _ = W.make_config(ns, 4096, R=2)
    out = torch.empty(ns * per, dtype=torch.float32, device="cuda")
    streams, counts = np.arange(ns), np.full(ns, per)
    chosen, report = W.tune_config(base, out, streams, counts, seed=7, pool_sizes=(64, 1024),
                                   passes=(1, 3), calib_values=1 << 26)
    assert [(c.pool_n, c.R) for c in report] == [(64, 1), (64, 3), (1024, 1), (1024, 3)]
    by = {(c.pool_n, c.R): c for c in report}
    bad = by[(64, 1)]
    assert not bad.passed and bad.failed_mask & (1 << Q["extreme_pairs"]) and bad.ms == 0
    assert by[(64, 3)].passed
    passed = [c for c in report if c.passed]
    key = (chosen.default_pool_n, chosen.passes_per_output)
    assert key in {(c.pool_n, c.R) for c in passed}
    assert by[key].ms == min(c.ms for c in passed)
    assert chosen.num_streams == ns and chosen.chi2 == base.chi2
    # the values follow from the recorded configuration
    g = W.Generator(ns, pool_n=key[0], R=key[1])
    g.seed(7)
    sample = [0, 1000, ns - 1]
    y = g.fill(sample, [3 * per] * 3)
    torch.cuda.synchronize()
    orc = O.Generator(ns, pool_n=key[0], R=key[1])
    orc.seed(7)
    assert_bits_equal(to_numpy_bits(y), bits(orc.fill(sample, [3 * per] * 3)), "chosen config")
    g.close()


def test_mixed_pool_sizes_choose_passes_only():
    import torch
    sizes = np.array([1024, 2048] * 256, np.uint32)
    ns = sizes.size
    base, keep = W.make_config(ns, sizes, R=2)
    counts = np.random.default_rng(2).integers(1, 30000, ns).astype(np.uint64)
    out = torch.empty(int(counts.sum()), dtype=torch.float32, device="cuda")
    chosen, report = W.tune_config(base, out, np.arange(ns), counts, seed=3, passes=(2, 3),
                                   calib_values=1 << 24)
    assert [(c.pool_n, c.R) for c in report] == [(0, 2), (0, 3)]
    assert chosen.passes_per_output in (2, 3)
    assert report[chosen.passes_per_output - 2].passed
    del keep


def test_tune_rejects_bad_candidates():
    import torch
    base, _ = W.make_config(8, 1024)
    out = torch.empty(64, device="cuda")
    with pytest.raises(W.WnError) as e:
        W.tune_config(base, out, [0], [64], pool_sizes=(1000,))
    assert e.value.status == W.WN_EINVAL
    with pytest.raises(W.WnError) as e:
        W.tune_config(base, out, [0], [64], passes=(65,))
    assert e.value.status == W.WN_EINVAL
