"""Shared helpers of the GPU tests: run the same requests through the HIP
library (C ABI) and the CPU oracle and compare bit patterns."""
import numpy as np

from oracle import oracle as O
from paper_1005_2314_amd import wn as W

WN_TO_ORC = {W.WN_F64: O.F64, W.WN_F32: O.F32, W.WN_BF16: O.BF16, W.WN_F16: O.F16}


def bits(a):
    a = np.asarray(a)
    return a.view({8: np.uint64, 4: np.uint32, 2: np.uint16}[a.dtype.itemsize])


def to_numpy_bits(t):
    import torch
    t = t.detach().cpu()
    if t.dtype in (torch.bfloat16, torch.float16):
        return t.view(torch.int16).numpy().view(np.uint16)
    return bits(t.numpy())


class Pair:
    """A GPU generator and an oracle generator with the same configuration."""

    def __init__(self, num_streams, pool_n=1024, R=2, pool="f32", chi2=0, K=16, seed=1,
                 variate=0):
        pool_dtype = W.WN_F64 if pool == "f64" else W.WN_F32
        self.gpu = W.Generator(num_streams, pool_n=pool_n, R=R, pool_dtype=pool_dtype,
                               chi2=chi2, K=K, variate=variate)
        self.orc = O.Generator(num_streams, pool_n=pool_n, R=R, pool_dtype=pool, chi2=chi2, K=K,
                               variate=variate)
        self.gpu.seed(seed)
        self.orc.seed(seed)

    def fill(self, streams, counts, out_dtype=W.WN_F32, orc_streams=None):
        """Fill on both sides; the oracle serves `orc_streams` (default all requests)."""
        import torch
        y = self.gpu.fill(streams, counts, out_dtype)
        torch.cuda.synchronize()
        g = to_numpy_bits(y)
        streams = np.asarray(streams, np.uint32)
        counts = np.asarray(counts, np.uint64)
        if orc_streams is None:
            o = bits(self.orc.fill(streams, counts, WN_TO_ORC[out_dtype]))
            return g, o
        # sampled comparison: pick the slices of the chosen streams
        offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        sel = [int(np.nonzero(streams == s)[0][0]) for s in orc_streams]
        o = bits(self.orc.fill(streams[sel], counts[sel], WN_TO_ORC[out_dtype]))
        gs = np.concatenate([g[offs[j]: offs[j + 1]] for j in sel]) if sel else g[:0]
        return gs, o


def assert_bits_equal(g, o, what=""):
    assert g.shape == o.shape, (what, g.shape, o.shape)
    bad = np.nonzero(g != o)[0]
    if bad.size:
        i = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} of {g.size} values differ, first at {i}: "
                             f"gpu {g[i]:#x} oracle {o[i]:#x}")
