"""ctypes wrapper of the CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  It never touches the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

F64, F32, BF16, F16 = 0, 1, 2, 3
CHI2_CUBIC, CHI2_OFF, CHI2_FISHER, CHI2_WH = 0, 1, 2, 3
HAZ_NONE, HAZ_GLOBAL_AFFINE, HAZ_IN_PLACE, HAZ_SHARED_MAP, HAZ_CURRENT_X = 0, 1, 2, 3, 4

_OUT_NP = {F64: np.float64, F32: np.float32, BF16: np.uint16, F16: np.uint16}


class _Config(C.Structure):
    _fields_ = [(name, C.c_uint32) for name in (
        "num_streams", "default_pool_n", "R", "pool_f64", "chi2", "K", "hazard", "warmup",
        "trace", "x_current", "transform", "emit_stride")] + [("mean", C.c_double),
                                                              ("stddev", C.c_double),
                                                              ("variate", C.c_uint32)]


class StreamInfo(C.Structure):
    _fields_ = [("xs", C.c_uint64), ("k", C.c_uint64), ("n", C.c_uint32),
                ("cursor", C.c_uint32), ("f", C.c_double), ("xnext", C.c_double),
                ("qlast", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path)
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        u16p = np.ctypeslib.ndpointer(np.uint16, flags="C")
        L.orc_xorshift64.argtypes = [C.POINTER(C.c_uint64), C.c_uint32, u64p]
        L.orc_xorshift64.restype = C.c_uint64
        L.orc_stream_state.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_stream_state.restype = C.c_uint64
        L.orc_decode.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.POINTER(C.c_int32),
                                 u32p, u32p]
        L.orc_gather_index.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, u32p]
        L.orc_pass_f32.argtypes = [f32p, C.c_uint32, C.c_int32, u32p, u32p, C.c_uint32]
        L.orc_pass_f64.argtypes = [f64p, C.c_uint32, C.c_int32, u32p, u32p, C.c_uint32]
        L.orc_transform_f64.argtypes = [f64p, C.c_int32, f64p]
        L.orc_decode_rotation.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, u32p, u32p, f64p]
        L.orc_rotation_pass_f32.argtypes = [f32p, C.c_uint32, u32p, u32p, C.c_double,
                                            C.c_double]
        L.orc_rotation_pass_f64.argtypes = [f64p, C.c_uint32, u32p, u32p, C.c_double,
                                            C.c_double]
        L.orc_warmup_passes.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_warmup_passes.restype = C.c_uint32
        L.orc_sumsq_f32.argtypes = [f32p, C.c_uint32]
        L.orc_sumsq_f32.restype = C.c_double
        L.orc_sumsq_f64.argtypes = [f64p, C.c_uint32]
        L.orc_sumsq_f64.restype = C.c_double
        L.orc_initial_pool_f32.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, f32p]
        L.orc_initial_pool_f32.restype = C.c_uint64
        L.orc_initial_pool_f64.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, f64p]
        L.orc_initial_pool_f64.restype = C.c_uint64
        L.orc_chi2_consts.argtypes = [C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.orc_chi2_sample.argtypes = [C.c_uint32, C.c_uint32, f64p, f64p, C.c_uint64]
        L.orc_cvt_bf16.argtypes = [f32p, u16p, C.c_uint64]
        L.orc_cvt_f16.argtypes = [f32p, u16p, C.c_uint64]
        L.orc_create.argtypes = [C.POINTER(_Config), C.c_void_p]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_seed.argtypes = [C.c_void_p, C.c_uint64]
        L.orc_fill.argtypes = [C.c_void_p, C.c_uint32, u32p, u64p, C.c_void_p, C.c_uint32,
                               C.c_int]
        L.orc_fill.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_stream_get.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(StreamInfo), C.c_void_p]
        L.orc_stream_get.restype = C.c_int
        L.orc_trace_get.argtypes = [C.c_void_p, C.c_uint32, f64p, C.c_uint64]
        L.orc_trace_get.restype = C.c_uint64
        L.orc_extreme_threshold.argtypes = [C.c_uint32]
        L.orc_extreme_threshold.restype = C.c_double
        _lib = L
    return _lib


# ---- low-level pieces -------------------------------------------------------

def xorshift64(state: int, count: int) -> np.ndarray:
    out = np.zeros(count, np.uint64)
    s = C.c_uint64(state)
    lib().orc_xorshift64(C.byref(s), count, out)
    return out


def stream_state(seed: int, stream: int) -> int:
    return int(lib().orc_stream_state(seed, stream))


def decode(u1: int, u2: int, L: int):
    k = C.c_int32()
    a = np.zeros(4, np.uint32)
    g = np.zeros(4, np.uint32)
    lib().orc_decode(u1, u2, L, C.byref(k), a, g)
    return int(k.value), a, g


def gather_index(u1: int, u2: int, n: int, hazard: int = HAZ_NONE) -> np.ndarray:
    idx = np.zeros(n, np.uint32)
    lib().orc_gather_index(u1, u2, n, hazard, idx)
    return idx


def run_pass(P: np.ndarray, k: int, alpha, gamma, hazard: int = HAZ_NONE) -> np.ndarray:
    P = np.array(P, copy=True)
    a = np.ascontiguousarray(alpha, np.uint32)
    g = np.ascontiguousarray(gamma, np.uint32)
    if P.dtype == np.float32:
        lib().orc_pass_f32(P, P.size, k, a, g, hazard)
    else:
        P = P.astype(np.float64)
        lib().orc_pass_f64(P, P.size, k, a, g, hazard)
    return P


def transform(x, k: int) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(4, np.float64)
    lib().orc_transform_f64(x, k, y)
    return y


TRANSFORM_A4, TRANSFORM_ROTATION = 0, 1


def decode_rotation(u1: int, u2: int, H: int):
    a = np.zeros(2, np.uint32)
    g = np.zeros(2, np.uint32)
    cs = np.zeros(2, np.float64)
    lib().orc_decode_rotation(u1, u2, H, a, g, cs)
    return a, g, float(cs[0]), float(cs[1])


def rotation_pass(P: np.ndarray, alpha, gamma, c: float, s: float) -> np.ndarray:
    P = np.array(P, copy=True)
    a = np.ascontiguousarray(alpha, np.uint32)
    g = np.ascontiguousarray(gamma, np.uint32)
    if P.dtype == np.float32:
        lib().orc_rotation_pass_f32(P, P.size, a, g, c, s)
    else:
        P = P.astype(np.float64)
        lib().orc_rotation_pass_f64(P, P.size, a, g, c, s)
    return P


def warmup_passes(n: int, transform: int = TRANSFORM_A4) -> int:
    return int(lib().orc_warmup_passes(n, transform))


def sumsq(P: np.ndarray) -> float:
    P = np.ascontiguousarray(P)
    if P.dtype == np.float32:
        return float(lib().orc_sumsq_f32(P, P.size))
    return float(lib().orc_sumsq_f64(np.ascontiguousarray(P, np.float64), P.size))


def initial_pool(seed: int, stream: int, n: int, pool_dtype: str = "f32"):
    """Stream `stream`'s pool before renormalisation and warm-up, and the
    xorshift state after drawing it."""
    if pool_dtype == "f64":
        P = np.empty(n, np.float64)
        xs = lib().orc_initial_pool_f64(seed, stream, n, P)
    else:
        P = np.empty(n, np.float32)
        xs = lib().orc_initial_pool_f32(seed, stream, n, P)
    return P, int(xs)


def chi2_consts(n: int):
    A, b = C.c_double(), C.c_double()
    lib().orc_chi2_consts(n, C.byref(A), C.byref(b))
    return A.value, b.value


def chi2_sample(n: int, x, mode: int = CHI2_CUBIC) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    S = np.zeros_like(x)
    lib().orc_chi2_sample(n, mode, x, S, x.size)
    return S


def cvt_bf16(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros(x.shape, np.uint16)
    lib().orc_cvt_bf16(x, y, x.size)
    return y


def cvt_f16(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.zeros(x.shape, np.uint16)
    lib().orc_cvt_f16(x, y, x.size)
    return y


def extreme_threshold(n: int) -> float:
    return float(lib().orc_extreme_threshold(n))


def extreme_counts(zmax_rows, c):
    """(pools with an extreme, adjacent pairs with two) from per-pool maxima of
    one stream, in pool order."""
    e = np.asarray(zmax_rows) >= c
    return int(e.sum()), int(np.count_nonzero(e[1:] & e[:-1]))


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---- the generator ----------------------------------------------------------

class Generator:
    """The oracle generator: same configuration surface as the GPU library."""

    def __init__(self, num_streams, pool_n=4096, R=2, pool_dtype="f32", chi2=CHI2_CUBIC,
                 K=16, hazard=HAZ_NONE, warmup=0, trace=False, x_current=False, transform=0,
                 mean=0.0, stddev=1.0, emit_stride=1, variate=0):
        self.num_streams = int(num_streams)
        per_stream = None
        if np.ndim(pool_n) > 0:
            per_stream = np.ascontiguousarray(pool_n, np.uint32)
            assert per_stream.size == self.num_streams
            default = int(per_stream[0])
        else:
            default = int(pool_n)
        self.pool_f64 = pool_dtype in ("f64", "float64", np.float64)
        cfg = _Config(self.num_streams, default, R, int(self.pool_f64), chi2, K, hazard, warmup,
                      int(bool(trace)), int(bool(x_current)), transform, emit_stride, mean,
                      stddev, variate)
        self._pool_n = per_stream
        self._h = lib().orc_create(C.byref(cfg),
                                   per_stream.ctypes.data if per_stream is not None else None)
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                lib().orc_destroy(h)
            except (TypeError, AttributeError):  # interpreter shutdown: module state is gone
                pass
            self._h = None

    def seed(self, seed: int):
        lib().orc_seed(self._h, seed)

    def fill(self, streams, counts, out_dtype=F32, threads=0) -> np.ndarray:
        streams = np.ascontiguousarray(streams, np.uint32)
        counts = np.ascontiguousarray(counts, np.uint64)
        total = int(counts.sum())
        out = np.zeros(total, _OUT_NP[out_dtype])
        rc = lib().orc_fill(self._h, streams.size, streams, counts,
                            out.ctypes.data if total else None, out_dtype, threads)
        if rc != 0:
            raise ValueError(f"oracle fill rejected the request (code {rc})")
        return out

    def stream(self, s: int):
        info = StreamInfo()
        n = int(self._pool_n[s]) if self._pool_n is not None else None
        if n is None:
            lib().orc_stream_get(self._h, s, C.byref(info), None)
            n = info.n
        pool = np.zeros(n, np.float64 if self.pool_f64 else np.float32)
        if lib().orc_stream_get(self._h, s, C.byref(info), pool.ctypes.data) != 0:
            raise IndexError(s)
        return info, pool

    def trace(self, s: int, max_records: int = 1 << 20) -> np.ndarray:
        """Per-pool records (Q, S, f, x, T, zmax), one row per pool produced."""
        buf = np.zeros(6 * max_records, np.float64)
        c = lib().orc_trace_get(self._h, s, buf, max_records)
        return buf[: 6 * c].reshape(c, 6)
