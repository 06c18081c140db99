"""ctypes binding of the C ABI in ``include/wn.h`` (argument marshalling only).

Every step of generation runs in the HIP kernels of ``libwn.so``.  PyTorch is
used only for device memory (output tensors) and streams.  If the library is
missing the binding raises; nothing falls back to a CPU path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# WN_LDS_POISON=1 selects the debug build (every LDS pool write preceded by a
# NaN fill of the buffer; build.build(poison=True)), for the poisoned parity run.
LIB_PATH = os.path.join(HERE, "libwn_poison.so" if os.environ.get("WN_LDS_POISON") == "1"
                        else "libwn.so")

WN_OK, WN_EINVAL, WN_ENOMEM, WN_EDEVICE, WN_ESTATE, WN_ENOTSUP = range(6)
WN_F64, WN_F32, WN_BF16, WN_F16 = range(4)
WN_CHI2_CUBIC, WN_CHI2_OFF, WN_CHI2_FISHER, WN_CHI2_WH = range(4)
STATUS_NAMES = {0: "WN_OK", 1: "WN_EINVAL", 2: "WN_ENOMEM", 3: "WN_EDEVICE", 4: "WN_ESTATE",
                5: "WN_ENOTSUP"}

# every symbol include/wn.h and include/wn_bench.h declare
EXPORTED = ("wn_create", "wn_seed", "wn_fill", "wn_sync", "wn_get_stream", "wn_destroy",
            "wn_state_size", "wn_save_state", "wn_load_state",
            "wn_last_error", "wn_version", "wn_set_tuning", "wn_get_tuning", "wn_autotune",
            "wn_fill_stats", "wn_fill_stats_noalloc", "wn_quality_check", "wn_tune_config",
            "wn_extreme_threshold", "wn_chi2_constants", "wn_bench_store",
            "wn_bench_traffic",
            "wn_bench_box_muller")


WN_X_PREVIOUS, WN_X_CURRENT = 0, 1
WN_NORMAL, WN_EXPONENTIAL = 0, 1
WN_TRANSFORM_A4, WN_TRANSFORM_ROTATION = 0, 1
WN_CONFIG_V1_SIZE = 40
WN_CONFIG_V2_SIZE = 64


class wn_config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("num_streams", C.c_uint32),
                ("pool_n", C.POINTER(C.c_uint32)), ("default_pool_n", C.c_uint32),
                ("passes_per_output", C.c_uint32), ("pool_dtype", C.c_int),
                ("chi2", C.c_int), ("renorm_period", C.c_uint32), ("device", C.c_int),
                ("chi2_source", C.c_int), ("transform", C.c_int), ("mean", C.c_double),
                ("stddev", C.c_double), ("emit_stride", C.c_uint32), ("variate", C.c_int)]


class wn_stream_info(C.Structure):
    _fields_ = [("xs", C.c_uint64), ("k", C.c_uint64), ("n", C.c_uint32),
                ("cursor", C.c_uint32), ("f", C.c_double), ("xnext", C.c_double),
                ("qlast", C.c_double)]


class wn_tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("lds_double_buffer", C.c_uint32),
                ("nontemporal_stores", C.c_uint32), ("waves_per_simd", C.c_uint32),
                ("wgs_per_cu", C.c_uint32), ("use_graph", C.c_uint32),
                ("long_priority_pct", C.c_uint32), ("streams_per_wg", C.c_uint32),
                ("defer_emission", C.c_uint32), ("group_items", C.c_uint32),
                ("threads_per_stream", C.c_uint32)]


HIST_BINS = 4096


class wn_stats(C.Structure):
    _fields_ = [("count", C.c_uint64), ("moment", C.c_double * 4), ("below", C.c_uint64),
                ("above", C.c_uint64), ("pools", C.c_uint64), ("t_sum", C.c_double),
                ("t_sumsq", C.c_double), ("t_pairs", C.c_uint64), ("t_lag", C.c_double),
                ("hist", C.c_uint64 * HIST_BINS), ("x_pools", C.c_uint64),
                ("x_pairs", C.c_uint64)]


WN_QUALITY_NAMES = ("mean", "var", "skew", "kurt", "hist", "pool_mean", "pool_var", "pool_lag",
                    "extreme_pairs")
WN_QUALITY_NZ = len(WN_QUALITY_NAMES)


class wn_quality(C.Structure):
    _fields_ = [("z", C.c_double * WN_QUALITY_NZ), ("passed", C.c_uint32),
                ("failed_mask", C.c_uint32)]


class wn_quality_tuning(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("pool_sizes", C.c_uint32 * 8),
                ("passes", C.c_uint32 * 8), ("calib_values", C.c_uint64), ("z_max", C.c_double)]


class wn_tune_candidate(C.Structure):
    _fields_ = [("pool_n", C.c_uint32), ("R", C.c_uint32), ("passed", C.c_uint32),
                ("failed_mask", C.c_uint32), ("worst_z", C.c_double), ("ms", C.c_float),
                ("reserved", C.c_uint32)]


class WnError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load libwn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first "
                              "(python paper_1005_2314_amd/build.py)")
        # PyTorch ships its own HIP runtime under the same soname as the system
        # one (libamdhip64.so.7); whichever is loaded first serves the whole
        # process.  Load torch's first, so that the library runs on the runtime
        # that owns the tensors and streams it is given (the other order leaves
        # torch without a device).
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.wn_create.argtypes = [C.POINTER(wn_config), C.POINTER(vp)]
        L.wn_create.restype = C.c_int
        L.wn_seed.argtypes = [vp, C.c_uint64, vp]
        L.wn_seed.restype = C.c_int
        L.wn_fill.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), vp,
                              C.c_int, vp]
        L.wn_fill.restype = C.c_int
        L.wn_sync.argtypes = [vp]
        L.wn_sync.restype = C.c_int
        L.wn_get_stream.argtypes = [vp, C.c_uint32, C.POINTER(wn_stream_info), vp]
        L.wn_get_stream.restype = C.c_int
        L.wn_destroy.argtypes = [vp]
        L.wn_destroy.restype = None
        L.wn_last_error.argtypes = []
        L.wn_last_error.restype = C.c_char_p
        L.wn_version.argtypes = []
        L.wn_version.restype = C.c_uint32
        L.wn_set_tuning.argtypes = [vp, C.POINTER(wn_tuning)]
        L.wn_set_tuning.restype = C.c_int
        L.wn_get_tuning.argtypes = [vp, C.POINTER(wn_tuning)]
        L.wn_get_tuning.restype = C.c_int
        L.wn_autotune.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                  vp, C.c_int, vp, C.POINTER(wn_tuning)]
        L.wn_autotune.restype = C.c_int
        L.wn_fill_stats.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                    vp, C.c_int, vp, vp]
        L.wn_fill_stats.restype = C.c_int
        L.wn_fill_stats_noalloc.argtypes = L.wn_fill_stats.argtypes
        L.wn_fill_stats_noalloc.restype = C.c_int
        L.wn_quality_check.argtypes = [C.POINTER(wn_stats), C.c_uint32, C.c_double,
                                       C.POINTER(wn_quality)]
        L.wn_quality_check.restype = C.c_int
        L.wn_tune_config.argtypes = [C.POINTER(wn_config), C.POINTER(wn_quality_tuning),
                                     C.c_uint32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                     vp, C.c_int, C.c_uint64, vp, C.POINTER(wn_config),
                                     C.POINTER(wn_tune_candidate), C.c_uint32,
                                     C.POINTER(C.c_uint32)]
        L.wn_tune_config.restype = C.c_int
        L.wn_extreme_threshold.argtypes = [C.c_uint32]
        L.wn_extreme_threshold.restype = C.c_double
        L.wn_chi2_constants.argtypes = [C.c_uint32, C.POINTER(C.c_double)]
        L.wn_chi2_constants.restype = C.c_int
        L.wn_state_size.argtypes = [vp]
        L.wn_state_size.restype = C.c_size_t
        L.wn_save_state.argtypes = [vp, vp, C.c_size_t]
        L.wn_save_state.restype = C.c_int
        L.wn_load_state.argtypes = [vp, vp, C.c_size_t]
        L.wn_load_state.restype = C.c_int
        L.wn_bench_store.argtypes = [vp, C.c_uint64, C.c_uint32, vp]
        L.wn_bench_store.restype = C.c_int
        L.wn_bench_traffic.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint64, vp]
        L.wn_bench_traffic.restype = C.c_int
        L.wn_bench_box_muller.argtypes = [vp, C.c_uint64, C.c_int, C.c_uint64, C.c_int, vp]
        L.wn_bench_box_muller.restype = C.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return load().wn_last_error().decode()


def check(status: int):
    if status != WN_OK:
        raise WnError(status, last_error())


# ---- the C functions under their own names ------------------------------------

def wn_create(cfg: wn_config):
    h = C.c_void_p()
    check(load().wn_create(C.byref(cfg), C.byref(h)))
    return h


def wn_seed(g, seed: int, stream=None):
    check(load().wn_seed(g, seed, stream))


def wn_fill(g, streams, counts, out_ptr, out_dtype: int, stream=None):
    streams = np.ascontiguousarray(streams, np.uint32)
    counts = np.ascontiguousarray(counts, np.uint64)
    check(load().wn_fill(g, streams.size, streams.ctypes.data_as(C.POINTER(C.c_uint32)),
                         counts.ctypes.data_as(C.POINTER(C.c_uint64)), out_ptr, out_dtype,
                         stream))


def wn_sync(g):
    check(load().wn_sync(g))


def wn_destroy(g):
    load().wn_destroy(g)


def wn_bench_store(dst_ptr, nbytes, width, stream=None):
    st = load().wn_bench_store(dst_ptr, nbytes, width, stream)
    if st != WN_OK:
        raise WnError(st, "wn_bench_store rejected its arguments")


def wn_bench_traffic(state_ptr, out_ptr, num_streams, pool_n, per_stream, stream=None):
    st = load().wn_bench_traffic(state_ptr, out_ptr, num_streams, pool_n, per_stream, stream)
    if st != WN_OK:
        raise WnError(st, "wn_bench_traffic rejected its arguments")


def wn_bench_box_muller(out_ptr, count, out_dtype, seed, fast=False, stream=None):
    st = load().wn_bench_box_muller(out_ptr, count, out_dtype, seed, int(bool(fast)), stream)
    if st != WN_OK:
        raise WnError(st, "wn_bench_box_muller rejected its arguments")


def make_config(num_streams, pool_n=4096, R=2, pool_dtype=WN_F32, chi2=WN_CHI2_CUBIC, K=16,
                device=0, chi2_source=WN_X_PREVIOUS, transform=WN_TRANSFORM_A4, mean=0.0,
                stddev=1.0, emit_stride=1, variate=WN_NORMAL):
    cfg = wn_config()
    cfg.struct_size = C.sizeof(wn_config)
    cfg.num_streams = int(num_streams)
    keep = None
    if np.ndim(pool_n) > 0:
        keep = np.ascontiguousarray(pool_n, np.uint32)
        cfg.pool_n = keep.ctypes.data_as(C.POINTER(C.c_uint32))
        cfg.default_pool_n = int(keep[0])
    else:
        cfg.pool_n = None
        cfg.default_pool_n = int(pool_n)
    cfg.passes_per_output = int(R)
    cfg.pool_dtype = int(pool_dtype)
    cfg.chi2 = int(chi2)
    cfg.renorm_period = int(K)
    cfg.device = int(device)
    cfg.chi2_source = int(chi2_source)
    cfg.transform = int(transform)
    cfg.mean = float(mean)
    cfg.stddev = float(stddev)
    cfg.emit_stride = int(emit_stride)
    cfg.variate = int(variate)
    return cfg, keep


_TORCH_DTYPES = None


def extreme_threshold(n):
    """c_n of the extreme-pool statistics (wn_extreme_threshold); NaN for a bad n."""
    return float(load().wn_extreme_threshold(int(n)))


def chi2_constants(n):
    """(nu, A, b, fisher_root, wh_scale, wh_shift) for pools of n values
    (wn_chi2_constants); WnError for a bad n."""
    out = (C.c_double * 6)()
    check(load().wn_chi2_constants(int(n), out))
    return tuple(out)


def quality_check(stats, pool_n, z_max=5.0):
    """wn_quality_check on a host wn_stats: (passed, {name: z}, failed_mask)."""
    q = wn_quality()
    check(load().wn_quality_check(C.byref(stats), int(pool_n), float(z_max), C.byref(q)))
    return bool(q.passed), dict(zip(WN_QUALITY_NAMES, list(q.z))), int(q.failed_mask)


def tune_config(cfg, out, streams, counts, seed=1, pool_sizes=(), passes=(), calib_values=0,
                z_max=0.0, stream=None):
    """wn_tune_config: the fastest (pool size, R) that passes the statistics
    battery, for the request (streams, counts) into the CUDA tensor `out`.
    Returns (chosen wn_config, list of wn_tune_candidate)."""
    import torch
    dt = {torch.float64: WN_F64, torch.float32: WN_F32, torch.bfloat16: WN_BF16,
          torch.float16: WN_F16}[out.dtype]
    o = wn_quality_tuning()
    o.struct_size = C.sizeof(wn_quality_tuning)
    for i, v in enumerate(pool_sizes):
        o.pool_sizes[i] = int(v)
    for i, v in enumerate(passes):
        o.passes[i] = int(v)
    o.calib_values = int(calib_values)
    o.z_max = float(z_max)
    streams = np.ascontiguousarray(streams, np.uint32)
    counts = np.ascontiguousarray(counts, np.uint64)
    chosen = wn_config()
    rep = (wn_tune_candidate * 64)()
    nrep = C.c_uint32()
    st = stream if stream is not None else torch.cuda.current_stream()
    status = load().wn_tune_config(C.byref(cfg), C.byref(o), streams.size,
                                   streams.ctypes.data_as(C.POINTER(C.c_uint32)),
                                   counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                                   C.c_void_p(out.data_ptr()), dt, int(seed),
                                   C.c_void_p(st.cuda_stream), C.byref(chosen), rep, 64,
                                   C.byref(nrep))
    report = [rep[i] for i in range(min(nrep.value, 64))]
    check(status)
    return chosen, report


def torch_dtype(out_dtype):
    import torch
    return {WN_F64: torch.float64, WN_F32: torch.float32, WN_BF16: torch.bfloat16,
            WN_F16: torch.float16}[out_dtype]


class Generator:
    """A set of independent streams on one GPU (owns a ``wn_gen``)."""

    def __init__(self, num_streams, pool_n=4096, R=2, pool_dtype=WN_F32, chi2=WN_CHI2_CUBIC,
                 K=16, device=0, chi2_source=WN_X_PREVIOUS, transform=WN_TRANSFORM_A4,
                 mean=0.0, stddev=1.0, emit_stride=1, variate=WN_NORMAL):
        self.cfg, keep = make_config(num_streams, pool_n, R, pool_dtype, chi2, K, device,
                                     chi2_source, transform, mean, stddev, emit_stride, variate)
        self.num_streams = int(num_streams)
        self.pool_f64 = pool_dtype == WN_F64
        self.device = device
        self._h = wn_create(self.cfg)
        del keep  # the library copied the pool sizes

    def close(self):
        if getattr(self, "_h", None):
            wn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream_handle(stream):
        if stream is None:
            import torch
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if isinstance(stream, int):
            return C.c_void_p(stream)
        return C.c_void_p(stream.cuda_stream)

    def seed(self, seed: int, stream=None):
        wn_seed(self._h, seed, self._stream_handle(stream))

    def fill_into(self, out, streams, counts, stream=None):
        """Fill a caller-owned CUDA tensor (dtype selects the output type)."""
        import torch
        dt = {torch.float64: WN_F64, torch.float32: WN_F32, torch.bfloat16: WN_BF16,
              torch.float16: WN_F16}[out.dtype]
        total = int(np.sum(np.asarray(counts, np.uint64)))
        if out.numel() < total or not out.is_contiguous() or not out.is_cuda:
            raise ValueError("out must be a contiguous CUDA tensor with sum(counts) elements")
        wn_fill(self._h, streams, counts, C.c_void_p(out.data_ptr()), dt,
                self._stream_handle(stream))
        return out

    def fill(self, streams, counts, out_dtype=WN_F32, stream=None):
        import torch
        total = int(np.sum(np.asarray(counts, np.uint64)))
        out = torch.empty(total, dtype=torch_dtype(out_dtype), device=f"cuda:{self.device}")
        return self.fill_into(out, streams, counts, stream)

    def sync(self):
        wn_sync(self._h)

    def fill_stats_into(self, out, streams, counts, stats, stream=None, noalloc=False):
        """wn_fill_stats (wn_fill_stats_noalloc with noalloc=True) into a
        caller-owned CUDA output tensor; `stats` is a CUDA uint8 tensor of
        sizeof(wn_stats) bytes (see read_stats)."""
        import torch
        dt = {torch.float64: WN_F64, torch.float32: WN_F32, torch.bfloat16: WN_BF16,
              torch.float16: WN_F16}[out.dtype]
        streams = np.ascontiguousarray(streams, np.uint32)
        counts = np.ascontiguousarray(counts, np.uint64)
        if stats.numel() * stats.element_size() < C.sizeof(wn_stats) or not stats.is_cuda:
            raise ValueError("stats must be a CUDA buffer of sizeof(wn_stats) bytes")
        fn = load().wn_fill_stats_noalloc if noalloc else load().wn_fill_stats
        check(fn(self._h, streams.size,
                                   streams.ctypes.data_as(C.POINTER(C.c_uint32)),
                                   counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                                   C.c_void_p(out.data_ptr()), dt,
                                   C.c_void_p(stats.data_ptr()), self._stream_handle(stream)))
        return out

    @staticmethod
    def stats_buffer(device=0):
        import torch
        return torch.zeros(C.sizeof(wn_stats), dtype=torch.uint8, device=f"cuda:{device}")

    @staticmethod
    def read_stats(buf):
        """Copy a device stats buffer to a host wn_stats."""
        host = buf.cpu().numpy()
        st = wn_stats()
        C.memmove(C.addressof(st), host.ctypes.data, C.sizeof(wn_stats))
        return st

    def set_tuning(self, lds_double_buffer=None, nontemporal_stores=None, waves_per_simd=None,
                   wgs_per_cu=None, use_graph=None, long_priority_pct=None, streams_per_wg=None,
                   defer_emission=None, group_items=None, threads_per_stream=None):
        t = self.tuning()
        if threads_per_stream is not None:
            t.threads_per_stream = int(threads_per_stream)
        if group_items is not None:
            t.group_items = int(group_items)
        if defer_emission is not None:
            t.defer_emission = int(defer_emission)
        if streams_per_wg is not None:
            t.streams_per_wg = int(streams_per_wg)
        if long_priority_pct is not None:
            t.long_priority_pct = int(long_priority_pct)
        if wgs_per_cu is not None:
            t.wgs_per_cu = int(wgs_per_cu)
        if use_graph is not None:
            t.use_graph = int(use_graph)
        if lds_double_buffer is not None:
            t.lds_double_buffer = int(lds_double_buffer)
        if nontemporal_stores is not None:
            t.nontemporal_stores = int(nontemporal_stores)
        if waves_per_simd is not None:
            t.waves_per_simd = int(waves_per_simd)
        check(load().wn_set_tuning(self._h, C.byref(t)))

    def tuning(self):
        t = wn_tuning()
        check(load().wn_get_tuning(self._h, C.byref(t)))
        return t

    def autotune(self, out, streams, counts, stream=None):
        """Pick the fastest launch choices for this request shape (state unchanged)."""
        import torch
        dt = {torch.float64: WN_F64, torch.float32: WN_F32, torch.bfloat16: WN_BF16,
              torch.float16: WN_F16}[out.dtype]
        streams = np.ascontiguousarray(streams, np.uint32)
        counts = np.ascontiguousarray(counts, np.uint64)
        t = wn_tuning()
        check(load().wn_autotune(self._h, streams.size,
                                 streams.ctypes.data_as(C.POINTER(C.c_uint32)),
                                 counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 C.c_void_p(out.data_ptr()), dt, self._stream_handle(stream),
                                 C.byref(t)))
        return t

    def save_state(self) -> bytes:
        """Checkpoint of every stream (host bytes)."""
        n = load().wn_state_size(self._h)
        buf = C.create_string_buffer(n)
        check(load().wn_save_state(self._h, buf, n))
        return buf.raw

    def load_state(self, blob: bytes):
        check(load().wn_load_state(self._h, C.c_char_p(blob), len(blob)))

    def stream_state(self, s: int):
        info = wn_stream_info()
        pool = None
        check(load().wn_get_stream(self._h, s, C.byref(info), None))
        pool = np.zeros(info.n, np.float64 if self.pool_f64 else np.float32)
        check(load().wn_get_stream(self._h, s, C.byref(info), C.c_void_p(pool.ctypes.data)))
        return info, pool
