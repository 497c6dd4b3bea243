"""MI355X (gfx950) cascaded-biquad filtering: Python binding of libsosfilt.

Thin ctypes layer over the C ABI in include/sosfilt.h. It only marshals
arguments (device pointers of torch tensors, the current HIP stream); every
step of the filter runs in the HIP kernels of libsosfilt.so. There is no CPU
fallback: if the library is missing, importing the binding's functions fails.

    from paper_2607_23763_amd import sosfilt
    y, zf = sosfilt(x, sos, zi)        # x: (n,) float32 on the GPU, sos: (K, 6)
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsosfilt.so")

SOS_OK = 0
SOS_EINVAL = -1
SOS_EA0 = -2
SOS_EUNSTABLE = -3
SOS_ENOMEM = -4
SOS_EHIP = -5
SOS_ETIMEOUT = -6
SOS_ECLOSED = -7
SOS_EBUSY = -8
SOS_ELIMIT = -9
SOS_MAX_SECTIONS = 64
SOS_ALG_DEFAULT = 0
SOS_ALG_DCCR = 1
SOS_ALG_PH = 2
SOS_ALG_AUTO = 3
SOS_ALG_TOEPLITZ = 4
_ALGS = {None: SOS_ALG_DEFAULT, "default": SOS_ALG_DEFAULT, "dccr": SOS_ALG_DCCR,
         "ph": SOS_ALG_PH, "auto": SOS_ALG_AUTO, "toeplitz": SOS_ALG_TOEPLITZ,
         SOS_ALG_DEFAULT: SOS_ALG_DEFAULT, SOS_ALG_DCCR: SOS_ALG_DCCR, SOS_ALG_PH: SOS_ALG_PH,
         SOS_ALG_AUTO: SOS_ALG_AUTO, SOS_ALG_TOEPLITZ: SOS_ALG_TOEPLITZ}

_lib = None
_lib_lock = threading.Lock()


class SosError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__("%s: %s (%d)" % (what or "sosfilt", strerror(code), code))


def lib():
    """Load libsosfilt.so (built by __graft_entry__.build()); raises if missing."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libsosfilt.so is not built (%s); run __graft_entry__.build()"
                                  % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
            L.sos_create.argtypes = [ctypes.POINTER(vp), i32]
            L.sos_destroy.argtypes = [vp]
            L.sos_strerror.argtypes = [i32]
            L.sos_strerror.restype = ctypes.c_char_p
            L.sos_last_error.argtypes = [vp]
            L.sos_set_tile.argtypes = [vp, i32, i32]
            L.sos_get_tile.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
            L.sos_filter.argtypes = [vp, vp, i32, vp, vp, i64, vp, vp, vp]
            L.sos_debug_carries.argtypes = [vp, vp, i64, ctypes.POINTER(i64),
                                            ctypes.POINTER(i32)]
            L.sos_prepare.argtypes = [vp, vp, i32, vp]
            L.sos_filter_prepared.argtypes = [vp, vp, vp, i64, vp, vp, vp]
            L.sos_bench_copy.argtypes = [vp, vp, i64, vp]
            L.sos_filter_noalloc.argtypes = [vp, i32, vp, vp, i64, vp, vp, vp, vp]
            L.sos_filter_noalloc.restype = i32
            L.sos_filter_batched.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp, vp, vp, vp,
                                             vp, vp]
            L.sos_set_precision.argtypes = [vp, i32]
            L.sos_set_timeout.argtypes = [vp, ctypes.c_double]
            L.sos_wall_clock_khz.argtypes = [vp]
            L.sos_get_precision.argtypes = [vp]
            L.sos_set_algorithm.argtypes = [vp, i32]
            L.sos_get_algorithm.argtypes = [vp]
            L.sos_filter_train.argtypes = [vp, vp, i32, vp, vp, i64, vp, vp, vp, vp]
            L.sos_filter_vjp.argtypes = [vp, vp, i32, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
            u64p = ctypes.POINTER(ctypes.c_uint64)
            dp = ctypes.POINTER(ctypes.c_double)
            L.sos_server_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t, i32]
            L.sos_server_destroy.argtypes = [vp]
            L.sos_server_limits.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                            ctypes.POINTER(i32), ctypes.POINTER(i32)]
            L.sos_stream_open.argtypes = [vp, vp, i32, vp, ctypes.POINTER(i64)]
            L.sos_stream_push.argtypes = [vp, i64, vp, i64, vp, u64p]
            L.sos_stream_push_many.argtypes = [vp, i32, vp, vp, vp, vp, vp]
            L.sos_stream_wait.argtypes = [vp, ctypes.c_uint64, dp]
            L.sos_stream_state.argtypes = [vp, i64, vp]
            L.sos_stream_close.argtypes = [vp, i64]
            L.sos_server_replay.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, dp]
            L.sos_graph_create_batched.argtypes = [ctypes.POINTER(vp), vp, i32, i32, i64, i64, vp,
                                                   vp, vp, vp, vp, vp, vp, vp]
            L.sos_graph_launch.argtypes = [vp, vp]
            L.sos_graph_last_error.argtypes = [vp]
            L.sos_graph_destroy.argtypes = [vp]
            L.sos_tune_batched.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                           vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(ctypes.c_float)]
            L.sos_tune_lookup.argtypes = [vp, i32, i32, i64, ctypes.POINTER(i32),
                                          ctypes.POINTER(i32)]
            L.sos_model_floors.argtypes = [ctypes.POINTER(ModelDevice), ctypes.c_double,
                                           ctypes.POINTER(ModelFloors)]
            L.sos_model_config.argtypes = [ctypes.POINTER(ModelDevice), i32, i32, i32, i32,
                                           ctypes.c_double, ctypes.POINTER(ModelConfig)]
            L.sos_model_device_gfx950.argtypes = [ctypes.POINTER(ModelDevice)]
            L.sos_fwd_kernel_attrs.argtypes = [i32, i32, i32, i32, ctypes.POINTER(i32),
                                               ctypes.POINTER(i32)]
            L.sos_fwd_capacity.argtypes = [i32, i32, i32, i32]
            L.sos_fwd_shape_supported.argtypes = [i32, i32]
            for name in ("sos_model_floors", "sos_model_config", "sos_model_device_gfx950",
                         "sos_fwd_kernel_attrs", "sos_fwd_capacity", "sos_fwd_shape_supported"):
                getattr(L, name).restype = i32
            L.sos_filter_train_batched.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp, vp,
                                                   vp, vp, vp, vp, vp]
            L.sos_filter_vjp_batched.argtypes = [vp, i32, i32, i64, i64, vp, vp, vp, vp, vp, vp,
                                                 vp, vp, vp, vp, vp, vp, vp]
            L.sos_filter_vjp_batched_sum.argtypes = L.sos_filter_vjp_batched.argtypes
            L.sos_filter_train_batched.restype = i32
            L.sos_filter_vjp_batched.restype = i32
            L.sos_filter_vjp_batched_sum.restype = i32
            for name in ("sos_graph_create_batched", "sos_graph_launch", "sos_graph_last_error",
                         "sos_graph_destroy", "sos_tune_batched", "sos_tune_lookup"):
                getattr(L, name).restype = i32
            for name in ("sos_server_create", "sos_server_destroy", "sos_server_limits",
                         "sos_stream_open", "sos_stream_push", "sos_stream_push_many",
                         "sos_stream_wait", "sos_stream_state", "sos_stream_close",
                         "sos_server_replay"):
                getattr(L, name).restype = i32
            for name in ("sos_create", "sos_destroy", "sos_last_error", "sos_set_tile",
                         "sos_get_tile", "sos_filter", "sos_debug_carries", "sos_prepare",
                         "sos_filter_prepared", "sos_bench_copy", "sos_filter_batched",
                         "sos_filter_train", "sos_filter_vjp", "sos_set_precision",
                         "sos_get_precision", "sos_set_timeout", "sos_wall_clock_khz",
                         "sos_set_algorithm", "sos_get_algorithm"):
                getattr(L, name).restype = i32
            _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().sos_strerror(int(code)).decode()
    except ImportError:
        return "status %d" % code


def _check(rc: int, what: str):
    if rc != SOS_OK:
        raise SosError(rc, what)


def _stream_ptr(device=None):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Handle:
    """Owns a libsosfilt handle (workspace: tables, lookback descriptors)."""

    def __init__(self, device: int = 0, tile=None, precision: int = 0, algorithm=None):
        self._h = ctypes.c_void_p()
        self.device = int(device)
        _check(lib().sos_create(ctypes.byref(self._h), self.device), "sos_create")
        if tile:
            self.set_tile(*tile)
        if precision:
            self.set_precision(precision)
        if algorithm:
            self.set_algorithm(algorithm)

    def set_algorithm(self, alg):
        """Section solver: "auto" (per signal: cyclic reduction, or PH on the
        accurate table layout when a section's poles lie close to the unit
        circle), "dccr" (cyclic reduction throughout), "ph" (particular +
        homogeneous), "toeplitz" (plain FP32 forward calls of up to 8
        sections through the whole-cascade block-Toeplitz kernel on the
        matrix cores, everything else as "ph"), or None / "default" (the
        environment's SOS_ALG, else "auto"; "auto" also takes the
        block-Toeplitz kernel for plain calls of orders 14-16 on at least
        2^25 samples, order 12 on at least 2^26)."""
        code = _ALGS.get(alg if not isinstance(alg, str) else alg.lower())
        if code is None:
            raise ValueError("unknown algorithm %r" % (alg,))
        _check(lib().sos_set_algorithm(self._h, code), "sos_set_algorithm")

    def algorithm(self) -> str:
        code = int(lib().sos_get_algorithm(self._h))
        return {SOS_ALG_DCCR: "dccr", SOS_ALG_PH: "ph", SOS_ALG_AUTO: "auto",
                SOS_ALG_TOEPLITZ: "toeplitz"}[code]

    def set_precision(self, bits: int):
        """Compute type of the kernels: 32 or 64 (0 = default)."""
        _check(lib().sos_set_precision(self._h, int(bits)), "sos_set_precision")

    def precision(self) -> int:
        return int(lib().sos_get_precision(self._h))

    def set_timeout(self, ms: float):
        """Bound on each lookback wait in milliseconds (0 = default)."""
        _check(lib().sos_set_timeout(self._h, float(ms)), "sos_set_timeout")

    def wall_clock_khz(self) -> int:
        return int(lib().sos_wall_clock_khz(self._h))

    def close(self):
        if self._h:
            lib().sos_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def set_tile(self, L: int, N: int):
        """Group shape: L lanes (64 per wavefront) x N samples per lane."""
        _check(lib().sos_set_tile(self._h, int(L), int(N)), "sos_set_tile")

    def tile(self):
        L = ctypes.c_int32()
        N = ctypes.c_int32()
        _check(lib().sos_get_tile(self._h, ctypes.byref(L), ctypes.byref(N)), "sos_get_tile")
        return L.value, N.value

    def last_error(self) -> int:
        return int(lib().sos_last_error(self._h))

    def carries(self):
        """Resolved per-(group, section) end states of the last call, (groups, K, 2)."""
        import numpy as np

        g = ctypes.c_int64()
        k = ctypes.c_int32()
        _check(lib().sos_debug_carries(self._h, None, 0, ctypes.byref(g), ctypes.byref(k)),
               "sos_debug_carries")
        out = np.empty((g.value, k.value, 2), dtype=np.float32)
        _check(lib().sos_debug_carries(self._h, out.ctypes.data_as(ctypes.c_void_p), out.size,
                                       ctypes.byref(g), ctypes.byref(k)), "sos_debug_carries")
        return out


_handles = {}
_handles_lock = threading.Lock()


def default_handle(device: int = 0) -> Handle:
    with _handles_lock:
        h = _handles.get(device)
        if h is None:
            h = Handle(device)
            _handles[device] = h
        return h


def _as_dev_f32(t, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU torch tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    return t.contiguous()


def sosfilt_noalloc(x, sos, y, zi=None, zf=None, err=None):
    """The plain filter through sos_filter_noalloc (no handle, no allocation in
    the library): y (and zf, err) are caller-provided float32 / int32 GPU
    tensors; err receives the call's device-side error bits."""
    x = _as_dev_f32(x, "x").reshape(-1)
    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    K = sos.shape[0]
    if zi is not None:
        zi = _as_dev_f32(zi, "zi").reshape(K, 2)
    if zf is not None:
        zf = _as_dev_f32(zf, "zf").reshape(K, 2)
    y = _as_dev_f32(y, "y").reshape(-1)
    if y.numel() != x.numel():
        raise ValueError("y must have x's length")
    _check(lib().sos_filter_noalloc(_p(sos) if K else None, K, _p(x), _p(y), x.numel(), _p(zi),
                                    _p(zf), _p(err), _stream_ptr(x.device)),
           "sos_filter_noalloc")
    return y, zf


def sosfilt_(x, sos, y=None, zi=None, zf=None, handle: Handle | None = None):
    """Low-level call: filter device tensor x into y (may be x) with the K x 6
    device tensor sos; optional zi (K, 2) and zf (K, 2) outputs. Enqueued on
    the current stream."""
    import torch

    x = _as_dev_f32(x, "x")
    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    K = sos.shape[0]
    if y is None:
        y = torch.empty_like(x)
    h = handle or default_handle(x.device.index or 0)
    rc = lib().sos_filter(
        h.ptr, ctypes.c_void_p(sos.data_ptr()), K, ctypes.c_void_p(x.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), x.numel(),
        ctypes.c_void_p(zi.data_ptr()) if zi is not None else None,
        ctypes.c_void_p(zf.data_ptr()) if zf is not None else None,
        _stream_ptr(x.device))
    _check(rc, "sos_filter")
    return y


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def prepare(sos, handle: Handle | None = None):
    """Enqueue the coefficient tables for sos (K x 6 device tensor) on the
    handle; later filter_prepared() calls reuse them."""
    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    h = handle or default_handle(sos.device.index or 0)
    _check(lib().sos_prepare(h.ptr, _p(sos), sos.shape[0], _stream_ptr(sos.device)), "sos_prepare")
    return h


def filter_prepared(x, y, zi=None, zf=None, handle: Handle | None = None):
    """Filter device tensor x into y (may be x) with the prepared tables."""
    h = handle or default_handle(x.device.index or 0)
    _check(lib().sos_filter_prepared(h.ptr, _p(x), _p(y), x.numel(), _p(zi), _p(zf),
                                     _stream_ptr(x.device)), "sos_filter_prepared")
    return y


def bench_copy(x, y):
    """Plain streaming copy y = x (memory-floor reference kernel)."""
    _check(lib().sos_bench_copy(_p(x), _p(y), x.numel(), _stream_ptr(x.device)), "sos_bench_copy")
    return y


def sosfilt(x, sos, zi=None, handle: Handle | None = None):
    """y, zf = sosfilt(x, sos, zi): cascade of K biquads over a 1-D float32
    GPU tensor; sos is (K, 6) [b0 b1 b2 a0 a1 a2]; zi/zf are (K, 2) TDF-II states."""
    import torch

    x = _as_dev_f32(x, "x").reshape(-1)
    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    K = sos.shape[0]
    if zi is not None:
        zi = _as_dev_f32(zi, "zi").reshape(K, 2)
    zf = torch.empty((K, 2), dtype=torch.float32, device=x.device)
    y = torch.empty_like(x)
    sosfilt_(x, sos, y=y, zi=zi, zf=zf, handle=handle)
    return y, zf


def _batch_args(x, sections, K, sig_off, zi, y, zf, sec_off, kmax):
    import torch

    x = _as_dev_f32(x, "x").reshape(-1)
    sections = _as_dev_f32(sections, "sections").reshape(-1, 6)
    if K.dtype != torch.int32 or not K.is_cuda:
        raise TypeError("K must be an int32 GPU tensor")
    if sig_off.dtype != torch.int64 or not sig_off.is_cuda:
        raise TypeError("sig_off must be an int64 GPU tensor")
    B = K.numel()
    if sec_off is None:
        sec_off = torch.zeros(B + 1, dtype=torch.int32, device=x.device)
        sec_off[1:] = torch.cumsum(K, 0, dtype=torch.int32)
    if kmax is None:
        kmax = int(K.max().item()) if B else 0
    nsec = sections.shape[0]
    if zi is not None:
        zi = _as_dev_f32(zi, "zi").reshape(-1, 2)
    if y is None:
        y = torch.empty_like(x)
    if zf is None:
        zf = torch.empty((nsec, 2), dtype=torch.float32, device=x.device)
    return dict(x=x, sections=sections, K=K.contiguous(), sig_off=sig_off.contiguous(),
                sec_off=sec_off.contiguous(), zi=zi, y=y, zf=zf, B=B, kmax=int(kmax), nsec=nsec)


def sosfilt_batched(x, sections, K, sig_off, zi=None, y=None, zf=None, sec_off=None, kmax=None,
                    handle: Handle | None = None):
    """Uneven batch: signal i is x[sig_off[i]:sig_off[i+1]] filtered by the K[i]
    rows of `sections` starting at row sec_off[i] (default: prefix of K).
    x, sections, zi: float32 GPU tensors; K (int32), sig_off (int64, B+1),
    sec_off (int32, B+1): GPU tensors. Returns (y, zf) with zf shaped like zi
    (sec_off[B] x 2). One persistent launch on the current stream."""
    a = _batch_args(x, sections, K, sig_off, zi, y, zf, sec_off, kmax)
    h = handle or default_handle(a["x"].device.index or 0)
    _check(lib().sos_filter_batched(h.ptr, a["B"], a["kmax"], a["nsec"], a["x"].numel(),
                                    _p(a["K"]), _p(a["sec_off"]), _p(a["sections"]),
                                    _p(a["sig_off"]), _p(a["x"]), _p(a["y"]), _p(a["zi"]),
                                    _p(a["zf"]), _stream_ptr(a["x"].device)),
           "sos_filter_batched")
    return a["y"], a["zf"]


def sosfilt_train_batched(x, sections, K, sig_off, zi=None, sec_off=None, kmax=None,
                          handle: Handle | None = None):
    """Batched forward keeping the section outputs for the adjoint
    (sos_filter_train_batched). Returns (y, zf, saved)."""
    import torch

    a = _batch_args(x, sections, K, sig_off, zi, None, None, sec_off, kmax)
    saved = torch.empty((max(a["kmax"] - 1, 1), a["x"].numel()), dtype=torch.float32,
                        device=a["x"].device)
    h = handle or default_handle(a["x"].device.index or 0)
    _check(lib().sos_filter_train_batched(h.ptr, a["B"], a["kmax"], a["nsec"], a["x"].numel(),
                                          _p(a["K"]), _p(a["sec_off"]), _p(a["sections"]),
                                          _p(a["sig_off"]), _p(a["x"]), _p(a["y"]), _p(a["zi"]),
                                          _p(a["zf"]), _p(saved), _stream_ptr(a["x"].device)),
           "sos_filter_train_batched")
    return a["y"], a["zf"], saved


def sosfilt_vjp_batched(sections, K, sig_off, x, y, saved, gy, gzf=None, sec_off=None,
                        kmax=None, handle: Handle | None = None, shared: bool = False):
    """Vector-Jacobian product of a batched forward (sos_filter_vjp_batched).
    Returns (gx, gzi, gsections), gzi and gsections shaped like zi and
    sections (rows of the batch's signals). With shared=True (every signal's
    rows hold the same cascade) gsections is kmax x 6, the gradients summed
    over the signals in FP64 by the library (sos_filter_vjp_batched_sum)."""
    import torch

    a = _batch_args(x, sections, K, sig_off, None, None, None, sec_off, kmax)
    y = _as_dev_f32(y, "y").reshape(-1)
    gy = _as_dev_f32(gy, "gy").reshape(-1)
    if gzf is not None:
        gzf = _as_dev_f32(gzf, "gzf").reshape(-1, 2)
    gx = torch.empty_like(a["x"])
    gzi = torch.zeros((a["nsec"], 2), dtype=torch.float32, device=a["x"].device)
    gs = torch.zeros((max(a["kmax"], 1) if shared else a["nsec"], 6), dtype=torch.float32,
                     device=a["x"].device)
    h = handle or default_handle(a["x"].device.index or 0)
    fn = lib().sos_filter_vjp_batched_sum if shared else lib().sos_filter_vjp_batched
    _check(fn(h.ptr, a["B"], a["kmax"], a["nsec"], a["x"].numel(), _p(a["K"]), _p(a["sec_off"]),
              _p(a["sections"]), _p(a["sig_off"]), _p(a["x"]), _p(y), _p(saved), _p(gy), _p(gzf),
              _p(gx), _p(gzi), _p(gs), _stream_ptr(a["x"].device)),
           "sos_filter_vjp_batched_sum" if shared else "sos_filter_vjp_batched")
    return gx, gzi, gs


class ModelDevice(ctypes.Structure):
    """sos_model_device: a device's per-SM (per-CU) budgets for the cost model."""
    _fields_ = [("sms", ctypes.c_int), ("smem_per_sm", ctypes.c_double),
                ("smem_per_tb", ctypes.c_double), ("regs_per_sm", ctypes.c_int),
                ("regs_per_simd_lane", ctypes.c_int), ("simds", ctypes.c_int),
                ("reg_granule", ctypes.c_int), ("max_threads_per_sm", ctypes.c_int),
                ("max_warps_per_sm", ctypes.c_int), ("max_tbs_per_sm", ctypes.c_int),
                ("warp", ctypes.c_int), ("issue_rate", ctypes.c_double),
                ("fma_latency", ctypes.c_double), ("bandwidth_gbs", ctypes.c_double),
                ("clock_ghz", ctypes.c_double), ("fp32_tflops", ctypes.c_double)]


class ModelFloors(ctypes.Structure):
    _fields_ = [("roof_gss", ctypes.c_double), ("w_min", ctypes.c_int)]


class ModelConfig(ctypes.Structure):
    _fields_ = [("s_buf", ctypes.c_double), ("tbs_per_sm", ctypes.c_int),
                ("warps_per_sm", ctypes.c_int), ("limit", ctypes.c_int),
                ("feasible", ctypes.c_int), ("starved", ctypes.c_int)]


SOS_MODEL_LIMIT_SMEM, SOS_MODEL_LIMIT_TBS, SOS_MODEL_LIMIT_THREADS, SOS_MODEL_LIMIT_REGS = 1, 2, 3, 4


def fwd_kernel_attrs(bits: int, alg: int, L: int, N: int):
    """(vector registers per lane, static LDS bytes) of a compiled forward
    kernel (sos_fwd_kernel_attrs)."""
    r, s = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sos_fwd_kernel_attrs(bits, alg, L, N, ctypes.byref(r), ctypes.byref(s)),
           "sos_fwd_kernel_attrs")
    return r.value, s.value


def model_device_gfx950() -> ModelDevice:
    d = ModelDevice()
    _check(lib().sos_model_device_gfx950(ctypes.byref(d)), "sos_model_device_gfx950")
    return d


def model_floors(dev: ModelDevice, ilp: float = 3.0) -> ModelFloors:
    """Eq. (28)'s roof (GS/s) and Eq. (29)'s hiding floor (sos_model_floors)."""
    f = ModelFloors()
    _check(lib().sos_model_floors(ctypes.byref(dev), float(ilp), ctypes.byref(f)),
           "sos_model_floors")
    return f


def model_config(dev: ModelDevice, L: int, N: int, pad: int = 1, regs: int = 0,
                 ilp: float = 3.0) -> ModelConfig:
    """Staging buffer, residency and hiding of an (L, N) tile (sos_model_config)."""
    c = ModelConfig()
    _check(lib().sos_model_config(ctypes.byref(dev), int(L), int(N), int(pad), int(regs),
                                  float(ilp), ctypes.byref(c)), "sos_model_config")
    return c


def tune_batched(x, sections, K, sig_off, zi=None, y=None, zf=None, sec_off=None, kmax=None,
                 handle: Handle | None = None, reps: int = 3):
    """Autotune (L, N) for this batch (sos_tune_batched); the handle keeps the
    winner. Returns ((L, N), ms, y, zf) with y, zf the winner's result."""
    a = _batch_args(x, sections, K, sig_off, zi, y, zf, sec_off, kmax)
    h = handle or default_handle(a["x"].device.index or 0)
    L, N, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check(lib().sos_tune_batched(h.ptr, a["B"], a["kmax"], a["nsec"], a["x"].numel(),
                                  _p(a["K"]), _p(a["sec_off"]), _p(a["sections"]),
                                  _p(a["sig_off"]), _p(a["x"]), _p(a["y"]), _p(a["zi"]),
                                  _p(a["zf"]), _stream_ptr(a["x"].device), int(reps),
                                  ctypes.byref(L), ctypes.byref(N), ctypes.byref(ms)),
           "sos_tune_batched")
    return (L.value, N.value), ms.value, a["y"], a["zf"]


class BatchGraph:
    """An uneven batch captured into a HIP graph (sos_graph_create_batched).
    The tensors passed here are the graph's buffers: refill them in place and
    call launch() to filter new data with the same shapes and bounds."""

    def __init__(self, x, sections, K, sig_off, zi=None, y=None, zf=None, sec_off=None,
                 kmax=None, handle: Handle | None = None):
        a = _batch_args(x, sections, K, sig_off, zi, y, zf, sec_off, kmax)
        self.args = a
        h = handle or default_handle(a["x"].device.index or 0)
        self._g = ctypes.c_void_p()
        import torch

        torch.cuda.current_stream(a["x"].device).synchronize()
        _check(lib().sos_graph_create_batched(ctypes.byref(self._g), h.ptr, a["B"], a["kmax"],
                                              a["nsec"], a["x"].numel(), _p(a["K"]),
                                              _p(a["sec_off"]), _p(a["sections"]),
                                              _p(a["sig_off"]), _p(a["x"]), _p(a["y"]),
                                              _p(a["zi"]), _p(a["zf"])),
               "sos_graph_create_batched")

    @property
    def y(self):
        return self.args["y"]

    @property
    def zf(self):
        return self.args["zf"]

    def launch(self):
        _check(lib().sos_graph_launch(self._g, _stream_ptr(self.args["x"].device)),
               "sos_graph_launch")

    def last_error(self) -> int:
        return int(lib().sos_graph_last_error(self._g))

    def close(self):
        if self._g:
            lib().sos_graph_destroy(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sosfilt_train(x, sos, zi=None, handle: Handle | None = None):
    """Forward pass that keeps what the adjoint needs: returns (y, zf, saved),
    saved = outputs of sections 0..K-2 ((K-1) x n, empty for K <= 1)."""
    import torch

    x = _as_dev_f32(x, "x").reshape(-1)
    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    K = sos.shape[0]
    if zi is not None:
        zi = _as_dev_f32(zi, "zi").reshape(K, 2)
    y = torch.empty_like(x)
    zf = torch.empty((K, 2), dtype=torch.float32, device=x.device)
    saved = torch.empty((max(K - 1, 0), x.numel()), dtype=torch.float32, device=x.device)
    h = handle or default_handle(x.device.index or 0)
    _check(lib().sos_filter_train(h.ptr, _p(sos), K, _p(x), _p(y), x.numel(), _p(zi), _p(zf),
                                  _p(saved) if saved.numel() else None, _stream_ptr(x.device)),
           "sos_filter_train")
    return y, zf, saved


def sosfilt_vjp(sos, x, y, saved, gy, gzf=None, handle: Handle | None = None):
    """(gx, gzi, gsos) for the forward call that produced y and saved."""
    import torch

    sos = _as_dev_f32(sos, "sos").reshape(-1, 6)
    K = sos.shape[0]
    gy = _as_dev_f32(gy, "gy").reshape(-1)
    if gzf is not None:
        gzf = _as_dev_f32(gzf, "gzf").reshape(K, 2)
    gx = torch.empty_like(gy)
    gzi = torch.empty((K, 2), dtype=torch.float32, device=gy.device)
    gsos = torch.empty((K, 6), dtype=torch.float32, device=gy.device)
    h = handle or default_handle(gy.device.index or 0)
    _check(lib().sos_filter_vjp(h.ptr, _p(sos), K, _p(x), _p(y),
                                _p(saved) if saved is not None and saved.numel() else None,
                                gy.numel(), _p(gy), _p(gzf), _p(gx), _p(gzi), _p(gsos),
                                _stream_ptr(gy.device)), "sos_filter_vjp")
    return gx, gzi, gsos


def _autograd_fn():
    import torch

    class SosFilterFn(torch.autograd.Function):
        """Differentiable cascade: forward = sos_filter_train, backward =
        sos_filter_vjp (hand-written adjoint kernel)."""

        @staticmethod
        def forward(ctx, x, sos, zi):
            y, zf, saved = sosfilt_train(x, sos, zi)
            ctx.save_for_backward(x, sos, y, saved)
            return y, zf

        @staticmethod
        def backward(ctx, gy, gzf):
            x, sos, y, saved = ctx.saved_tensors
            if gy is None:
                gy = torch.zeros_like(y)
            gx, gzi, gsos = sosfilt_vjp(sos, x.contiguous(), y, saved, gy.contiguous(),
                                        None if gzf is None else gzf.contiguous())
            return gx, gsos, gzi

    class SosFilterBatchFn(torch.autograd.Function):
        """A batch of equal-length signals x (B x n): forward =
        sos_filter_train_batched, backward = sos_filter_vjp_batched (one
        persistent adjoint launch for the whole batch). sos is K x 6 (shared
        by the batch: its gradient is summed over the signals by the library,
        sos_filter_vjp_batched_sum) or B x K x 6; zi is B x K x 2."""

        @staticmethod
        def forward(ctx, x, sos, zi):
            B, n = x.shape
            K = sos.shape[-2]
            rows = (sos.expand(B, K, 6) if sos.dim() == 2 else sos).reshape(B * K, 6).contiguous()
            dev = x.device
            Ks = torch.full((B,), K, dtype=torch.int32, device=dev)
            sig_off = torch.arange(B + 1, dtype=torch.int64, device=dev) * n
            sec_off = torch.arange(B + 1, dtype=torch.int32, device=dev) * K
            xf = x.reshape(-1).contiguous()
            y, zf, saved = sosfilt_train_batched(xf, rows, Ks, sig_off, zi.reshape(-1, 2),
                                                 sec_off=sec_off, kmax=K)
            ctx.save_for_backward(xf, rows, Ks, sig_off, sec_off, y, saved)
            ctx.shape = (B, n, K, sos.dim())
            return y.reshape(B, n), zf.reshape(B, K, 2)

        @staticmethod
        def backward(ctx, gy, gzf):
            xf, rows, Ks, sig_off, sec_off, y, saved = ctx.saved_tensors
            B, n, K, sdim = ctx.shape
            gy = torch.zeros_like(y) if gy is None else gy.reshape(-1).contiguous()
            gzf = None if gzf is None else gzf.reshape(-1, 2).contiguous()
            gx, gzi, gs = sosfilt_vjp_batched(rows, Ks, sig_off, xf, y, saved, gy, gzf,
                                              sec_off=sec_off, kmax=K, shared=sdim == 2)
            return gx.reshape(B, n), gs.reshape(K, 6) if sdim == 2 else gs.reshape(B, K, 6), \
                gzi.reshape(B, K, 2)

    return SosFilterFn, SosFilterBatchFn


_fn = None


def sosfilt_autograd(x, sos, zi=None):
    """y, zf with gradients flowing to x, sos and zi through the adjoint kernel.
    x of shape (n,) with sos K x 6 and zi K x 2, or a batch x of shape (B, n)
    with sos K x 6 (shared) or B x K x 6 and zi B x K x 2."""
    import torch

    global _fn
    if _fn is None:
        _fn = _autograd_fn()
    K = sos.shape[-2]
    if x.dim() == 2:
        if zi is None:
            zi = torch.zeros((x.shape[0], K, 2), dtype=torch.float32, device=x.device)
        return _fn[1].apply(x, sos, zi)
    if zi is None:
        zi = torch.zeros((K, 2), dtype=torch.float32, device=x.device)
    return _fn[0].apply(x, sos, zi)


class Server:
    """Continuous-batching server over the C ABI (sos_server_* / sos_stream_*).

    Streams keep their sections, tables and TDF-II state on the device; chunks
    are float32 CUDA tensors that must stay alive until `wait` returns for
    them (the server keeps a reference to each pushed chunk and output until
    then). The tile, compute type and lookback bound come from `handle` (or a
    new handle made with `tile` / `precision`)."""

    def __init__(self, handle: Handle | None = None, budget: int = 0, max_slots: int = 1024,
                 device: int = 0, tile=None, precision: int = 0):
        h = handle or Handle(device, tile=tile, precision=precision)
        self.device = h.device
        self._s = ctypes.c_void_p()
        _check(lib().sos_server_create(ctypes.byref(self._s), h.ptr, int(budget), int(max_slots)),
               "sos_server_create")
        self._keep = {}
        self._K = {}

    @property
    def ptr(self):
        if not self._s:
            raise SosError(SOS_ECLOSED, "server is closed")
        return self._s

    def limits(self):
        r, c = ctypes.c_int64(), ctypes.c_int64()
        L, N = ctypes.c_int(), ctypes.c_int()
        _check(lib().sos_server_limits(self.ptr, ctypes.byref(r), ctypes.byref(c), ctypes.byref(L),
                                       ctypes.byref(N)), "sos_server_limits")
        return {"max_rows": r.value, "max_chunk": c.value, "tile": (L.value, N.value)}

    def open(self, sections, zi=None) -> int:
        """Open a stream; sections (K x 6) and zi (K x 2) are host arrays."""
        import numpy as np

        sec = np.ascontiguousarray(np.asarray(sections, dtype=np.float32).reshape(-1, 6))
        z = None if zi is None else np.ascontiguousarray(np.asarray(zi, dtype=np.float32))
        if z is not None and z.size != 2 * sec.shape[0]:
            raise ValueError("zi must hold K x 2 values")
        sid = ctypes.c_int64()
        _check(lib().sos_stream_open(self.ptr, sec.ctypes.data if sec.size else None, sec.shape[0],
                                     None if z is None else z.ctypes.data, ctypes.byref(sid)),
               "sos_stream_open")
        self._K[sid.value] = sec.shape[0]
        return sid.value

    def push(self, stream_id: int, chunk, out=None):
        """Enqueue a chunk (1-D float32 CUDA tensor); returns (ticket, out)."""
        import torch

        if chunk.dtype != torch.float32 or not chunk.is_cuda or not chunk.is_contiguous():
            raise TypeError("chunk must be a contiguous float32 CUDA tensor")
        if out is None:
            out = torch.empty_like(chunk)
        tk = ctypes.c_uint64()
        # the caller's stream must have produced `chunk` before the server reads it
        torch.cuda.current_stream(chunk.device).synchronize()
        _check(lib().sos_stream_push(self.ptr, int(stream_id), _p(chunk), chunk.numel(), _p(out),
                                     ctypes.byref(tk)), "sos_stream_push")
        self._keep[tk.value] = (chunk, out)
        return tk.value, out

    def wait(self, ticket: int) -> float:
        """Block until the chunk is done; returns its latency in seconds."""
        lat = ctypes.c_double()
        rc = lib().sos_stream_wait(self.ptr, ctypes.c_uint64(ticket), ctypes.byref(lat))
        self._keep.pop(ticket, None)
        _check(rc, "sos_stream_wait")
        return lat.value

    def state(self, stream_id: int):
        import numpy as np

        buf = np.zeros((max(self._K.get(int(stream_id), 0), 1), 2), dtype=np.float32)
        _check(lib().sos_stream_state(self.ptr, int(stream_id), buf.ctypes.data),
               "sos_stream_state")
        return buf[:self._K.get(int(stream_id), 0)]

    def close_stream(self, stream_id: int):
        _check(lib().sos_stream_close(self.ptr, int(stream_id)), "sos_stream_close")
        self._K.pop(int(stream_id), None)

    def replay(self, stream_ids, offs, lens, arrival_s, x, y):
        """Native load driver; returns (latencies [s] per chunk, wall seconds)."""
        import numpy as np

        ids = np.ascontiguousarray(stream_ids, dtype=np.int64)
        o = np.ascontiguousarray(offs, dtype=np.int64)
        n = np.ascontiguousarray(lens, dtype=np.int64)
        t = np.ascontiguousarray(arrival_s, dtype=np.float64)
        lat = np.zeros(len(ids), dtype=np.float64)
        wall = ctypes.c_double()
        import torch

        torch.cuda.current_stream(x.device).synchronize()
        _check(lib().sos_server_replay(self.ptr, len(ids), ids.ctypes.data, o.ctypes.data,
                                       n.ctypes.data, t.ctypes.data, _p(x), _p(y), lat.ctypes.data,
                                       ctypes.byref(wall)), "sos_server_replay")
        return lat, wall.value

    def close(self):
        if self._s:
            lib().sos_server_destroy(self._s)
            self._s = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
