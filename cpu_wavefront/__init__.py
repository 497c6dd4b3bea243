"""Multi-core CPU comparator: the paper's wavefront execution (Sec. III-A).

Reported by ``bench.py`` beside the GPU rate (and by nothing else): a faster,
fairer CPU figure than the single-thread oracle. Plain C with pthreads in
``sos_wavefront.c``, compiled with gcc by ``build()``. It is not part of the
filter library and shares no code with it or with the oracle; its output is
checked against the oracle by ``tests/test_cpu_wavefront.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sos_wavefront.c")
_LIB = os.path.join(_HERE, "libwavefront.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile sos_wavefront.c into libwavefront.so (gcc -O3, x86-64 with AVX2
    and FMA for the 8-wide vectors of the multi-block node kernels)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O3", "-mavx2", "-mfma", "-fPIC", "-shared", "-o", tmp, _SRC,
                           "-lpthread"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = ctypes.CDLL(_LIB)
            vp = ctypes.c_void_p
            L.sos_wavefront.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_int64, vp, vp,
                                        ctypes.c_int64, ctypes.c_int]
            L.sos_wavefront.restype = ctypes.c_int
            L.sos_wavefront_nodes.argtypes = L.sos_wavefront.argtypes + [ctypes.c_int]
            L.sos_wavefront_nodes.restype = ctypes.c_int
            _lib = L
    return _lib


def default_threads() -> int:
    """Host threads this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


NODES = {"serial": 0, "multiblock": 1}


def sosfilt(sos, x, zi=None, group: int = 1 << 16, threads: int | None = None, out=None,
            node: str = "serial"):
    """Cascade filter of float32 x (K x 6 sos rows, K x 2 TDF-II zi) by the
    wavefront over groups of `group` samples, each node the serial filter or
    the multi-block node kernel (`node`). Returns (y, zf) as float32."""
    sos = np.ascontiguousarray(sos, dtype=np.float32).reshape(-1, 6)
    K = sos.shape[0]
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x) if out is None else out
    zf = np.empty((K, 2), dtype=np.float32)
    zi_a = None if zi is None else np.ascontiguousarray(zi, dtype=np.float32).reshape(K, 2)
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    rc = _load().sos_wavefront_nodes(p(sos), K, p(x), p(y), x.size, p(zi_a), p(zf), int(group),
                                     int(threads or default_threads()), NODES[node])
    if rc != 0:
        raise ValueError("sos_wavefront failed (%d)" % rc)
    return y, zf
