"""FP64 sequential reference for cascaded biquad filtering.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``. The product path (the HIP library
and its Python binding) never imports, links or calls anything here, and this
package imports nothing from the product.

The arithmetic lives in ``sos_oracle.c`` (plain C, double precision, no
fast-math); this module compiles it with gcc on first use and wraps it for
numpy arrays. Definitions followed:

* ``sosfilt``      -- Eq. (1) of Zhai & Paris Part II (Sec. II-A): a cascade of
  K biquads, section k's output is section k+1's input, each section evaluated
  sequentially in transposed direct form II after dividing its row by a0.
  zi/zf are the per-section TDF-II states (the scipy ``sosfilt`` convention).
* ``sosfilt_vjp``  -- reverse-mode derivative of that same sequential program
  (the paper has no gradient; this is the definition of one).
* ``sosfilt_batched`` -- the same filter on independent signals, spread over
  a pool of host threads (only for timing the CPU baseline).

Parity status: every function here is pinned by tests/test_oracle_pins.py
(closed-form impulse responses, steady-state sinusoid gain, superposition,
chunk chaining, dense solve of the paper's multi-block system, scipy's
sosfilt, finite differences for the gradient).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile sos_oracle.c into liboracle.so with gcc (-O2, IEEE semantics)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.oracle_sosfilt.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int64, _dp, _dp, _dp]
            lib.oracle_sosfilt.restype = ctypes.c_int
            lib.oracle_sosfilt_vjp.argtypes = [_dp, ctypes.c_int, _dp, ctypes.c_int64, _dp,
                                               _dp, _dp, _dp, _dp, _dp]
            lib.oracle_sosfilt_vjp.restype = ctypes.c_int
            lib.oracle_sosfilt_batched.argtypes = [ctypes.c_int, _i32p, _i64p, _dp, _i64p, _dp,
                                                   _dp, _dp, _dp, ctypes.c_int]
            lib.oracle_sosfilt_batched.restype = ctypes.c_int
            _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def sosfilt(sos, x, zi=None):
    """Filter x (1-D) with the K x 6 cascade sos; returns (y, zf) in float64.

    Inputs are promoted to float64 exactly (float32 values stay exact)."""
    sos = _f64(sos).reshape(-1, 6)
    x = _f64(x).reshape(-1)
    K = sos.shape[0]
    zi_a = None if zi is None else _f64(zi).reshape(K, 2)
    y = np.empty_like(x)
    zf = np.empty((K, 2), dtype=np.float64)
    rc = _load().oracle_sosfilt(_ptr(sos), K, _ptr(x), x.size, _ptr(zi_a), _ptr(y), _ptr(zf))
    if rc != 0:
        raise ValueError("oracle_sosfilt failed with code %d" % rc)
    return y, zf


def sosfilt_vjp(sos, x, zi, gy, gzf=None):
    """Gradients of <gy, y> + <gzf, zf> w.r.t. (x, zi, sos), all float64."""
    sos = _f64(sos).reshape(-1, 6)
    x = _f64(x).reshape(-1)
    K = sos.shape[0]
    zi_a = None if zi is None else _f64(zi).reshape(K, 2)
    gy = _f64(gy).reshape(-1)
    assert gy.size == x.size
    gzf_a = None if gzf is None else _f64(gzf).reshape(K, 2)
    gx = np.empty_like(x)
    gzi = np.empty((K, 2), dtype=np.float64)
    gsos = np.empty((K, 6), dtype=np.float64)
    rc = _load().oracle_sosfilt_vjp(_ptr(sos), K, _ptr(x), x.size, _ptr(zi_a), _ptr(gy),
                                    _ptr(gzf_a), _ptr(gx), _ptr(gzi), _ptr(gsos))
    if rc != 0:
        raise ValueError("oracle_sosfilt_vjp failed with code %d" % rc)
    return gx, gzi, gsos


def sosfilt_batched(Ks, sos_rows, sig_off, x, zi=None, nthreads=1):
    """Independent signals: signal i is x[sig_off[i]:sig_off[i+1]] filtered by
    the Ks[i] rows of sos_rows starting at sum(Ks[:i]). Returns (y, zf)."""
    Ks = np.ascontiguousarray(np.asarray(Ks, dtype=np.int32))
    B = Ks.size
    sec_off = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(Ks, out=sec_off[1:])
    sos_rows = _f64(sos_rows).reshape(-1, 6)
    sig_off = np.ascontiguousarray(np.asarray(sig_off, dtype=np.int64))
    x = _f64(x).reshape(-1)
    zi_a = None if zi is None else _f64(zi).reshape(-1)
    y = np.empty_like(x)
    zf = np.empty(2 * int(sec_off[-1]), dtype=np.float64)
    rc = _load().oracle_sosfilt_batched(
        B, Ks.ctypes.data_as(_i32p), sec_off.ctypes.data_as(_i64p), _ptr(sos_rows),
        sig_off.ctypes.data_as(_i64p), _ptr(x), _ptr(y), _ptr(zi_a), _ptr(zf), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_sosfilt_batched failed with code %d" % rc)
    return y, zf.reshape(-1, 2)
