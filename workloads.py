"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs: filter coefficients, signals and initial
states, plus the shapes of batches and streams. It contains none of the
filtering arithmetic, so the reference and the HIP path can both consume it
without sharing any of the method's code.

Recipes (Zhai & Paris, Part II, Sec. IV-F, and the workload descriptions this
project measures on):

* Butterworth low-pass of order 2K at cutoff 0.2*pi (scipy Wn = 0.2), designed
  directly in second-order sections, rounded to float32 (the paper designs in
  SOS form and stores float32 coefficients).
* Random stable sections: complex pole pair r*exp(+-j*theta) with
  r ~ U[r_lo, r_hi], theta ~ U[0, pi]; zero pair on the unit circle
  exp(+-j*phi), phi ~ U[0, pi]; each section scaled so |H_k| = 1 at the pole
  angle, which keeps cascaded outputs O(1).
* Signals: i.i.d. N(0, 1) float32 from numpy's PCG64 generator.
* Initial states: N(0, 0.1) read as variance 0.1.
"""
from __future__ import annotations

import numpy as np

BUTTER_WN = 0.2


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def butterworth_sos(K: int, wn: float = BUTTER_WN) -> np.ndarray:
    """Order-2K Butterworth low-pass as K x 6 float32 rows [b0 b1 b2 a0 a1 a2]."""
    from scipy.signal import butter

    if K == 0:
        return np.zeros((0, 6), dtype=np.float32)
    sos = butter(2 * K, wn, output="sos")
    return np.ascontiguousarray(sos.astype(np.float32))


def random_stable_sos(K: int, g: np.random.Generator, r_lo: float = 0.5, r_hi: float = 0.99,
                      r_fixed: float | None = None) -> np.ndarray:
    """K random stable sections (float32 rows), zeros on the unit circle."""
    out = np.zeros((K, 6), dtype=np.float64)
    for k in range(K):
        r = r_fixed if r_fixed is not None else g.uniform(r_lo, r_hi)
        th = g.uniform(0.0, np.pi)
        ph = g.uniform(0.0, np.pi)
        b = np.array([1.0, -2.0 * np.cos(ph), 1.0])
        a = np.array([1.0, -2.0 * r * np.cos(th), r * r])
        z = np.exp(-1j * th)
        hb = b[0] + b[1] * z + b[2] * z * z
        ha = a[0] + a[1] * z + a[2] * z * z
        mag = abs(hb / ha)
        if mag < 1e-3:        # zero pair sitting on the pole angle: keep unit numerator
            mag = 1.0
        out[k, :3] = b / mag
        out[k, 3:] = a
    return np.ascontiguousarray(out.astype(np.float32))


def signal(n: int, seed: int) -> np.ndarray:
    """n i.i.d. N(0,1) float32 samples."""
    return rng(seed).standard_normal(n, dtype=np.float32)


def initial_state(K: int, g: np.random.Generator, var: float = 0.1) -> np.ndarray:
    return (g.standard_normal((K, 2)) * np.sqrt(var)).astype(np.float32)


# --------------------------------------------------------------------------
# Workloads with names and sizes
# --------------------------------------------------------------------------

def single_biquad(n: int = 1 << 20, seed: int = 1):
    """One 2nd-order Butterworth section at 0.2*Nyquist, one N(0,1) signal, zi = 0."""
    return butterworth_sos(1), signal(n, seed)


def sweep_sections(K: int, kind: str = "butter", seed: int = 20):
    """Cascade used by the throughput sweep: Butterworth order 2K, or K random
    stable sections drawn from seed + K."""
    if kind == "butter":
        return butterworth_sos(K)
    if kind == "random":
        return random_stable_sos(K, rng(seed + K))
    raise ValueError(kind)


def uneven_batch(B: int = 4096, log2_lo: float = 10.0, log2_hi: float = 22.0, seed: int = 3,
                 k_lo: int = 1, k_hi: int = 8, zi_var: float = 0.1):
    """Uneven batch: lengths floor(2**U), U ~ U[log2_lo, log2_hi]; K_i ~ U{k_lo..k_hi};
    random stable sections per signal; zi ~ N(0, zi_var). Signals are not drawn
    here (they can be large); use batch_signal() for the samples."""
    g = rng(seed)
    lens = np.floor(2.0 ** g.uniform(log2_lo, log2_hi, size=B)).astype(np.int64)
    Ks = g.integers(k_lo, k_hi + 1, size=B).astype(np.int32)
    rows = np.concatenate([random_stable_sos(int(k), g) for k in Ks]) if B else \
        np.zeros((0, 6), np.float32)
    zi = (g.standard_normal((int(Ks.sum()), 2)) * np.sqrt(zi_var)).astype(np.float32)
    sig_off = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(lens, out=sig_off[1:])
    return Ks, rows, sig_off, zi


def batch_signal(total: int, seed: int = 30) -> np.ndarray:
    return signal(total, seed)


def serving_trace(S: int = 1024, R: int | None = None, rate_chunks_per_s: float = 1e5,
                  lo: int = 4096, hi: int = 65536, k_lo: int = 1, k_hi: int = 8,
                  seed: int = 4):
    """Serving load: S streams, stream s filtered by K_s ~ U{k_lo..k_hi} random
    stable sections (zero initial state); R chunks (default 4 per stream) with
    lengths floor(2**U), U ~ U[log2 lo, log2 hi], arriving as a Poisson process
    of the given aggregate rate, each assigned to a uniformly drawn stream
    (a stream's chunks are its arrivals in time order).

    Returns (Ks, sections list, stream_of_chunk, lens, offs, arrival_s) with
    offs the exclusive prefix of lens (one packed sample buffer for all
    chunks)."""
    g = rng(seed)
    Ks = g.integers(k_lo, k_hi + 1, size=S).astype(np.int32)
    sections = [random_stable_sos(int(k), g) for k in Ks]
    R = 4 * S if R is None else R
    lens = np.floor(2.0 ** g.uniform(np.log2(lo), np.log2(hi), size=R)).astype(np.int64)
    ids = g.integers(0, S, size=R).astype(np.int64)
    arrival = np.cumsum(g.exponential(1.0 / rate_chunks_per_s, size=R))
    offs = np.zeros(R, dtype=np.int64)
    np.cumsum(lens[:-1], out=offs[1:])
    return Ks, sections, ids, lens, offs, arrival
