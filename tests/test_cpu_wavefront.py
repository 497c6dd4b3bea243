"""The multi-core CPU comparator (wavefront over groups and sections, Sec.
III-A) reproduces the oracle: FP32 sequential filtering per node, so within
the FP32 floor of the order, for any number of threads and any group size,
including ragged last groups, n = 0, K = 0 and in-place use."""
import numpy as np
import pytest

import cpu_wavefront as W
import oracle
import workloads


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("K", [1, 3, 8])
def test_matches_oracle(K, threads):
    g = workloads.rng(500 + K)
    sos = workloads.random_stable_sos(K, g)
    sos[0] *= 1.5                                      # a0 != 1
    zi = workloads.initial_state(K, g)
    for n, group in ((1, 7), (1000, 64), (12345, 1000), (50000, 4096)):
        x = workloads.signal(n, seed=n)
        y, zf = W.sosfilt(sos, x, zi, group=group, threads=threads)
        yr, zfr = oracle.sosfilt(sos, x, zi)
        assert rel(y, yr) <= 1e-5, (K, threads, n, group)
        assert rel(zf, zfr) <= 1e-5, (K, threads, n, group)


def test_independent_of_threads_and_group_boundaries():
    """The state handed from group to group is exactly the sequential one:
    the FP32 result does not depend on the thread count, and group sizes only
    change where the (exact) hand-over happens."""
    sos = workloads.sweep_sections(4, "butter")
    x = workloads.signal(30001, seed=3)
    ref, zref = W.sosfilt(sos, x, group=30001, threads=1)
    for threads in (2, 5, 16):
        for group in (1, 17, 4096):
            y, zf = W.sosfilt(sos, x, group=group, threads=threads)
            assert np.array_equal(y, ref) and np.array_equal(zf, zref), (threads, group)


def test_degenerate_and_in_place():
    sos = workloads.sweep_sections(2, "butter")
    zi = workloads.initial_state(2, workloads.rng(1))
    y, zf = W.sosfilt(sos, np.zeros(0, np.float32), zi)
    assert y.size == 0 and np.array_equal(zf, zi)
    x = workloads.signal(777, seed=4)
    y, zf = W.sosfilt(np.zeros((0, 6), np.float32), x)
    assert np.array_equal(y, x) and zf.size == 0
    xc = x.copy()
    W.sosfilt(sos, xc, zi, group=100, threads=4, out=xc)
    yr, _ = oracle.sosfilt(sos, x, zi)
    assert rel(xc, yr) <= 1e-5
    bad = sos.copy()
    bad[1, 3] = 0.0
    with pytest.raises(ValueError):
        W.sosfilt(bad, x)
