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


@pytest.mark.parametrize("threads", [1, 3, 8])
@pytest.mark.parametrize("K", [1, 4, 8])
def test_multiblock_nodes_match_oracle(K, threads):
    """The multi-block node kernels (lanes run from rest, a scan of the lanes'
    states through T^NB, the homogeneous correction) against the oracle:
    whole blocks, a group's serial tail, groups smaller than a block, a0 != 1
    and random initial states. Bounds: the order's, or 10x the error of a
    sequential FP32 filter on the same input."""
    from tests.gpu_util import fp32_bounds

    g = workloads.rng(600 + K)
    for kind in ("butter", "random"):
        sos = workloads.sweep_sections(K, kind) if kind == "butter" else \
            workloads.random_stable_sos(K, g)
        sos = sos * np.float32(1.25)                   # a0 != 1, same filter
        zi = workloads.initial_state(K, g)
        for n, group in ((1, 7), (3000, 1000), (70001, 8192), ((1 << 18) + 5, 1 << 16)):
            x = workloads.signal(n, seed=n + K)
            y, zf = W.sosfilt(sos, x, zi, group=group, threads=threads, node="multiblock")
            yr, zfr = oracle.sosfilt(sos, x, zi)
            by, bz = fp32_bounds(K, sos / sos[:, 3:4], x, zi, yr, zfr)
            assert rel(y, yr) <= max(by, 1e-5 if K <= 4 else 1e-4), (kind, K, n, group)
            assert rel(zf, zfr) <= max(bz, 1e-5 if K <= 4 else 1e-4), (kind, K, n, group)


def test_multiblock_nodes_degenerate_and_in_place():
    sos = workloads.sweep_sections(2, "butter")
    zi = workloads.initial_state(2, workloads.rng(2))
    y, zf = W.sosfilt(sos, np.zeros(0, np.float32), zi, node="multiblock")
    assert y.size == 0 and np.array_equal(zf, zi)
    x = workloads.signal(40000, seed=5)
    xc = x.copy()
    W.sosfilt(sos, xc, zi, group=4096, threads=4, out=xc, node="multiblock")
    yr, _ = oracle.sosfilt(sos, x, zi)
    assert rel(xc, yr) <= 1e-5
    with pytest.raises(KeyError):
        W.sosfilt(sos, x, node="nope")
