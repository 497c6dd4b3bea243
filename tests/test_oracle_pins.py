"""The FP64 oracle against closed forms, invariants, the paper's dense
multi-block system, scipy and finite differences (see tests/pins.py)."""
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("check", pins.ALL_FORWARD, ids=lambda c: c.__name__)
def test_forward_pin(check):
    check(oracle.sosfilt)


def test_vjp_finite_differences():
    pins.check_vjp_finite_differences(oracle.sosfilt, oracle.sosfilt_vjp)


def test_batched_equals_single():
    import numpy as np
    import workloads

    Ks, rows, sig_off, zi = workloads.uneven_batch(B=9, log2_lo=3, log2_hi=11, seed=5)
    x = workloads.batch_signal(int(sig_off[-1]), seed=6).astype(np.float64)
    y, zf = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi, nthreads=3)
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(len(Ks)):
        yi, zfi = oracle.sosfilt(rows[so[i]:so[i + 1]], x[sig_off[i]:sig_off[i + 1]],
                                 zi[so[i]:so[i + 1]])
        assert np.array_equal(yi, y[sig_off[i]:sig_off[i + 1]])
        assert np.array_equal(zfi, zf[so[i]:so[i + 1]])


def test_fp32_gzi_yardstick_is_the_reverse_sweep():
    """The FP32 yardstick the GPU tests hold initial-state gradients to, run
    in FP64, reproduces the oracle's initial-state gradient (the reverse
    sweep, itself pinned by finite differences): it computes the quantity it
    measures the FP32 error of."""
    import numpy as np

    import oracle
    import workloads
    from tests.gpu_util import sequential_gzi

    g = workloads.rng(41)
    for K, n in ((1, 50), (3, 700), (8, 5000)):
        sos = workloads.random_stable_sos(K, g)
        x = workloads.signal(n, seed=42)
        zi = workloads.initial_state(K, g)
        gy = workloads.signal(n, seed=43)
        gzf = workloads.initial_state(K, g, var=1.0)
        _, rzi, _ = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
        got = sequential_gzi(sos, gy, gzf, np.float64)
        assert np.max(np.abs(got - rzi)) <= 1e-10 * max(1.0, np.max(np.abs(rzi))), (K, n)


def test_fp32_gs_yardstick_is_the_reverse_sweep():
    """The FP32 yardstick for coefficient gradients, run in FP64, reproduces
    the oracle's coefficient gradient, also for rows scaled so that a0 != 1
    and for non-zero initial states."""
    import numpy as np

    import oracle
    import workloads
    from tests.gpu_util import sequential_gs

    g = workloads.rng(44)
    for K, n in ((1, 60), (3, 700), (8, 5000)):
        sos = workloads.random_stable_sos(K, g) * g.uniform(0.5, 2.0, size=(K, 1))
        x = workloads.signal(n, seed=45)
        zi = workloads.initial_state(K, g)
        gy = workloads.signal(n, seed=46)
        _, _, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
        got = sequential_gs(sos, x, zi, gy, np.float64)
        assert np.max(np.abs(got - rs)) <= 1e-9 * max(1.0, np.max(np.abs(rs))), (K, n)
