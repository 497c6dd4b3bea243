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
