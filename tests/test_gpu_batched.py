"""GPU parity of the uneven-batch entry point (sos_filter_batched): every
signal of the batch against the FP64 oracle, the same result alone and in the
mix, empty and zero-section signals, and rejection of inconsistent entries."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, rel_l2, tol_for, zf_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def dev(torch, a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_batch(torch, P, Ks, rows, sig_off, x, zi, tile=None, precision=0):
    h = P.Handle(0, tile=tile, precision=precision)
    y, zf = P.sosfilt_batched(dev(torch, x), dev(torch, rows), dev(torch, Ks.astype(np.int32)),
                              dev(torch, sig_off.astype(np.int64)),
                              zi=None if zi is None else dev(torch, zi), handle=h)
    torch.cuda.synchronize()
    return y.cpu().numpy(), zf.cpu().numpy(), h.last_error()


@pytest.mark.parametrize("tile,precision", [((64, 16), 32), ((256, 32), 32), ((512, 32), 32),
                                            ((1024, 32), 32), ((512, 32), 64)])
def test_uneven_batch_matches_oracle(env, tile, precision):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=96, log2_lo=2, log2_hi=17, seed=11)
    x = workloads.batch_signal(int(sig_off[-1]), seed=12)
    y, zf, err = run_batch(torch, P, Ks, rows, sig_off, x, zi, tile, precision)
    assert err == P.SOS_OK
    yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi, nthreads=8)
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(len(Ks)):
        a, b = sig_off[i], sig_off[i + 1]
        rows_i = rows[so[i]:so[i + 1]]
        zi_i = zi[so[i]:so[i + 1]]
        by = bz = tol_for(int(Ks[i]))
        if precision != 64 and b > a:
            by, bz = fp32_bounds(int(Ks[i]), rows_i, x[a:b], zi_i, yr[a:b],
                                 zfr[so[i]:so[i + 1]])
        e = rel_l2(y[a:b], yr[a:b])
        assert e <= by, (i, Ks[i], b - a, e)
        ez = rel_l2(zf[so[i]:so[i + 1]], zfr[so[i]:so[i + 1]])
        bz = zf_bound(int(Ks[i]), by, bz, yr[a:b], zfr[so[i]:so[i + 1]])
        assert ez <= bz, (i, Ks[i], b - a, ez)


def test_alone_equals_in_the_mix(env):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=40, log2_lo=8, log2_hi=16, seed=21)
    x = workloads.batch_signal(int(sig_off[-1]), seed=22)
    y, zf, err = run_batch(torch, P, Ks, rows, sig_off, x, zi)
    assert err == P.SOS_OK
    so = np.r_[0, np.cumsum(Ks)]
    for i in (0, 7, 19, 39):
        a, b = sig_off[i], sig_off[i + 1]
        y1, zf1 = P.sosfilt(dev(torch, x[a:b]), dev(torch, rows[so[i]:so[i + 1]]),
                            dev(torch, zi[so[i]:so[i + 1]]))
        torch.cuda.synchronize()
        assert rel_l2(y[a:b], y1.cpu().numpy()) <= 1e-5
        assert rel_l2(zf[so[i]:so[i + 1]], zf1.cpu().numpy()) <= 1e-5


def test_empty_and_zero_section_signals(env):
    torch, P = env
    g = workloads.rng(5)
    lens = np.array([0, 5000, 0, 1, 70000, 3], dtype=np.int64)
    Ks = np.array([2, 0, 0, 3, 1, 2], dtype=np.int32)
    rows = np.concatenate([workloads.random_stable_sos(int(k), g) for k in Ks])
    zi = workloads.initial_state(int(Ks.sum()), g)
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    x = workloads.batch_signal(int(sig_off[-1]), seed=6)
    y, zf, err = run_batch(torch, P, Ks, rows, sig_off, x, zi)
    assert err == P.SOS_OK
    yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi)
    assert rel_l2(y, yr) <= 1e-5
    assert np.allclose(zf, zfr, rtol=1e-5, atol=1e-6)
    a, b = sig_off[1], sig_off[2]
    assert np.array_equal(y[a:b], x[a:b])          # K = 0: copy


def test_inconsistent_signal_is_skipped_and_reported(env):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=6, log2_lo=10, log2_hi=12, seed=31,
                                                   k_lo=1, k_hi=3)
    x = workloads.batch_signal(int(sig_off[-1]), seed=32)
    h = P.Handle(0)
    Kd = Ks.copy()
    Kd[2] = 9                                      # above kmax = 3
    yd = torch.full((x.size,), 7.0, device="cuda")
    P.sosfilt_batched(dev(torch, x), dev(torch, rows), dev(torch, Kd),
                      dev(torch, sig_off), zi=dev(torch, zi), y=yd, kmax=3,
                      sec_off=dev(torch, np.r_[0, np.cumsum(Ks)].astype(np.int32)), handle=h)
    assert h.last_error() == P.SOS_EINVAL
    y = yd.cpu().numpy()
    yr, _ = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi)
    for i in range(6):
        a, b = sig_off[i], sig_off[i + 1]
        if i == 2:
            assert np.all(y[a:b] == 7.0)          # untouched
        else:
            assert rel_l2(y[a:b], yr[a:b]) <= 1e-5


@pytest.mark.parametrize("B", [3, 1500])     # one kernel for the work table, then two
def test_inconsistent_empty_signal_leaves_zf_alone(env, B):
    """An empty signal whose section offset runs past the section rows is
    reported and skipped: its final state is not written, so nothing past
    the end of zf changes (a guard region after zf keeps its sentinel)."""
    torch, P = env
    rng = workloads.rng(33)
    rows = np.concatenate([workloads.random_stable_sos(2, rng) for _ in range(B)])
    R = rows.shape[0]                                  # 2 rows per signal
    Ks = np.full(B, 2, dtype=np.int32)
    so = np.arange(B + 1, dtype=np.int32) * 2
    lens = np.full(B, 300, dtype=np.int64)
    bad = 1
    lens[bad] = 0
    Ks[bad] = 2
    so_bad = so.copy()
    so_bad[bad] = R - 1                                # so + K = R + 1 > R
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    x = workloads.batch_signal(int(sig_off[-1]), seed=34)
    zi = workloads.initial_state(R, rng)
    zf_full = torch.full((R + 4, 2), 7.0, device="cuda")
    zf = zf_full[:R]
    h = P.Handle(0)
    y, _ = P.sosfilt_batched(dev(torch, x), dev(torch, rows), dev(torch, Ks), dev(torch, sig_off),
                             zi=dev(torch, zi), zf=zf, sec_off=dev(torch, so_bad), kmax=2,
                             handle=h)
    assert h.last_error() == P.SOS_EINVAL
    guard = zf_full[R:].cpu().numpy()
    assert np.all(guard == 7.0), guard
    y = y.cpu().numpy()
    for i in (0, B - 1):                               # consistent neighbours still filtered
        a, b = sig_off[i], sig_off[i + 1]
        yr, zfr = oracle.sosfilt(rows[so[i]:so[i] + 2], x[a:b], zi[so[i]:so[i] + 2])
        assert rel_l2(y[a:b], yr) <= 1e-5, i


@pytest.mark.parametrize("alg", ["dccr", "ph"])
@pytest.mark.parametrize("tile", [(512, 64), (256, 32), (64, 16)])
def test_small_grid_many_groups_per_workgroup(env, tile, alg, monkeypatch):
    """Three workgroups for the whole batch: each draws many tickets, so the
    next group is loaded while the current one is corrected and stored across
    signal boundaries, partial last groups, a signal with no sections and a
    signal with an unusable section (which poisons only that signal)."""
    torch, P = env
    monkeypatch.setenv("SOS_GRID", "3")
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=40, log2_lo=2, log2_hi=17, seed=41)
    x = workloads.batch_signal(int(sig_off[-1]), seed=42)
    so = np.r_[0, np.cumsum(Ks)]
    bad = 11                                         # a2 > 1 in its last section
    rows = rows.copy()
    rows[so[bad + 1] - 1, 5] = 1.5 * rows[so[bad + 1] - 1, 3]
    h = P.Handle(0, tile=tile, algorithm=alg)
    Kd = Ks.copy()
    Kd[23] = 0                                       # no sections: a copy
    y, zf = P.sosfilt_batched(dev(torch, x), dev(torch, rows), dev(torch, Kd),
                              dev(torch, sig_off), zi=dev(torch, zi),
                              sec_off=dev(torch, so.astype(np.int32)), kmax=int(Ks.max()),
                              handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_EUNSTABLE
    y, zf = y.cpu().numpy(), zf.cpu().numpy()
    yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi, nthreads=8)
    for i in range(len(Ks)):
        a, b = sig_off[i], sig_off[i + 1]
        if i == bad:
            assert b == a or np.all(np.isnan(y[a:b]))
            continue
        if i == 23:
            assert np.array_equal(y[a:b], x[a:b])
            continue
        rows_i, zi_i = rows[so[i]:so[i + 1]], zi[so[i]:so[i + 1]]
        by = bz = tol_for(int(Ks[i]))
        if b > a:
            by, bz = fp32_bounds(int(Ks[i]), rows_i, x[a:b], zi_i, yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(y[a:b], yr[a:b]) <= by, (i, Ks[i], b - a)
        bz = zf_bound(int(Ks[i]), by, bz, yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(zf[so[i]:so[i + 1]], zfr[so[i]:so[i + 1]]) <= bz, (i, Ks[i], b - a)
