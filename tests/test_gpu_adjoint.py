"""GPU parity of the adjoint (sos_filter_train + sos_filter_vjp and the
autograd Function) against the FP64 oracle's reverse sweep, which is itself
pinned by central finite differences (tests/test_oracle_pins.py)."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def gpu_vjp(torch, P, sos, x, zi, gy, gzf, tile=None, precision=0):
    h = P.Handle(0, tile=tile, precision=precision)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    y, zf, saved = P.sosfilt_train(d(x), d(sos), d(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp(d(sos), d(x), y, saved, d(gy), d(gzf), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    return gx.cpu().numpy(), gzi.cpu().numpy(), gs.cpu().numpy()


@pytest.mark.parametrize("tile", [(64, 16), (256, 32), (512, 16)])
@pytest.mark.parametrize("K,n", [(1, 5000), (2, 70001), (4, 1 << 16), (4, 3), (3, 1)])
def test_vjp_matches_oracle(env, K, n, tile):
    torch, P = env
    g = workloads.rng(100 + K + n % 97)
    sos = workloads.random_stable_sos(K, g)
    sos[0] *= 1.25                                       # a0 != 1
    x = workloads.signal(n, seed=7)
    zi = workloads.initial_state(K, g)
    gy = workloads.signal(n, seed=8)
    gzf = workloads.initial_state(K, g, var=1.0)
    gx, gzi, gs = gpu_vjp(torch, P, sos, x, zi, gy, gzf, tile)
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
    print("K", K, "n", n, "tile", tile, rel_l2(gx, rx), rel_l2(gzi, rzi), rel_l2(gs, rs))
    assert rel_l2(gx, rx) <= 1e-5
    assert rel_l2(gzi, rzi) <= 1e-5
    assert rel_l2(gs, rs) <= 1e-4


@pytest.mark.parametrize("tile", [(512, 32), (64, 16)])
def test_vjp_small_grid(env, tile, monkeypatch):
    """Two workgroups for the whole reversed-time pass: each draws many
    tickets, including the first group of the signal last."""
    torch, P = env
    monkeypatch.setenv("SOS_GRID", "2")
    L, N = tile
    K, n = 4, 5 * L * N + 77
    g = workloads.rng(130)
    sos = workloads.random_stable_sos(K, g)
    x = workloads.signal(n, seed=17)
    zi = workloads.initial_state(K, g)
    gy = workloads.signal(n, seed=18)
    gzf = workloads.initial_state(K, g, var=1.0)
    gx, gzi, gs = gpu_vjp(torch, P, sos, x, zi, gy, gzf, tile)
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
    assert rel_l2(gx, rx) <= 1e-5
    assert rel_l2(gzi, rzi) <= 1e-5
    assert rel_l2(gs, rs) <= 1e-4


@pytest.mark.parametrize("precision", [64, 32])
def test_vjp_order16_lightly_damped(env, precision):
    """8 sections, poles at radius 0.995, section 0 scaled to unit white-noise
    gain (the differentiation workload's stress case). FP64 compute meets the
    order-16 bound with room to spare; the default handle (FP32 samples, FP64
    state path and coefficient sums) meets it for gx, gzi and every
    coefficient gradient."""
    import scipy.signal

    torch, P = env
    g = workloads.rng(9)
    sos = workloads.random_stable_sos(8, g, r_fixed=0.995)
    h = np.zeros(20000)
    h[0] = 1.0
    hr, _ = oracle.sosfilt(sos, h)
    sos[0, :3] /= np.sqrt(np.sum(hr ** 2))
    n = 1 << 16
    x = workloads.signal(n, seed=10)
    zi = np.zeros((8, 2), np.float32)
    gy = workloads.signal(n, seed=11)
    gx, gzi, gs = gpu_vjp(torch, P, sos, x, zi, gy, np.zeros((8, 2), np.float32),
                          precision=precision)
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
    # with zero final-state cotangent, gx is the cascade applied to gy in reversed time
    seq = scipy.signal.sosfilt(sos[::-1].astype(np.float32), gy[::-1].astype(np.float32))[::-1]
    print("order16 precision", precision, rel_l2(gx, rx), rel_l2(gzi, rzi), rel_l2(gs, rs),
          "fp32 sequential floor", rel_l2(seq, rx))
    if precision == 64:
        assert rel_l2(gx, rx) <= 1e-5
        assert rel_l2(gzi, rzi) <= 1e-5
        assert rel_l2(gs, rs) <= 1e-5
    else:
        assert rel_l2(gx, rx) <= 1e-4
        assert rel_l2(gzi, rzi) <= 1e-4
        assert rel_l2(gs, rs) <= 1e-4


def test_autograd_function(env):
    torch, P = env
    K, n = 4, 40000
    sos = workloads.sweep_sections(K, "butter")
    x = workloads.signal(n, seed=3)
    zi = workloads.initial_state(K, workloads.rng(4))
    gy = workloads.signal(n, seed=5)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    st = torch.tensor(sos, device="cuda", requires_grad=True)
    zt = torch.tensor(zi, device="cuda", requires_grad=True)
    y, zf = P.sosfilt_autograd(xt, st, zt)
    (y * torch.tensor(gy, device="cuda")).sum().backward()
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
    assert rel_l2(xt.grad.cpu().numpy(), rx) <= 1e-5
    assert rel_l2(zt.grad.cpu().numpy(), rzi) <= 1e-5
    assert rel_l2(st.grad.cpu().numpy(), rs) <= 1e-4


@pytest.mark.parametrize("tile,precision", [(None, 64), ((64, 16), 64), ((256, 32), 64),
                                            (None, 32), ((256, 32), 32)])
def test_batched_vjp_matches_oracle(env, tile, precision):
    """Uneven batch (empty and one-sample signals included): the batched
    adjoint per signal against the oracle's reverse sweep run signal by signal.
    FP64 compute meets the order bounds; FP32 equals the single-signal adjoint
    on every signal (same kernels through the batch plumbing) and stays within
    1e-3 of the oracle (random order-16 cascades reach 1.4e-4 in the final-state
    cotangent of short signals, identically in both FP32 paths)."""
    torch, P = env
    from tests.gpu_util import tol_for

    Ks, rows, sig_off, zi = workloads.uneven_batch(B=24, log2_lo=0, log2_hi=15.6, seed=81)
    lens = np.diff(sig_off)
    lens[3] = 0
    lens[4] = 1
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    total = int(sig_off[-1])
    g = workloads.rng(82)
    x = workloads.batch_signal(total, seed=83)
    gy = workloads.batch_signal(total, seed=84)
    gzf = workloads.initial_state(int(Ks.sum()), g, var=1.0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, tile=tile, precision=precision)
    Kd, sd = dev(Ks.astype(np.int32)), dev(sig_off)
    y, zf, saved = P.sosfilt_train_batched(dev(x), dev(rows), Kd, sd, zi=dev(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp_batched(dev(rows), Kd, sd, dev(x), y, saved, dev(gy), dev(gzf),
                                        handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    gx, gzi, gs = gx.cpu().numpy(), gzi.cpu().numpy(), gs.cpu().numpy()
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(len(Ks)):
        a, b = sig_off[i], sig_off[i + 1]
        r, zi_i, gzf_i = rows[so[i]:so[i + 1]], zi[so[i]:so[i + 1]], gzf[so[i]:so[i + 1]]
        rx, rzi, rs = oracle.sosfilt_vjp(r, x[a:b], zi_i, gy[a:b], gzf_i)
        e = (rel_l2(gx[a:b], rx) if b > a else 0.0, rel_l2(gzi[so[i]:so[i + 1]], rzi),
             rel_l2(gs[so[i]:so[i + 1]], rs))
        if precision == 64:
            assert max(e) <= tol_for(int(Ks[i])), (i, Ks[i], b - a, e)
            continue
        assert max(e) <= 1e-3, (i, Ks[i], b - a, e)
        if b > a:
            # the batch's own tile: with none set, the one-signal forward
            # picks a smaller tile for short signals and rounds differently
            hp = P.Handle(0, tile=tile or h.tile())
            yp, _, sp = P.sosfilt_train(dev(x[a:b]), dev(r), dev(zi_i), handle=hp)
            gxp, gzip, gsp = P.sosfilt_vjp(dev(r), dev(x[a:b]), yp, sp, dev(gy[a:b]), dev(gzf_i),
                                           handle=hp)
            torch.cuda.synchronize()
            assert rel_l2(gx[a:b], gxp.cpu().numpy()) <= 1e-6, i
            assert rel_l2(gzi[so[i]:so[i + 1]], gzip.cpu().numpy()) <= 1e-6, i
            assert rel_l2(gs[so[i]:so[i + 1]], gsp.cpu().numpy()) <= 1e-6, i


def test_batch_autograd_shared_coefficients(env):
    """256-signal x 2^12-sample batch sharing one order-8 cascade: gradients
    of x, zi and the shared coefficients (summed over the batch) against the
    oracle on 4 signals and the exact sum over all."""
    torch, P = env
    B, n, K = 256, 1 << 12, 4
    sos = workloads.sweep_sections(K, "butter")
    g = workloads.rng(85)
    x = workloads.batch_signal(B * n, seed=86).reshape(B, n)
    zi = workloads.initial_state(B * K, g).reshape(B, K, 2)
    gy = workloads.batch_signal(B * n, seed=87).reshape(B, n)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    st = torch.tensor(sos, device="cuda", requires_grad=True)
    zt = torch.tensor(zi, device="cuda", requires_grad=True)
    y, zf = P.sosfilt_autograd(xt, st, zt)
    (y * torch.tensor(gy, device="cuda")).sum().backward()
    gx, gz, gs = xt.grad.cpu().numpy(), zt.grad.cpu().numpy(), st.grad.cpu().numpy()
    total = np.zeros((K, 6))
    for i in range(B):
        rx, rzi, rs = oracle.sosfilt_vjp(sos, x[i], zi[i], gy[i], None)
        total += rs
        if i in (0, 1, 128, 255):
            assert rel_l2(gx[i], rx) <= 1e-5, i
            assert rel_l2(gz[i], rzi) <= 1e-5, i
    assert rel_l2(gs, total) <= 1e-5


def test_vjp_batched_sum_is_the_fp64_sum_of_rows(env):
    """sos_filter_vjp_batched_sum against the per-row gradients of
    sos_filter_vjp_batched from the same forward, summed in FP64 on the host:
    an uneven batch of one order-8 cascade where some signals run only its
    first sections (their rows are a prefix), with an empty signal."""
    torch, P = env
    sos = workloads.sweep_sections(4, "butter")
    Ks = np.array([4, 4, 2, 4, 1, 4, 3, 4, 4, 4], np.int32)
    lens = np.array([5000, 70000, 1, 0, 33000, 4096, 12345, 65536, 2, 20000], np.int64)
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    rows = np.concatenate([sos[:k] for k in Ks])
    total = int(sig_off[-1])
    g = workloads.rng(88)
    x = workloads.batch_signal(total, seed=89)
    gy = workloads.batch_signal(total, seed=90)
    zi = workloads.initial_state(int(Ks.sum()), g)
    gzf = workloads.initial_state(int(Ks.sum()), g, var=1.0)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0)
    Kd, sd = dev(Ks), dev(sig_off)
    y, zf, saved = P.sosfilt_train_batched(dev(x), dev(rows), Kd, sd, zi=dev(zi), handle=h)
    args = (dev(rows), Kd, sd, dev(x), y, saved, dev(gy), dev(gzf))
    gx, gzi, gs = P.sosfilt_vjp_batched(*args, handle=h)
    gx2, gzi2, gsum = P.sosfilt_vjp_batched(*args, handle=h, shared=True)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    assert tuple(gsum.shape) == (4, 6)
    assert torch.equal(gx, gx2) and torch.equal(gzi, gzi2)
    gs = gs.cpu().numpy().astype(np.float64)
    so = np.r_[0, np.cumsum(Ks)]
    ref = np.zeros((4, 6))
    for i, k in enumerate(Ks):
        ref[:k] += gs[so[i]:so[i + 1]]
    got = gsum.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-6 * np.abs(ref).max(axis=1, keepdims=True) + 1e-30)


def test_vjp_batched_skips_an_inconsistent_signal(env):
    """A signal whose section offset runs past the rows is skipped and
    reported by the batched adjoint: its coefficient-gradient rows are not
    written (a guard region after the gradient rows keeps its sentinel), its
    gx is left alone, and the other signals' gradients equal those of the
    consistent call."""
    import ctypes

    torch, P = env
    rng = workloads.rng(91)
    B, K = 3, 2
    rows = np.concatenate([workloads.random_stable_sos(K, rng) for _ in range(B)])
    R = rows.shape[0]
    Ks = np.full(B, K, dtype=np.int32)
    so = (np.arange(B + 1) * K).astype(np.int32)
    lens = np.array([3000, 2500, 4000], np.int64)
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    n = int(sig_off[-1])
    x = workloads.batch_signal(n, seed=92)
    gy = workloads.batch_signal(n, seed=93)
    zi = workloads.initial_state(R, rng)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0)
    xd, rd, Kd, sd = dev(x), dev(rows), dev(Ks), dev(sig_off)
    y, zf, saved = P.sosfilt_train_batched(xd, rd, Kd, sd, zi=dev(zi), sec_off=dev(so), kmax=K,
                                           handle=h)
    gx_ref, gzi_ref, gs_ref = P.sosfilt_vjp_batched(rd, Kd, sd, xd, y, saved, dev(gy),
                                                    sec_off=dev(so), kmax=K, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    so_bad = so.copy()
    so_bad[1] = R - 1                                  # so + K = R + 1 > R
    gx = torch.full((n,), 7.0, device="cuda")
    gzi = torch.zeros((R, 2), device="cuda")
    gs_full = torch.full((R + 4, 6), 7.0, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    sod, gyd = dev(so_bad), dev(gy)                    # kept alive while the launch runs
    rc = P.lib().sos_filter_vjp_batched(h.ptr, B, K, R, n, p(Kd), p(sod), p(rd), p(sd), p(xd),
                                        p(y), p(saved), p(gyd), None, p(gx), p(gzi),
                                        p(gs_full), P._stream_ptr())
    torch.cuda.synchronize()
    assert rc == P.SOS_OK and h.last_error() == P.SOS_EINVAL
    assert torch.all(gs_full[R:] == 7.0).item()
    a, b = int(sig_off[1]), int(sig_off[2])
    assert torch.all(gx[a:b] == 7.0).item()
    for i in (0, 2):
        a, b = int(sig_off[i]), int(sig_off[i + 1])
        assert rel_l2(gx[a:b].cpu().numpy(), gx_ref[a:b].cpu().numpy()) <= 1e-6, i
        r0, r1 = int(so[i]), int(so[i + 1])
        assert rel_l2(gs_full[r0:r1].cpu().numpy(), gs_ref[r0:r1].cpu().numpy()) <= 1e-6, i
