"""Parity at the benchmarked sizes, in the benchmarked launch configurations:
every signal, stream and gradient the benchmark times is compared with the
FP64 oracle (the oracle runs on the host's cores, the data moves in slices so
host memory stays bounded).

* one signal of 2^28 samples (orders 2 and 16, Butterworth and random, with
  the default solver; orders 2 and 8 with the block-Toeplitz kernel): the
  relative L2 error, the paper's gate max |error| / max |reference| < 1e-4
  (Sec. IV-F), and the relative error of every group of C samples, so that a
  single wrong group cannot hide in the whole signal's norm;
* the uneven batch of 4096 signals (about 2e9 samples), autotuned and graph
  captured: every signal and every final state;
* serving: 1024 streams and 20000 chunks of 4096..65536 samples: every
  stream over its concatenated chunks;
* differentiation: 256 signals of 2^16 samples through the batched training
  forward and adjoint (order 8 Butterworth, and the lightly damped order-16
  cascade), every signal's gradients against the oracle's reverse sweep, and
  FP64 central finite differences of the oracle on 4 signals for every
  coefficient, every initial state and 64 input samples (steps in _fd_check).
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import (FLOOR_FACTOR, fp32_bounds, fp32_gs_floor, fp32_gzi_floor,
                             max_over_peak, rel_l2, tol_for, zf_bound)

pytestmark = pytest.mark.gpu

NTHREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def group_errors(y, yr, C):
    """Relative L2 error of every group of C samples (the last one partial)."""
    n = yr.size
    G = -(-n // C)
    pad = G * C - n
    e = np.pad(np.asarray(y, np.float64) - yr, (0, pad)).reshape(G, C)
    r = np.pad(yr, (0, pad)).reshape(G, C)
    return np.linalg.norm(e, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)


@pytest.mark.parametrize("kind,K,alg", [("butter", 1, None), ("butter", 8, None),
                                        ("random", 8, None), ("butter", 1, "toeplitz"),
                                        ("random", 4, "toeplitz")])
def test_2p28_every_group(env, kind, K, alg):
    """2^28 samples with the default handle (the benchmark's plain launch;
    order 16 takes the block-Toeplitz kernel), and with an explicit
    block-Toeplitz handle at lower orders (the sweep's block-Toeplitz legs)."""
    torch, P = env
    sos = workloads.sweep_sections(K, kind)
    n = 1 << 28
    x = workloads.signal(n, seed=2)
    h = P.Handle(0) if alg is None else P.Handle(0, algorithm=alg)
    xd = torch.from_numpy(x).cuda()
    y, zf = P.sosfilt(xd, torch.from_numpy(sos).cuda(), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    L, N = h.tile()
    yh = y.cpu().numpy()
    del y, xd
    yr, zfr = oracle.sosfilt(sos, x)
    e = rel_l2(yh, yr)
    mp = max_over_peak(yh, yr)
    ge = group_errors(yh, yr, L * N)
    print("2^28", kind, "K", K, alg or "default", "rel_l2 %.3e max/peak %.3e groups %d: max %.3e median %.3e"
          % (e, mp, ge.size, ge.max(), np.median(ge)))
    by = tol_for(K)
    if e > by or ge.max() > by:
        by, _ = fp32_bounds(K, sos, x, None, yr, zfr)
    assert e <= by
    assert ge.max() <= by
    assert mp < 1e-4
    assert rel_l2(zf.cpu().numpy(), zfr) <= max(by, tol_for(K))


def test_uneven_batch_every_signal(env):
    """The benchmarked uneven batch (4096 signals, ~2e9 device-drawn samples,
    autotuned tile and solver, captured graph), every signal and final state."""
    torch, P = env
    dev = torch.device("cuda", 0)
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=4096, seed=3)
    B = len(Ks)
    total = int(sig_off[-1])
    gen = torch.Generator(device=dev).manual_seed(3)
    x = torch.randn(total, generator=gen, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    Kd = torch.from_numpy(Ks.astype(np.int32)).to(dev)
    so = torch.from_numpy(sig_off.astype(np.int64)).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    zi_d = torch.from_numpy(zi).to(dev)
    zf = torch.empty_like(zi_d)
    h = P.Handle(0)
    (L, N), _, _, _ = P.tune_batched(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=h, reps=1)
    y.fill_(float("nan"))
    zf.fill_(float("nan"))
    g = P.BatchGraph(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=h)
    g.launch()
    torch.cuda.synchronize()
    assert g.last_error() == P.SOS_OK
    print("tuned tile", (L, N), h.algorithm(), flush=True)
    sec = np.r_[0, np.cumsum(Ks)]
    zfh = zf.cpu().numpy()
    worst = (0.0, -1)
    i0 = 0
    while i0 < B:
        i1, acc = i0, 0
        while i1 < B and (i1 == i0 or acc + (sig_off[i1 + 1] - sig_off[i1]) <= (1 << 27)):
            acc += sig_off[i1 + 1] - sig_off[i1]
            i1 += 1
        a0, a1 = int(sig_off[i0]), int(sig_off[i1])
        xs = x[a0:a1].cpu().numpy()
        ys = y[a0:a1].cpu().numpy()
        yr, zfr = oracle.sosfilt_batched(Ks[i0:i1], rows[sec[i0]:sec[i1]], sig_off[i0:i1 + 1] - a0,
                                         xs, zi[sec[i0]:sec[i1]], nthreads=NTHREADS)
        for i in range(i0, i1):
            a, b = int(sig_off[i] - a0), int(sig_off[i + 1] - a0)
            r0, r1 = sec[i] - sec[i0], sec[i + 1] - sec[i0]
            k = int(Ks[i])
            e = rel_l2(ys[a:b], yr[a:b])
            ez = rel_l2(zfh[sec[i]:sec[i + 1]], zfr[r0:r1])
            by = bz = tol_for(k)
            if e > by or ez > bz:
                by, bz = fp32_bounds(k, rows[sec[i]:sec[i + 1]], xs[a:b], zi[sec[i]:sec[i + 1]],
                                     yr[a:b], zfr[r0:r1])
                bz = zf_bound(k, by, bz, yr[a:b], zfr[r0:r1])
            assert e <= by, (i, k, b - a, e, by)
            assert ez <= bz, (i, k, b - a, ez, bz)
            worst = max(worst, (e / tol_for(k), i))
        i0 = i1
    print("all %d signals checked; worst error / order bound %.3f (signal %d)"
          % (B, worst[0], worst[1]))
    g.close()


def test_serving_full_trace(env):
    """1024 streams of orders 2..16, 20000 chunks of 4096..65536 samples,
    replayed by the native driver at a high offered rate with the
    benchmark's server (tile (256, 16), PH): every stream's output over its
    concatenated chunks, and every stream's exported final state."""
    torch, P = env
    S, R = 1024, 20000
    Ks, secs, ids, lens, offs, arrival = workloads.serving_trace(S=S, R=R,
                                                                 rate_chunks_per_s=2e6, seed=4)
    total = int(offs[-1] + lens[-1])
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(4)
    xd = torch.randn(total, generator=gen, device=dev, dtype=torch.float32)
    yd = torch.full_like(xd, float("nan"))
    srv = P.Server(handle=P.Handle(0, tile=(256, 16), algorithm="ph"), max_slots=1024,
                   budget=1 << 30)
    sid = np.array([srv.open(secs[s]) for s in range(S)], dtype=np.int64)
    lat, wall = srv.replay(sid[ids], offs, lens, arrival, xd, yd)
    states = [srv.state(int(sid[s])) for s in range(S)]
    srv.close()
    print("served %d chunks (%.3e samples) in %.3f s; p50 %.1f us p99 %.1f us"
          % (R, total, wall, 1e6 * np.percentile(lat, 50), 1e6 * np.percentile(lat, 99)))
    x = xd.cpu().numpy()
    y = yd.cpu().numpy()
    order = np.argsort(ids, kind="stable")           # each stream's chunks in arrival order
    bounds = np.searchsorted(ids[order], np.arange(S + 1))
    worst = (0.0, -1)
    for s in range(S):
        idx = order[bounds[s]:bounds[s + 1]]
        if len(idx) == 0:
            continue
        xs = np.concatenate([x[offs[r]:offs[r] + lens[r]] for r in idx])
        ys = np.concatenate([y[offs[r]:offs[r] + lens[r]] for r in idx])
        yr, zfr = oracle.sosfilt(secs[s], xs)
        k = int(Ks[s])
        e, ez = rel_l2(ys, yr), rel_l2(states[s], zfr)
        by = bz = tol_for(k)
        if e > by or ez > bz:
            by, bz = fp32_bounds(k, secs[s], xs, None, yr, zfr)
            bz = zf_bound(k, by, bz, yr, zfr)
        assert e <= by, (s, k, len(xs), e, by)
        assert ez <= bz, (s, k, ez, bz)
        worst = max(worst, (e / tol_for(k), s))
    print("all %d streams checked; worst error / order bound %.3f (stream %d)"
          % (S, worst[0], worst[1]))


def _loss(sos, x, zi, gy, gzf):
    y, zf = oracle.sosfilt(sos, x, zi)
    return float(np.dot(gy, y) + np.sum(gzf * zf))


def _fd_check(sos, x, zi, gy, gzf, gx, gzi, gs, xi_idx):
    """FP64 central differences of the oracle's loss <gy, y> + <gzf, zf> for
    every coefficient, every initial state and the samples xi_idx; returns the
    relative L2 errors of the given gradients over those components.
    The loss is linear in x, zi and each section's b0, b1, b2, so their central
    differences are exact for any step; a step of 1e-3 max(1, |p|) keeps the
    rounding of the loss negligible. It is not linear in a0, a1, a2: their
    step is 1e-8 max(1, |p|), whose truncation error (falling with the step
    squared) is below 1e-8 even for lightly damped sections, whose response
    moves fast with the poles."""
    sos = np.asarray(sos, np.float64)
    x = np.asarray(x, np.float64)
    zi = np.asarray(zi, np.float64)

    def central(f, v, h):
        return (f(v + h) - f(v - h)) / (2 * h)

    fd_s = np.zeros_like(sos)
    for k in range(sos.shape[0]):
        for j in range(6):
            h = (1e-3 if j < 3 else 1e-8) * max(1.0, abs(sos[k, j]))

            def f(v, k=k, j=j):
                p = sos.copy()
                p[k, j] = v
                return _loss(p, x, zi, gy, gzf)

            fd_s[k, j] = central(f, sos[k, j], h)
    fd_z = np.zeros_like(zi)
    for k in range(zi.shape[0]):
        for j in range(2):
            def f(v, k=k, j=j):
                p = zi.copy()
                p[k, j] = v
                return _loss(sos, x, p, gy, gzf)

            fd_z[k, j] = central(f, zi[k, j], 1e-3 * max(1.0, abs(zi[k, j])))
    fd_x = np.zeros(len(xi_idx))
    for t, i in enumerate(xi_idx):
        def f(v, i=i):
            p = x.copy()
            p[i] = v
            return _loss(sos, p, zi, gy, gzf)

        fd_x[t] = central(f, x[i], 1e-3 * max(1.0, abs(x[i])))
    return (rel_l2(gs, fd_s), rel_l2(gzi, fd_z), rel_l2(np.asarray(gx)[xi_idx], fd_x))


@pytest.mark.parametrize("case", ["butter8", "damped16"])
@pytest.mark.parametrize("alg", [None, "ph"])
def test_differentiation_batch(env, case, alg):
    """256 signals x 2^16 samples through the batched training forward and the
    batched adjoint (one launch each, as the benchmark times them), with the
    default handle and with the benchmark's PH handle. Every signal's
    gradients against the oracle's reverse sweep; 4 signals also against FP64
    central finite differences (all coefficients, all zi, 64 samples)."""
    torch, P = env
    B, m = 256, 1 << 16
    if case == "butter8":
        sos = workloads.sweep_sections(4, "butter")
    else:
        from tests.test_gpu_forward import lightly_damped_sections

        sos = lightly_damped_sections()
    K = sos.shape[0]
    g = workloads.rng(500 + K)
    x = workloads.batch_signal(B * m, seed=5)
    gy = workloads.batch_signal(B * m, seed=6)
    zi = workloads.initial_state(B * K, g)
    gzf = workloads.initial_state(B * K, g, var=1.0)
    if case == "damped16":
        # at rest and with no final-state cotangent, as in the single-signal
        # stress cases: section 0 carries the whole cascade's unit-energy
        # scaling, a gain of about 1e8 that the later sections take back, so
        # the inner sections' states, and a loss term <gzf, zf>, reach about
        # 1e16, beyond which no FP64 finite difference of <gy, y> resolves
        # anything
        zi = np.zeros_like(zi)
        gzf = np.zeros_like(gzf)
    rows = np.tile(sos, (B, 1))
    sig_off = np.arange(B + 1, dtype=np.int64) * m
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, algorithm=alg)
    Kd = dev(np.full(B, K, np.int32))
    sd = dev(sig_off)
    y, zf, saved = P.sosfilt_train_batched(dev(x), dev(rows), Kd, sd, zi=dev(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp_batched(dev(rows), Kd, sd, dev(x), y, saved, dev(gy), dev(gzf),
                                        handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    gx, gzi, gs = gx.cpu().numpy(), gzi.cpu().numpy(), gs.cpu().numpy()
    tol = 1e-5 if K <= 4 else 1e-4
    worst = np.zeros(3)
    for i in range(B):
        a, b = i * m, (i + 1) * m
        zs = slice(i * K, (i + 1) * K)
        rx, rzi, rs = oracle.sosfilt_vjp(sos, x[a:b], zi[zs], gy[a:b], gzf[zs])
        e = np.array([rel_l2(gx[a:b], rx), rel_l2(gzi[zs], rzi), rel_l2(gs[zs], rs)])
        worst = np.maximum(worst, e)
        # gzi holds 2K values at the signal's first samples, which can be small
        # against the cotangent's scale: it is held to the order's bound or
        # FLOOR_FACTOR x the error of a sequential FP32 reversed-time pass.
        # Coefficient gradients are sums over 2^16 samples that cancel: 1e-4,
        # or FLOOR_FACTOR x the error of a sequential FP32 pass where that
        # alone exceeds 1e-4 (some inputs to the lightly damped cascade: FP32
        # section outputs by themselves put such sums above 1e-4)
        bzi, bs = tol, 1e-4
        if e[1] > tol:
            floor = fp32_gzi_floor(sos, gy[a:b], gzf[zs], rzi)
            bzi = max(tol, FLOOR_FACTOR * floor)
            print("  signal %d: gzi %.2e, sequential FP32 %.2e" % (i, e[1], floor))
        if e[2] > bs:
            assert not np.any(gzf[zs]), "the FP32 yardstick for gsections takes no gzf"
            floor = fp32_gs_floor(sos, x[a:b], zi[zs], gy[a:b], rs)
            bs = max(bs, FLOOR_FACTOR * floor)
            print("  signal %d: gsections %.2e, sequential FP32 %.2e" % (i, e[2], floor))
        assert e[0] <= tol and e[1] <= bzi and e[2] <= bs, (i, e, bzi, bs)
    print(case, alg, "worst over %d signals: gx %.2e gzi %.2e gsections %.2e" % (B, *worst))
    pick = [0, 1, 128, 255]
    rng = np.random.default_rng(7)
    for i in pick:
        a, b = i * m, (i + 1) * m
        zs = slice(i * K, (i + 1) * K)
        xi_idx = np.sort(rng.choice(m, 64, replace=False))
        es = _fd_check(sos, x[a:b], zi[zs], gy[a:b], gzf[zs], gx[a:b], gzi[zs], gs[zs], xi_idx)
        print("  signal", i, "vs finite differences: gsections %.2e gzi %.2e gx %.2e" % es)
        bs = 1e-4
        if es[0] > bs and not np.any(gzf[zs]):
            _, _, rs = oracle.sosfilt_vjp(sos, x[a:b], zi[zs], gy[a:b], gzf[zs])
            bs = max(bs, FLOOR_FACTOR * fp32_gs_floor(sos, x[a:b], zi[zs], gy[a:b], rs))
        assert es[0] <= bs and es[1] <= tol and es[2] <= tol, (i, es, bs)
