"""GPU parity of the PH section solver (sos_set_algorithm(h, SOS_ALG_PH)):
the particular solution of every lane followed by the homogeneous correction
(Sec. II-C, Eqs. (9) and (11)), in place of divide-and-conquer cyclic
reduction. Same oracle, inputs and bounds as the DC-CR tests: relative L2
error <= 1e-5 for orders <= 8 and <= 1e-4 at order 16, zf to the same bounds;
every tile, both compute types, the batched, captured, served and training
paths that take the handle's solver."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, max_over_peak, rel_l2, tol_for, zf_bound

pytestmark = pytest.mark.gpu

TILES = ((64, 16), (64, 64), (256, 32), (512, 16), (512, 32), (512, 64), (1024, 16), (1024, 32))


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def ph_handle(P, tile=None, precision=0):
    h = P.Handle(0, tile=tile, precision=precision, algorithm="ph")
    assert h.algorithm() == "ph"
    return h


def run(torch, P, sos, x, zi=None, handle=None):
    y, zf = P.sosfilt(dev(torch, x), dev(torch, np.asarray(sos, np.float32)),
                      None if zi is None else dev(torch, np.asarray(zi, np.float32)),
                      handle=handle)
    torch.cuda.synchronize()
    assert handle.last_error() == P.SOS_OK
    return y.cpu().numpy(), zf.cpu().numpy()


def test_algorithm_selection(env, monkeypatch):
    torch, P = env
    monkeypatch.delenv("SOS_ALG", raising=False)
    h = P.Handle(0)
    assert h.algorithm() == "auto"
    h.set_algorithm("ph")
    assert h.algorithm() == "ph"
    h.set_algorithm("dccr")
    assert h.algorithm() == "dccr"
    h.set_algorithm(None)
    assert h.algorithm() == "auto"
    monkeypatch.setenv("SOS_ALG", "ph")
    assert h.algorithm() == "ph"            # the default follows the environment
    monkeypatch.setenv("SOS_ALG", "dccr")
    assert h.algorithm() == "dccr"
    monkeypatch.setenv("SOS_ALG", "toeplitz")
    assert h.algorithm() == "toeplitz"
    h.set_algorithm("auto")
    assert h.algorithm() == "auto"          # an explicit choice wins
    h.set_algorithm("toeplitz")
    assert h.algorithm() == "toeplitz"
    assert P.lib().sos_set_algorithm(h.ptr, 5) == P.SOS_EINVAL
    assert P.lib().sos_set_algorithm(h.ptr, -1) == P.SOS_EINVAL
    assert P.lib().sos_set_algorithm(None, P.SOS_ALG_PH) == P.SOS_EINVAL
    assert P.lib().sos_get_algorithm(None) == P.SOS_EINVAL
    with pytest.raises(ValueError):
        h.set_algorithm("fft")


@pytest.mark.parametrize("kind", ["butter", "random"])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
def test_sweep_sections(env, K, kind):
    torch, P = env
    sos = workloads.sweep_sections(K, kind)
    n = (1 << 18) + 12345
    x = workloads.signal(n, seed=2)
    zi = workloads.initial_state(K, workloads.rng(40 + K))
    yr, zfr = oracle.sosfilt(sos, x, zi)
    for tile in TILES:
        y, zf = run(torch, P, sos, x, zi, ph_handle(P, tile))
        e = rel_l2(y, yr)
        print(kind, "K", K, "tile", tile, "rel_l2", e, "zf", rel_l2(zf, zfr))
        assert e <= tol_for(K), (kind, K, tile, e)
        assert rel_l2(zf, zfr) <= tol_for(K), (kind, K, tile)


@pytest.mark.parametrize("tile", TILES)
def test_edge_lengths(env, tile):
    torch, P = env
    L, N = tile
    C = L * N
    CW = 64 * N
    g = workloads.rng(78)
    h = ph_handle(P, tile)
    for K in (1, 3):
        sos = workloads.random_stable_sos(K, g)
        zi = workloads.initial_state(K, g)
        for n in (1, 2, 3, 5, N - 1, N, N + 1, CW - 1, CW + 1, C - 1, C, C + 1, 2 * C,
                  3 * C + 17):
            x = workloads.signal(n, seed=n + 1)
            y, zf = run(torch, P, sos, x, zi, h)
            yr, zfr = oracle.sosfilt(sos, x, zi)
            assert rel_l2(y, yr) <= 1e-5, (K, n, tile)
            assert rel_l2(zf, zfr) <= 1e-5, (K, n, tile, zf, zfr)


@pytest.mark.parametrize("tile", [(64, 16), (512, 32), (512, 64)])
def test_small_grid_and_in_place(env, tile, monkeypatch):
    """One or three workgroups for the whole signal (each draws many tickets,
    prefetching the next group while correcting the current one), then the
    same filter in place."""
    torch, P = env
    L, N = tile
    C = L * N
    g = workloads.rng(89)
    h = ph_handle(P, tile)
    for grid in (1, 3):
        monkeypatch.setenv("SOS_GRID", str(grid))
        for K in (1, 4):
            sos = workloads.random_stable_sos(K, g)
            zi = workloads.initial_state(K, g)
            x = workloads.signal(5 * C + 77, seed=grid * 10 + K)
            y, zf = run(torch, P, sos, x, zi, h)
            yr, zfr = oracle.sosfilt(sos, x, zi)
            assert rel_l2(y, yr) <= 1e-5, (grid, K, tile)
            assert rel_l2(zf, zfr) <= 1e-5, (grid, K, tile)
    monkeypatch.delenv("SOS_GRID")
    xd = dev(torch, x)
    P.sosfilt_(xd, dev(torch, sos.astype(np.float32)), zi=dev(torch, zi), y=xd, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    assert rel_l2(xd.cpu().numpy(), yr) <= 1e-5


@pytest.mark.parametrize("tile", [(64, 16), (512, 64), (1024, 32)])
@pytest.mark.parametrize("K", [1, 4, 8])
def test_precision64(env, K, tile):
    torch, P = env
    sos = workloads.sweep_sections(K, "random")
    n = (1 << 17) + 999
    x = workloads.signal(n, seed=12)
    zi = workloads.initial_state(K, workloads.rng(50 + K))
    y, zf = run(torch, P, sos, x, zi, ph_handle(P, tile, precision=64))
    yr, zfr = oracle.sosfilt(sos, x, zi)
    print("ph fp64 K", K, "tile", tile, rel_l2(y, yr), rel_l2(zf, zfr))
    assert rel_l2(y, yr) <= 1e-6
    assert rel_l2(zf, zfr) <= 1e-6


def lightly_damped_sections(K=8, r=0.995, seed=9):
    """K sections with every pole at radius r, scaled to unit white-noise gain
    (the squared impulse response, from the oracle, sums to 1)."""
    sos = workloads.random_stable_sos(K, workloads.rng(seed), r_fixed=r)
    imp = np.zeros(40000)
    imp[0] = 1.0
    hr, _ = oracle.sosfilt(sos, imp)
    sos[0, :3] /= np.sqrt(np.sum(hr ** 2))
    return sos.astype(np.float32)


@pytest.mark.parametrize("tile", [(64, 16), (512, 64)])
def test_lightly_damped_order16(env, tile):
    """Order 16, poles at radius 0.995: FP64 meets the order-16 bound, and so
    does FP32 PH (FP64 state path, orthonormal correction basis). FP32 DC-CR
    forced on every section is reported beside the sequential FP32 floor: its
    fold amplifies rounding near the mirror frequencies of these poles, which
    is why the default solver takes PH for them."""
    import scipy.signal

    torch, P = env
    sos = lightly_damped_sections()
    n = 1 << 18
    x = workloads.signal(n, seed=13)
    yr, zfr = oracle.sosfilt(sos, x)
    y64, zf64 = run(torch, P, sos, x, None, ph_handle(P, tile, precision=64))
    y32, _ = run(torch, P, sos, x, None, ph_handle(P, tile, precision=32))
    yd, _ = run(torch, P, sos, x, None, P.Handle(0, tile=tile, precision=32, algorithm="dccr"))
    floor = rel_l2(scipy.signal.sosfilt(sos, x.astype(np.float32)), yr)
    print("order16 r=0.995 tile", tile, "ph fp64", rel_l2(y64, yr), "ph fp32", rel_l2(y32, yr),
          "dccr fp32", rel_l2(yd, yr), "fp32 sequential floor", floor)
    assert rel_l2(y64, yr) <= 1e-5
    assert rel_l2(zf64, zfr) <= 1e-5
    assert rel_l2(y32, yr) <= 1e-4
    assert np.isfinite(yd).all()


@pytest.mark.parametrize("K", [1, 8])
def test_full_size_2p28(env, K):
    """2^28 samples in the launch configuration the benchmark times."""
    torch, P = env
    sos = workloads.sweep_sections(K, "butter")
    n = 1 << 28
    x = workloads.signal(n, seed=2)
    h = ph_handle(P)
    xd = dev(torch, x)
    y, zf = P.sosfilt(xd, dev(torch, sos), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    yh = y.cpu().numpy()
    del y, xd
    yr, zfr = oracle.sosfilt(sos, x)
    e = rel_l2(yh, yr)
    print("ph 2^28 K", K, "rel_l2", e, "max/peak", max_over_peak(yh, yr))
    assert e <= tol_for(K)
    assert rel_l2(zf.cpu().numpy(), zfr) <= tol_for(K)


@pytest.mark.parametrize("tile,precision", [((64, 16), 32), ((512, 32), 32), ((256, 64), 32),
                                            ((512, 32), 64)])
def test_uneven_batch(env, tile, precision):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=96, log2_lo=2, log2_hi=17, seed=13)
    x = workloads.batch_signal(int(sig_off[-1]), seed=14)
    h = ph_handle(P, tile, precision)
    y, zf = P.sosfilt_batched(dev(torch, x), dev(torch, rows), dev(torch, Ks.astype(np.int32)),
                              dev(torch, sig_off.astype(np.int64)), zi=dev(torch, zi), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    y, zf = y.cpu().numpy(), zf.cpu().numpy()
    yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi, nthreads=8)
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(len(Ks)):
        a, b = sig_off[i], sig_off[i + 1]
        by = bz = tol_for(int(Ks[i]))
        if precision != 64 and b > a:
            by, bz = fp32_bounds(int(Ks[i]), rows[so[i]:so[i + 1]], x[a:b], zi[so[i]:so[i + 1]],
                                 yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(y[a:b], yr[a:b]) <= by, (i, Ks[i], b - a)
        bz = zf_bound(int(Ks[i]), by, bz, yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(zf[so[i]:so[i + 1]], zfr[so[i]:so[i + 1]]) <= bz, (i, Ks[i], b - a)


def test_graph_replays(env):
    """A batch captured with the PH solver: replays with new data (and eager
    work between them) equal the eager PH call and the oracle's bounds."""
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=48, log2_lo=2, log2_hi=16, seed=65)
    total = int(sig_off[-1])
    xg, zig, rowsg = dev(torch, workloads.batch_signal(total, seed=66)), dev(torch, zi), \
        dev(torch, rows)
    Kg, sg = dev(torch, Ks.astype(np.int32)), dev(torch, sig_off.astype(np.int64))
    gr = P.BatchGraph(xg, rowsg, Kg, sg, zi=zig, handle=ph_handle(P, (256, 32)))
    he = ph_handle(P, (256, 32))
    for rep in range(3):
        x = workloads.batch_signal(total, seed=67 + rep)
        zi_r = workloads.initial_state(int(Ks.sum()), workloads.rng(80 + rep))
        xg.copy_(dev(torch, x))
        zig.copy_(dev(torch, zi_r))
        gr.launch()
        torch.cuda.synchronize()
        assert gr.last_error() == P.SOS_OK
        y_graph = gr.y.cpu().numpy()
        ye, _ = P.sosfilt_batched(dev(torch, x), rowsg, Kg, sg, zi=dev(torch, zi_r), handle=he)
        torch.cuda.synchronize()
        ye = ye.cpu().numpy()
        scale = max(np.abs(ye).max(), 1.0)
        assert np.abs(y_graph - ye).max() <= 1e-5 * scale, rep
        yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi_r, nthreads=8)
        so = np.r_[0, np.cumsum(Ks)]
        for i in range(len(Ks)):
            a, b = sig_off[i], sig_off[i + 1]
            if b > a:
                by, _ = fp32_bounds(int(Ks[i]), rows[so[i]:so[i + 1]], x[a:b],
                                    zi_r[so[i]:so[i + 1]], yr[a:b], zfr[so[i]:so[i + 1]])
                assert rel_l2(y_graph[a:b], yr[a:b]) <= by, (rep, i)
    gr.close()


def test_server_streams(env):
    """Chunks of many streams served with the PH solver equal the oracle run
    over each stream's concatenated chunks."""
    torch, P = env
    Ks, secs, ids, lens, offs, _ = workloads.serving_trace(S=16, R=80, rate_chunks_per_s=1e6,
                                                          lo=64, hi=20000, seed=43)
    offs = np.zeros(len(lens), dtype=np.int64)
    np.cumsum(lens[:-1], out=offs[1:])
    x = workloads.signal(int(lens.sum()), seed=44)
    xd = dev(torch, x)
    srv = P.Server(handle=ph_handle(P, (256, 16)), max_slots=64)
    sid = [srv.open(secs[s]) for s in range(len(Ks))]
    yd = torch.full_like(xd, float("nan"))
    tickets = []
    for r in range(len(ids)):
        o, n = int(offs[r]), int(lens[r])
        tickets.append(srv.push(sid[ids[r]], xd[o:o + n], yd[o:o + n])[0])
    for t in tickets:
        srv.wait(t)
    states = {s: srv.state(sid[s]) for s in range(len(Ks))}
    srv.close()
    y = yd.cpu().numpy()
    for s in range(len(Ks)):
        idx = np.nonzero(ids == s)[0]
        if len(idx) == 0:
            continue
        xs = np.concatenate([x[offs[r]:offs[r] + lens[r]] for r in idx])
        ys = np.concatenate([y[offs[r]:offs[r] + lens[r]] for r in idx])
        yr, zfr = oracle.sosfilt(secs[s], xs)
        by, bz = fp32_bounds(int(Ks[s]), secs[s], xs, None, yr, zfr)
        assert rel_l2(ys, yr) <= by, (s, Ks[s])
        assert rel_l2(states[s], zfr) <= zf_bound(int(Ks[s]), by, bz, yr, zfr), s


@pytest.mark.parametrize("tile", [(64, 16), (256, 32), (512, 16)])
@pytest.mark.parametrize("K,n", [(1, 5000), (4, 70001), (8, 1 << 16), (3, 1)])
def test_vjp_with_ph(env, K, n, tile):
    """Both passes with the PH solver (the training forward, then the
    reversed-time recursion of the adjoint) against the oracle's VJP."""
    torch, P = env
    g = workloads.rng(300 + K + n % 97)
    sos = workloads.random_stable_sos(K, g)
    sos[0] *= 1.25                                       # a0 != 1
    x = workloads.signal(n, seed=17)
    zi = workloads.initial_state(K, g)
    gy = workloads.signal(n, seed=18)
    gzf = workloads.initial_state(K, g, var=1.0)
    h = ph_handle(P, tile)
    d = lambda a: dev(torch, np.asarray(a, np.float32))
    y, zf, saved = P.sosfilt_train(d(x), d(sos), d(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp(d(sos), d(x), y, saved, d(gy), d(gzf), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
    print("ph vjp K", K, "n", n, "tile", tile, rel_l2(gx.cpu().numpy(), rx),
          rel_l2(gzi.cpu().numpy(), rzi), rel_l2(gs.cpu().numpy(), rs))
    assert rel_l2(gx.cpu().numpy(), rx) <= tol_for(K)
    assert rel_l2(gzi.cpu().numpy(), rzi) <= tol_for(K)
    assert rel_l2(gs.cpu().numpy(), rs) <= 1e-4


def test_batched_vjp_with_ph(env):
    """Uneven batch (empty and one-sample signals included), training forward
    and VJP in one launch each with the PH solver, against the oracle."""
    torch, P = env
    g = workloads.rng(310)
    B = 24
    Ks = g.integers(1, 5, size=B).astype(np.int32)
    Ks[3] = 2
    lens = np.floor(2.0 ** g.uniform(0, 15, size=B)).astype(np.int64)
    lens[5], lens[9] = 0, 1
    sig_off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    rows = np.concatenate([workloads.random_stable_sos(int(k), g) for k in Ks]).astype(np.float32)
    zi = workloads.initial_state(int(Ks.sum()), g)
    x = workloads.batch_signal(int(sig_off[-1]), seed=311)
    gy = workloads.batch_signal(int(sig_off[-1]), seed=312)
    gzf = workloads.initial_state(int(Ks.sum()), g, var=1.0)
    h = ph_handle(P, (256, 32))
    y, zf, saved = P.sosfilt_train_batched(dev(torch, x), dev(torch, rows), dev(torch, Ks),
                                           dev(torch, sig_off), zi=dev(torch, zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp_batched(dev(torch, rows), dev(torch, Ks), dev(torch, sig_off),
                                        dev(torch, x), y, saved, dev(torch, gy),
                                        gzf=dev(torch, gzf), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    gx, gzi, gs = gx.cpu().numpy(), gzi.cpu().numpy(), gs.cpu().numpy()
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(B):
        a, b = sig_off[i], sig_off[i + 1]
        r = slice(so[i], so[i + 1])
        rx, rzi, rs = oracle.sosfilt_vjp(rows[r], x[a:b], zi[r], gy[a:b], gzf[r])
        e = (rel_l2(gx[a:b], rx) if b > a else 0.0, rel_l2(gzi[r], rzi), rel_l2(gs[r], rs))
        print("signal", i, "K", Ks[i], "n", b - a, e)
        assert e[0] <= tol_for(int(Ks[i])), (i, e)
        assert e[1] <= 1e-4 and e[2] <= 1e-4, (i, e)


def test_training_forward_then_vjp(env):
    """The training forward (which also keeps every section's output) with the
    PH solver, then the adjoint: gradients equal the oracle's VJP."""
    torch, P = env
    K, n = 3, 70001
    g = workloads.rng(101)
    sos = workloads.random_stable_sos(K, g)
    x = workloads.signal(n, seed=7)
    zi = workloads.initial_state(K, g)
    gy = workloads.signal(n, seed=8)
    gzf = workloads.initial_state(K, g, var=1.0)
    h = ph_handle(P, (256, 32))
    d = lambda a: dev(torch, np.asarray(a, np.float32))
    y, zf, saved = P.sosfilt_train(d(x), d(sos), d(zi), handle=h)
    gx, gzi, gs = P.sosfilt_vjp(d(sos), d(x), y, saved, d(gy), d(gzf), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    yr, zfr = oracle.sosfilt(sos, x, zi)
    assert rel_l2(y.cpu().numpy(), yr) <= 1e-5
    assert rel_l2(zf.cpu().numpy(), zfr) <= 1e-5
    rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, gzf)
    assert rel_l2(gx.cpu().numpy(), rx) <= 1e-5
    assert rel_l2(gzi.cpu().numpy(), rzi) <= 1e-5
    assert rel_l2(gs.cpu().numpy(), rs) <= 1e-4
