"""GPU parity of the plain filter (sos_filter) against the FP64 oracle.

Every case draws seeded inputs from workloads.py, runs the HIP path through
the C ABI, and compares element by element with oracle.sosfilt on the same
float32 values promoted to float64. Bounds: relative L2 error <= 1e-5 for
orders <= 8 (K <= 4) and <= 1e-4 at order 16 (K = 8); zf to the same bounds.
"""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, max_over_peak, rel_l2, tol_for, zf_bound

pytestmark = pytest.mark.gpu

# (L lanes per group, N samples per lane): one-wave groups and 4/8/16-wave groups
TILES = ((64, 16), (64, 64), (256, 32), (512, 16), (512, 32), (512, 64), (1024, 16), (1024, 32))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def P():
    import paper_2607_23763_amd as P

    P.lib()
    return P


def run(torch, P, sos, x, zi=None, tile=None, handle=None, alg=None):
    h = handle or P.Handle(0, tile=tile, algorithm=alg)
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(sos, dtype=np.float32)).cuda()
    zd = None if zi is None else torch.from_numpy(np.ascontiguousarray(zi, np.float32)).cuda()
    y, zf = P.sosfilt(xd, sd, zd, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    return y.cpu().numpy(), zf.cpu().numpy(), h


@pytest.mark.parametrize("tile", TILES)
def test_single_biquad_2p20(torch_cuda, P, tile):
    """2nd-order Butterworth at 0.2*Nyquist, 2^20 N(0,1) samples, zi = 0."""
    sos, x = workloads.single_biquad(1 << 20, seed=1)
    y, zf, _ = run(torch_cuda, P, sos, x, tile=tile)
    yr, zfr = oracle.sosfilt(sos, x)
    print("tile", tile, "rel_l2", rel_l2(y, yr), "max/peak", max_over_peak(y, yr))
    assert rel_l2(y, yr) <= 1e-5
    assert max_over_peak(y, yr) < 1e-4
    assert rel_l2(zf, zfr) <= 1e-5


@pytest.mark.parametrize("kind", ["butter", "random"])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
def test_sweep_sections(torch_cuda, P, K, kind):
    sos = workloads.sweep_sections(K, kind)
    n = (1 << 18) + 12345
    x = workloads.signal(n, seed=2)
    zi = workloads.initial_state(K, workloads.rng(40 + K))
    for tile in TILES:
        y, zf, _ = run(torch_cuda, P, sos, x, zi, tile=tile)
        yr, zfr = oracle.sosfilt(sos, x, zi)
        e = rel_l2(y, yr)
        print(kind, "K", K, "tile", tile, "rel_l2", e, "zf", rel_l2(zf, zfr))
        assert e <= tol_for(K), (kind, K, tile, e)
        assert rel_l2(zf, zfr) <= tol_for(K), (kind, K, tile)


@pytest.mark.parametrize("tile", TILES)
def test_edge_lengths(torch_cuda, P, tile):
    L, N = tile
    C = L * N
    CW = 64 * N
    g = workloads.rng(77)
    for K in (1, 3):
        sos = workloads.random_stable_sos(K, g)
        zi = workloads.initial_state(K, g)
        for n in (1, 2, 3, 5, N - 1, N, N + 1, CW - 1, CW + 1, C - 1, C, C + 1, 2 * C,
                  3 * C + 17):
            x = workloads.signal(n, seed=n)
            y, zf, _ = run(torch_cuda, P, sos, x, zi, tile=tile)
            yr, zfr = oracle.sosfilt(sos, x, zi)
            assert rel_l2(y, yr) <= 1e-5, (K, n, tile)
            assert rel_l2(zf, zfr) <= 1e-5, (K, n, tile, zf, zfr)


@pytest.mark.parametrize("tile", TILES)
def test_small_grid_many_groups_per_workgroup(torch_cuda, P, tile, monkeypatch):
    """One, two or five workgroups for the whole signal: each draws many
    tickets and loads the next group while the current one is corrected and
    stored, up to the partial last group; also in place."""
    L, N = tile
    C = L * N
    g = workloads.rng(88)
    for grid in (1, 2, 5):
        monkeypatch.setenv("SOS_GRID", str(grid))
        for K in (1, 4):
            sos = workloads.random_stable_sos(K, g)
            zi = workloads.initial_state(K, g)
            n = 7 * C + 123
            x = workloads.signal(n, seed=grid * 10 + K)
            y, zf, _ = run(torch_cuda, P, sos, x, zi, tile=tile)
            yr, zfr = oracle.sosfilt(sos, x, zi)
            assert rel_l2(y, yr) <= 1e-5, (grid, K, tile)
            assert rel_l2(zf, zfr) <= 1e-5, (grid, K, tile)
    monkeypatch.setenv("SOS_GRID", "2")
    torch = torch_cuda
    xd = torch.from_numpy(x).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(sos, dtype=np.float32)).cuda()
    h = P.Handle(0, tile=tile)
    P.sosfilt_(xd, sd, zi=torch.from_numpy(zi).cuda(), y=xd, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    assert rel_l2(xd.cpu().numpy(), yr) <= 1e-5


def test_in_place_and_misaligned(torch_cuda, P):
    torch = torch_cuda
    K = 4
    sos = workloads.sweep_sections(K, "random")
    n = 200003
    x = workloads.signal(n, seed=9)
    yr, zfr = oracle.sosfilt(sos, x)
    sd = torch.from_numpy(sos).cuda()
    # in place
    xd = torch.from_numpy(x).cuda()
    zf = torch.empty((K, 2), device="cuda")
    P.sosfilt_(xd, sd, y=xd, zf=zf)
    torch.cuda.synchronize()
    assert rel_l2(xd.cpu().numpy(), yr) <= 1e-5
    # input and output at every 4-byte offset from a 16-byte boundary (128-bit
    # accesses at dword alignment), the two offsets differing
    for oi, oo in ((1, 1), (2, 3), (3, 2), (0, 1), (1, 0)):
        buf = torch.zeros(n + 4, device="cuda")
        buf[oi:oi + n] = torch.from_numpy(x).cuda()
        out = torch.zeros(n + 4, device="cuda")
        P.sosfilt_(buf[oi:oi + n], sd, y=out[oo:oo + n], zf=zf)
        torch.cuda.synchronize()
        assert rel_l2(out[oo:oo + n].cpu().numpy(), yr) <= 1e-5, (oi, oo)
        o = out.cpu().numpy()
        assert not o[:oo].any() and not o[oo + n:].any(), (oi, oo)   # nothing written outside
        assert rel_l2(zf.cpu().numpy(), zfr) <= 1e-5


@pytest.mark.parametrize("alg", ["dccr", "ph"])
def test_degenerate_k0_n0(torch_cuda, P, alg):
    torch = torch_cuda
    h = P.Handle(0, algorithm=alg)
    x = torch.from_numpy(workloads.signal(1000, 3)).cuda()
    y, zf = P.sosfilt(x, torch.zeros((0, 6), device="cuda"), handle=h)
    torch.cuda.synchronize()
    assert torch.equal(y, x) and zf.numel() == 0
    sos = torch.from_numpy(workloads.butterworth_sos(2)).cuda()
    zi = torch.from_numpy(workloads.initial_state(2, workloads.rng(1))).cuda()
    y, zf = P.sosfilt(torch.zeros(0, device="cuda"), sos, zi, handle=h)
    torch.cuda.synchronize()
    assert y.numel() == 0 and torch.equal(zf, zi)
    y, zf = P.sosfilt(torch.zeros(0, device="cuda"), sos, None, handle=h)
    torch.cuda.synchronize()
    assert torch.count_nonzero(zf).item() == 0


@pytest.mark.parametrize("alg", ["dccr", "ph"])
def test_lookback_carries_are_oracle_states(torch_cuda, P, alg):
    """The resolved carry each group publishes equals the oracle's state after
    the group's last sample."""
    K = 3
    sos = workloads.sweep_sections(K, "random")
    zi = workloads.initial_state(K, workloads.rng(5))
    tile = (256, 16)
    C = tile[0] * tile[1]
    G = 37
    x = workloads.signal(G * C, seed=4)
    _, _, h = run(torch_cuda, P, sos, x, zi, tile=tile, alg=alg)
    car = h.carries()
    assert car.shape == (G, K, 2)
    for g in range(G):
        _, st = oracle.sosfilt(sos, x[:(g + 1) * C], zi)
        scale = max(1.0, np.max(np.abs(st)))
        assert np.max(np.abs(car[g] - st)) <= 2e-5 * scale, (g, car[g], st)


@pytest.mark.parametrize("alg", ["dccr", "ph"])
def test_bad_sections_report_and_poison(torch_cuda, P, alg):
    torch = torch_cuda
    h = P.Handle(0, algorithm=alg)
    x = torch.from_numpy(workloads.signal(5000, 2)).cuda()
    sos = workloads.butterworth_sos(2).copy()
    sos[1, 3] = 0.0                                   # a0 == 0
    y, zf = P.sosfilt(x, torch.from_numpy(sos).cuda(), handle=h)
    assert h.last_error() == P.SOS_EA0
    assert torch.isnan(y).all().item() and torch.isnan(zf).all().item()
    sos = workloads.butterworth_sos(1).copy()
    sos[0, 5] = 1.5                                   # |a2| > 1
    y, zf = P.sosfilt(x, torch.from_numpy(sos).cuda(), handle=h)
    assert h.last_error() == P.SOS_EUNSTABLE
    assert torch.isnan(y).all().item()
    # the handle keeps working afterwards
    sos = workloads.butterworth_sos(1)
    y, zf = P.sosfilt(x, torch.from_numpy(sos).cuda(), handle=h)
    assert h.last_error() == P.SOS_OK
    yr, _ = oracle.sosfilt(sos, x.cpu().numpy())
    assert rel_l2(y.cpu().numpy(), yr) <= 1e-5


def lightly_damped_sections(K=8, r=0.995, seed=9):
    """K sections with every pole at radius r (random angles and zeros), the
    first section scaled so the cascade has unit white-noise gain (sum of the
    squared impulse response, computed by the oracle, equals 1)."""
    sos = workloads.random_stable_sos(K, workloads.rng(seed), r_fixed=r)
    imp = np.zeros(40000)
    imp[0] = 1.0
    h, _ = oracle.sosfilt(sos, imp)
    sos[0, :3] /= np.sqrt(np.sum(h ** 2))
    return sos.astype(np.float32)


def fp32_sequential_error(sos, x, zi, yr):
    """Relative L2 error of a sequential FP32 cascade (scipy's direct-form
    sosfilt run in float32): the accuracy floor of any FP32 filter."""
    import scipy.signal

    y32 = scipy.signal.sosfilt(sos.astype(np.float32), x.astype(np.float32),
                               zi=None if zi is None else zi.astype(np.float32))
    y32 = y32[0] if zi is not None else y32
    return rel_l2(y32, yr)


@pytest.mark.parametrize("tile", [(64, 16), (512, 16), (512, 64), (1024, 32)])
@pytest.mark.parametrize("K", [1, 4, 8])
def test_precision64_matches_oracle(torch_cuda, P, K, tile):
    """FP64 compute type: same layout and launch, errors from FP32 data only."""
    sos = workloads.sweep_sections(K, "random")
    n = (1 << 17) + 999
    x = workloads.signal(n, seed=12)
    zi = workloads.initial_state(K, workloads.rng(50 + K))
    h = P.Handle(0, tile=tile, precision=64)
    assert h.precision() == 64
    y, zf, _ = run(torch_cuda, P, sos, x, zi, handle=h)
    yr, zfr = oracle.sosfilt(sos, x, zi)
    print("fp64 K", K, "tile", tile, "rel_l2", rel_l2(y, yr), "zf", rel_l2(zf, zfr))
    assert rel_l2(y, yr) <= 1e-6
    assert rel_l2(zf, zfr) <= 1e-6


@pytest.mark.parametrize("tile", [None, (64, 16), (512, 32), (512, 64), (1024, 32)])
def test_lightly_damped_order16(torch_cuda, P, tile):
    """Order 16, all poles at radius 0.995 (the differentiation workload's
    stress case): the default handle (FP32 samples, FP64 state path, the
    automatic solver choice) meets the order-16 bound for y and zf, and the
    FP64 compute type meets 1e-5."""
    sos = lightly_damped_sections()
    n = 1 << 18
    x = workloads.signal(n, seed=13)
    yr, zfr = oracle.sosfilt(sos, x)
    h64 = P.Handle(0, tile=tile, precision=64)
    y64, zf64, _ = run(torch_cuda, P, sos, x, handle=h64)
    h32 = P.Handle(0, tile=tile)
    assert h32.precision() == 32 and h32.algorithm() == "auto"
    y32, zf32, _ = run(torch_cuda, P, sos, x, handle=h32)
    floor = fp32_sequential_error(sos, x, None, yr)
    print("order16 r=0.995 tile", tile, "fp64", rel_l2(y64, yr), "fp32", rel_l2(y32, yr),
          "zf", rel_l2(zf32, zfr), "max/peak", max_over_peak(y32, yr),
          "fp32 sequential floor", floor)
    assert rel_l2(y64, yr) <= 1e-5
    assert rel_l2(zf64, zfr) <= 1e-5
    assert rel_l2(y32, yr) <= 1e-4
    assert rel_l2(zf32, zfr) <= 1e-4
    assert max_over_peak(y32, yr) <= 1e-4


def test_auto_solver_picks_per_section(torch_cuda, P):
    """The automatic choice: Butterworth order 16 (every section's peak gain
    below the bound) runs DC-CR on every section, so it equals a DC-CR handle;
    the lightly damped cascade (every section above) equals a PH handle. The
    lookback's composition order varies between runs, hence the 1e-6."""
    n = (1 << 18) + 321
    x = workloads.signal(n, seed=14)
    for sos, other in ((workloads.sweep_sections(8, "butter"), "dccr"),
                       (lightly_damped_sections(), "ph")):
        ya, _, _ = run(torch_cuda, P, sos, x, handle=P.Handle(0, tile=(512, 64)))
        yo, _, _ = run(torch_cuda, P, sos, x, handle=P.Handle(0, tile=(512, 64), algorithm=other))
        print("auto vs", other, rel_l2(ya, yo))
        assert rel_l2(ya, yo) <= 1e-6


@pytest.mark.parametrize("alg", ["dccr", "ph"])
def test_lookback_timeout_is_bounded_and_reported(torch_cuda, P, alg):
    """A one-tick bound on each lookback wait, forced from the host: the launch
    still ends, any group whose wait ran out is NaN and the handle reports
    SOS_ETIMEOUT; with the default bound restored the same handle is exact."""
    torch = torch_cuda
    K = 4
    sos = workloads.sweep_sections(K, "random")
    n = 1 << 22
    x = workloads.signal(n, seed=31)
    h = P.Handle(0, tile=(256, 16), algorithm=alg)
    print("device wall clock kHz", h.wall_clock_khz())
    xd = torch.from_numpy(x).cuda()
    sd = torch.from_numpy(sos).cuda()
    h.set_timeout(1e-6)
    y, _ = P.sosfilt(xd, sd, handle=h)
    torch.cuda.synchronize()
    err = h.last_error()
    has_nan = bool(torch.isnan(y).any().item())
    print("one-tick bound: status", err, "NaN outputs", has_nan)
    assert err in (P.SOS_OK, P.SOS_ETIMEOUT)
    assert has_nan == (err == P.SOS_ETIMEOUT)
    h.set_timeout(0)
    y, _ = P.sosfilt(xd, sd, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    yr, _ = oracle.sosfilt(sos, x)
    assert rel_l2(y.cpu().numpy(), yr) <= 1e-5


@pytest.mark.parametrize("alg", ["dccr", "ph"])
@pytest.mark.parametrize("K", [12, 32, 64])
def test_long_cascades(torch_cuda, P, K, alg):
    """Cascades beyond order 16, up to the 64 sections the ABI allows: random
    stable sections of unit gain at their pole angle and random zi. FP32 is
    held to the order's bound or 16x the sequential FP32 error, FP64 compute
    to 1e-5; also as one signal of an uneven batch beside short ones."""
    torch = torch_cuda
    g = workloads.rng(600 + K)
    sos = workloads.random_stable_sos(K, g, r_lo=0.5, r_hi=0.95)
    zi = workloads.initial_state(K, g)
    n = (1 << 17) + 4321
    x = workloads.signal(n, seed=K)
    yr, zfr = oracle.sosfilt(sos, x, zi)
    y, zf, _ = run(torch, P, sos, x, zi, alg=alg)
    by, bz = fp32_bounds(K, sos, x, zi, yr, zfr)
    bz = zf_bound(K, by, bz, yr, zfr)
    print("K", K, alg, "fp32 rel_l2", rel_l2(y, yr), "bound", by, "zf", rel_l2(zf, zfr), bz)
    assert rel_l2(y, yr) <= by
    assert rel_l2(zf, zfr) <= bz
    y64, zf64, _ = run(torch, P, sos, x, zi, handle=P.Handle(0, precision=64, algorithm=alg))
    print("K", K, alg, "fp64 rel_l2", rel_l2(y64, yr), "zf", rel_l2(zf64, zfr))
    assert rel_l2(y64, yr) <= 1e-5 and rel_l2(zf64, zfr) <= 1e-5
    # the same cascade as one signal of a batch, between two short order-2 ones
    rows = np.concatenate([workloads.butterworth_sos(1), sos, workloads.butterworth_sos(1)])
    Ks = np.array([1, K, 1], dtype=np.int32)
    zib = np.concatenate([np.zeros((1, 2), np.float32), zi, np.zeros((1, 2), np.float32)])
    xb = np.concatenate([workloads.signal(999, seed=1), x, workloads.signal(5000, seed=5)])
    sig_off = np.array([0, 999, 999 + n, 999 + n + 5000], dtype=np.int64)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, algorithm=alg)
    yb, zfb = P.sosfilt_batched(d(xb), d(rows.astype(np.float32)), d(Ks), d(sig_off),
                                zi=d(zib), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    yb = yb.cpu().numpy()
    assert rel_l2(yb[999:999 + n], yr) <= by
    assert rel_l2(zfb.cpu().numpy()[1:1 + K], zfr) <= bz
    for (a, b), r in (((0, 999), rows[:1]), ((999 + n, 999 + n + 5000), rows[-1:])):
        ys, _ = oracle.sosfilt(r, xb[a:b])
        assert rel_l2(yb[a:b], ys) <= 1e-5


@pytest.mark.parametrize("alg", ["dccr", "ph"])
def test_length_chosen_tile(torch_cuda, P, alg):
    """With no tile set, sos_filter picks the group shape from the signal
    length; lengths on both sides of each switch (2^20 and 2^22 samples) stay
    within the bounds, and the tables it prepared serve sos_filter_prepared
    until a tile is set on the handle."""
    torch = torch_cuda
    K = 8
    sos = workloads.sweep_sections(K, "butter")
    zi = workloads.initial_state(K, workloads.rng(61))
    h = P.Handle(0, algorithm=alg)
    for n in (1000, (1 << 20) - 3, (1 << 20) + 1, (1 << 22) + 7):
        x = workloads.signal(n, seed=62)
        y, zf, _ = run(torch, P, sos, x, zi, handle=h)
        yr, zfr = oracle.sosfilt(sos, x, zi)
        print(alg, "n", n, "rel_l2", rel_l2(y, yr), "zf", rel_l2(zf, zfr))
        assert rel_l2(y, yr) <= tol_for(K), n
        assert rel_l2(zf, zfr) <= tol_for(K), n
    # tables sos_filter prepared for a short signal, reused at another length
    x = workloads.signal(5000, seed=63)
    run(torch, P, sos, x, zi, handle=h)
    x2 = workloads.signal((1 << 21) + 11, seed=64)
    xd = torch.from_numpy(x2).cuda()
    yd = torch.empty_like(xd)
    P.filter_prepared(xd, yd, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    yr, _ = oracle.sosfilt(sos, x2)
    assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K)
    # a tile set afterwards invalidates them
    h.set_tile(512, 64)
    with pytest.raises(P.SosError):
        P.filter_prepared(xd, yd, handle=h)


@pytest.mark.parametrize("precision", [32, 64])
def test_paths_interleaved_on_one_handle(torch_cuda, P, precision):
    """Every ticketed launch leaves the handle's ticket counter and descriptor
    epoch ready for the next one (the plain filter enqueues no arm step):
    plain, prepared, batched, training forward and adjoint calls alternate on
    one handle, with one-group-per-workgroup and multi-round grids, and each
    result still matches the oracle."""
    torch = torch_cuda
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, tile=(256, 16), precision=precision)
    K = 4
    sos = workloads.sweep_sections(K, "random")
    zi = workloads.initial_state(K, workloads.rng(71))
    Ks, rows, sig_off, bzi = workloads.uneven_batch(B=24, log2_lo=2, log2_hi=16, seed=72)
    bx = workloads.batch_signal(int(sig_off[-1]), seed=73)
    so = np.r_[0, np.cumsum(Ks)]
    tol = 1e-6 if precision == 64 else tol_for(K)
    for rep in range(2):
        for n in (3000, (1 << 20) + 5):          # one round of groups, then many
            x = workloads.signal(n, seed=74 + rep)
            y, zf, _ = run(torch, P, sos, x, zi, handle=h)
            yr, zfr = oracle.sosfilt(sos, x, zi)
            assert rel_l2(y, yr) <= tol and rel_l2(zf, zfr) <= tol, (rep, n)
            xd = dev(x)
            yd = torch.empty_like(xd)
            P.prepare(dev(np.asarray(sos, np.float32)), handle=h)
            for _ in range(2):
                P.filter_prepared(xd, yd, handle=h)
            torch.cuda.synchronize()
            yr0, _ = oracle.sosfilt(sos, x)
            assert rel_l2(yd.cpu().numpy(), yr0) <= tol, (rep, n, "prepared")
        yb, zfb = P.sosfilt_batched(dev(bx), dev(rows), dev(Ks.astype(np.int32)),
                                    dev(sig_off.astype(np.int64)), zi=dev(bzi), handle=h)
        torch.cuda.synchronize()
        yb = yb.cpu().numpy()
        for i in (0, 7, 23):
            a, b = sig_off[i], sig_off[i + 1]
            yr, _ = oracle.sosfilt(rows[so[i]:so[i + 1]], bx[a:b], bzi[so[i]:so[i + 1]])
            tb = 1e-6 if precision == 64 else tol_for(int(Ks[i]))
            assert rel_l2(yb[a:b], yr) <= tb, i
        x = workloads.signal(50000, seed=80 + rep)
        gy = workloads.signal(50000, seed=90 + rep)
        y, zf, saved = P.sosfilt_train(dev(x), dev(np.asarray(sos, np.float32)), dev(zi), handle=h)
        gx, gzi, gs = P.sosfilt_vjp(dev(np.asarray(sos, np.float32)), dev(x), y, saved, dev(gy),
                                    handle=h)
        torch.cuda.synchronize()
        rx, rzi, rs = oracle.sosfilt_vjp(sos, x, zi, gy, None)
        assert rel_l2(gx.cpu().numpy(), rx) <= 1e-3, rep
        assert rel_l2(gs.cpu().numpy(), rs) <= 1e-3, rep
    assert h.last_error() == P.SOS_OK


def test_plain_filter_captured_in_a_graph(torch_cuda, P):
    """A plain filter captured into a graph carries its own arm step, so its
    replays stay correct when eager batched launches, which leave the ticket
    counter advanced, run on the same handle between them. Every call runs
    once at its exact size before the capture, so no later call grows (and
    frees) a buffer the graph holds."""
    torch = torch_cuda
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, tile=(256, 16))
    K = 2
    sos = workloads.sweep_sections(K, "random")
    sosd = dev(np.asarray(sos, np.float32))
    n = 200003
    x = workloads.signal(n, seed=91)
    xd = dev(x)
    yd = torch.empty_like(xd)
    yr, _ = oracle.sosfilt(sos, x)
    Ks, rows, sig_off, bzi = workloads.uneven_batch(B=16, log2_lo=4, log2_hi=15, seed=92)
    bx = workloads.batch_signal(int(sig_off[-1]), seed=93)
    bargs = (dev(bx), dev(rows), dev(Ks.astype(np.int32)), dev(sig_off.astype(np.int64)))
    so = np.r_[0, np.cumsum(Ks)]
    i = 5
    ybr, _ = oracle.sosfilt(rows[so[i]:so[i + 1]], bx[sig_off[i]:sig_off[i + 1]], bzi[so[i]:so[i + 1]])

    def batched():
        yb, _ = P.sosfilt_batched(*bargs, zi=dev(bzi), handle=h)
        torch.cuda.synchronize()
        e = rel_l2(yb.cpu().numpy()[sig_off[i]:sig_off[i + 1]], ybr)
        assert e <= tol_for(int(Ks[i])), e

    P.sosfilt_(xd, sosd, yd, handle=h)
    batched()
    P.sosfilt_(xd, sosd, yd, handle=h)
    torch.cuda.synchronize()
    assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.sosfilt_(xd, sosd, yd, handle=h)
    for rep in range(3):
        batched()
        yd.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K), rep
        P.sosfilt_(xd, sosd, yd, handle=h)          # eager, after the replay
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K), rep
    assert h.last_error() == P.SOS_OK


def test_batched_launch_captured_then_plain_calls(torch_cuda, P):
    """The mirror case: a batched launch captured into a graph on the caller's
    handle, replayed between eager plain calls on that handle. Each replay
    leaves the ticket counter advanced while the host still believes the
    handle armed (its last eager call was plain), so once a batched launch has
    been captured every plain call arms first."""
    torch = torch_cuda
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0, tile=(256, 16))
    K = 3
    sos = workloads.sweep_sections(K, "random")
    sosd = dev(np.asarray(sos, np.float32))
    n = 150001
    x = workloads.signal(n, seed=94)
    xd = dev(x)
    yd = torch.empty_like(xd)
    yr, _ = oracle.sosfilt(sos, x)
    Ks, rows, sig_off, bzi = workloads.uneven_batch(B=12, log2_lo=4, log2_hi=15, seed=95)
    bx = workloads.batch_signal(int(sig_off[-1]), seed=96)
    bargs = (dev(bx), dev(rows), dev(Ks.astype(np.int32)), dev(sig_off.astype(np.int64)))
    bzid = dev(bzi)
    so = np.r_[0, np.cumsum(Ks)]
    refs = [oracle.sosfilt(rows[so[i]:so[i + 1]], bx[sig_off[i]:sig_off[i + 1]],
                           bzi[so[i]:so[i + 1]])[0] for i in range(len(Ks))]
    # every argument given, so that the call needs no host synchronisation
    bkw = dict(zi=bzid, y=torch.empty_like(bargs[0]), zf=torch.empty_like(dev(bzi)),
               sec_off=dev(so.astype(np.int32)), kmax=int(Ks.max()), handle=h)
    P.sosfilt_(xd, sosd, yd, handle=h)
    P.sosfilt_batched(*bargs, **bkw)                 # sizes every buffer before the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        yb, _ = P.sosfilt_batched(*bargs, **bkw)
    for rep in range(3):
        P.sosfilt_(xd, sosd, yd, handle=h)
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K), rep
        yb.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        ybh = yb.cpu().numpy()
        for i in range(len(Ks)):
            assert rel_l2(ybh[sig_off[i]:sig_off[i + 1]], refs[i]) <= tol_for(int(Ks[i])), (rep, i)
        yd.fill_(float("nan"))
        P.sosfilt_(xd, sosd, yd, handle=h)          # eager, right after the replay
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= tol_for(K), rep
    assert h.last_error() == P.SOS_OK


@pytest.mark.parametrize("alg", ["dccr", "ph", None])
@pytest.mark.parametrize("a1,a2", [(-2 * np.cos(0.3), 1.0),   # pair of poles on the unit circle
                                   (1.5, 0.5),                # real pole at z = -1
                                   (-1.5, 0.5),               # real pole at z = +1
                                   (0.0, -1.0)])              # poles at z = +1 and -1
def test_poles_on_the_unit_circle_are_rejected(torch_cuda, P, alg, a1, a2):
    """The stability check is the open triangle |a2| < 1, |a1| < 1 + a2:
    poles on the unit circle (where the state-map powers do not decay across
    groups) report SOS_EUNSTABLE and poison the output; a section just
    inside is filtered."""
    torch = torch_cuda
    h = P.Handle(0, algorithm=alg)
    x = torch.from_numpy(workloads.signal(5000, 3)).cuda()
    sos = np.array([[1.0, 0.3, 0.2, 1.0, a1, a2]], np.float32)
    y, zf = P.sosfilt(x, torch.from_numpy(sos).cuda(), handle=h)
    assert h.last_error() == P.SOS_EUNSTABLE
    assert torch.isnan(y).all().item()
    inside = sos.copy()
    inside[0, 4:] *= np.float32(0.999)               # both poles pulled inside
    y, zf = P.sosfilt(x, torch.from_numpy(inside).cuda(), handle=h)
    assert h.last_error() == P.SOS_OK
    yr, _ = oracle.sosfilt(inside.astype(np.float64), x.cpu().numpy())
    assert np.all(np.isfinite(y.cpu().numpy()))
    assert rel_l2(y.cpu().numpy(), yr) <= 1e-3
