"""GPU checks of the serving layer (sos_server_* / sos_stream_*): every
stream's chunks, filtered through the continuous-batching server with its
state kept on the device, equal the FP64 oracle run once over the stream's
concatenated chunks; a stream's output is the same alone and in the mix; the
admission limits and error paths hold.

Random cascades of orders up to 16 with zero initial state can attenuate the
signal by orders of magnitude (sections resonating at different frequencies,
each with a notch); there even a sequential FP32 filter misses the order's
bound. FP32 results are held to fp32_bound (the order's bound, or a fixed
multiple of the sequential FP32 error when that is larger) and the FP64
compute type to the order's bound itself."""
import threading

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bound, fp32_bounds, fp32_floor, rel_l2, tol_for, zf_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def small_trace(S=24, R=120, seed=41):
    Ks, secs, ids, lens, offs, arrival = workloads.serving_trace(
        S=S, R=R, rate_chunks_per_s=1e6, lo=64, hi=20000, seed=seed)
    lens[5] = 0                  # an empty chunk
    lens[7] = 1                  # a one-sample chunk
    offs = np.zeros(R, dtype=np.int64)
    np.cumsum(lens[:-1], out=offs[1:])
    return Ks, secs, ids, lens, offs, arrival


def oracle_per_stream(Ks, secs, ids, lens, offs, x, zis=None):
    """Per stream: oracle output over the concatenated chunks, final state,
    and the bound its FP32 result is held to."""
    ys, zfs, bounds = {}, {}, {}
    for s in range(len(Ks)):
        idx = np.nonzero(ids == s)[0]
        if len(idx) == 0:
            continue
        xs = np.concatenate([x[offs[r]:offs[r] + lens[r]] for r in idx])
        zi = None if zis is None else zis[s]
        y, zf = oracle.sosfilt(secs[s], xs, zi)
        ys[s], zfs[s] = y, zf
        by, bz = fp32_bounds(int(Ks[s]), secs[s], xs, zi, y, zf)
        bounds[s] = (by, zf_bound(int(Ks[s]), by, bz, y, zf))
    return ys, zfs, bounds


def gathered(y, ids, lens, offs, s):
    idx = np.nonzero(ids == s)[0]
    return np.concatenate([y[offs[r]:offs[r] + lens[r]] for r in idx])


def serve_all(torch, P, Ks, secs, ids, lens, offs, xd, tile=(256, 16), zis=None, order=None,
              max_slots=64, precision=0):
    srv = P.Server(tile=tile, max_slots=max_slots, precision=precision)
    sid = [srv.open(secs[s], None if zis is None else zis[s]) for s in range(len(Ks))]
    yd = torch.full_like(xd, float("nan"))
    tickets = []
    for r in (range(len(ids)) if order is None else order):
        o, n = int(offs[r]), int(lens[r])
        tk, _ = srv.push(sid[ids[r]], xd[o:o + n], yd[o:o + n])
        tickets.append(tk)
    lat = [srv.wait(t) for t in tickets]
    states = {s: srv.state(sid[s]) for s in range(len(Ks))}
    srv.close()
    return yd.cpu().numpy(), states, np.array(lat)


def test_streams_match_oracle(env):
    torch, P = env
    Ks, secs, ids, lens, offs, _ = small_trace()
    x = workloads.signal(int(lens.sum()), seed=42)
    xd = torch.from_numpy(x).cuda()
    y, states, lat = serve_all(torch, P, Ks, secs, ids, lens, offs, xd)
    y64, states64, _ = serve_all(torch, P, Ks, secs, ids, lens, offs, xd, precision=64)
    yr, zfr, bnd = oracle_per_stream(Ks, secs, ids, lens, offs, x)
    for s in yr:
        e = rel_l2(gathered(y, ids, lens, offs, s), yr[s])
        assert e <= bnd[s][0], (s, Ks[s], e, bnd[s])
        assert rel_l2(states[s], zfr[s]) <= bnd[s][1], s
        e64 = rel_l2(gathered(y64, ids, lens, offs, s), yr[s])
        assert e64 <= tol_for(int(Ks[s])), (s, Ks[s], e64)
        assert rel_l2(states64[s], zfr[s]) <= tol_for(int(Ks[s])), s
    print("streams whose FP32 bound exceeds the order's:",
          sum(bnd[s][0] > tol_for(int(Ks[s])) for s in bnd), "of", len(bnd))
    assert (lat > 0).all()
    print("chunks", len(ids), "latency p50 %.1f us p99 %.1f us" %
          (1e6 * np.percentile(lat, 50), 1e6 * np.percentile(lat, 99)))


def test_alone_equals_in_the_mix(env):
    """Each stream served alone (a fresh server holding only that stream)
    gives the same output as in the mix with the others, within the order's
    bound; the number of bit-identical streams is reported."""
    torch, P = env
    Ks, secs, ids, lens, offs, _ = small_trace(S=12, R=72, seed=43)
    x = workloads.signal(int(lens.sum()), seed=44)
    xd = torch.from_numpy(x).cuda()
    y_mix, _, _ = serve_all(torch, P, Ks, secs, ids, lens, offs, xd)
    same = 0
    for s in range(len(Ks)):
        idx = np.nonzero(ids == s)[0]
        if len(idx) == 0:
            continue
        sub_ids = np.zeros(len(idx), dtype=np.int64)
        y_alone, _, _ = serve_all(torch, P, Ks[s:s + 1], secs[s:s + 1], sub_ids, lens[idx],
                                  offs[idx], xd)
        a = gathered(y_alone, sub_ids, lens[idx], offs[idx], 0)
        m = gathered(y_mix, ids, lens, offs, s)
        xs = gathered(x, ids, lens, offs, s)
        yr, _ = oracle.sosfilt(secs[s], xs)
        bnd = fp32_bound(int(Ks[s]), fp32_floor(secs[s], xs, None, yr))
        assert rel_l2(a, m) <= bnd, s
        assert rel_l2(a, yr) <= bnd, s
        same += int(np.array_equal(a, m))
    print("bit-identical alone vs mixed:", same, "of", len(set(ids.tolist())))


def test_checkpoint_resume(env):
    """The state read after some chunks, given as zi to a new stream, continues
    the stream exactly as if it had not been interrupted."""
    torch, P = env
    K = 5
    sos = workloads.random_stable_sos(K, workloads.rng(45))
    x = workloads.signal(30000, seed=46)
    xd = torch.from_numpy(x).cuda()
    srv = P.Server(tile=(256, 16))
    a = srv.open(sos)
    y = torch.empty_like(xd)
    for lo, hi in ((0, 7000), (7000, 12001)):
        srv.wait(srv.push(a, xd[lo:hi], y[lo:hi])[0])
    st = srv.state(a)
    b = srv.open(sos, st)
    for lo, hi in ((12001, 20000), (20000, 30000)):
        srv.wait(srv.push(b, xd[lo:hi], y[lo:hi])[0])
    yr, zfr = oracle.sosfilt(sos, x)
    assert rel_l2(y.cpu().numpy(), yr) <= 1e-5
    assert rel_l2(srv.state(b), zfr) <= 1e-5
    srv.close()


def test_admission_and_errors(env):
    torch, P = env
    h = P.Handle(0, tile=(64, 16))
    row_bytes = 6 * 4 + 2 * 4 + 1296 * 4
    srv = P.Server(handle=h, budget=2 * 20 * row_bytes + (1 << 20), max_slots=8)
    lim = srv.limits()
    assert lim["max_rows"] >= 20 and lim["tile"] == (64, 16)
    sos = workloads.random_stable_sos(4, workloads.rng(47))
    opened = []
    with pytest.raises(P.SosError) as e:
        while True:
            opened.append(srv.open(sos))
    assert e.value.code == P.SOS_EBUSY
    assert len(opened) == lim["max_rows"] // 4
    srv.close_stream(opened.pop())
    opened.append(srv.open(sos))                      # the rows are reusable
    bad = sos.copy()
    bad[1, 5] = 1.5                                   # |a2| > 1
    srv.close_stream(opened.pop())
    with pytest.raises(P.SosError) as e:
        srv.open(bad)
    assert e.value.code == P.SOS_EUNSTABLE
    big = torch.zeros(lim["max_chunk"] + 1, device="cuda")
    with pytest.raises(P.SosError) as e:
        srv.push(opened[0], big)
    assert e.value.code == P.SOS_EINVAL
    srv.close_stream(opened[0])
    with pytest.raises(P.SosError) as e:
        srv.push(opened[0], big[:10])
    assert e.value.code == P.SOS_ECLOSED
    srv.close()


def test_concurrent_pushers(env):
    """Four host threads push to disjoint streams of one server at once."""
    torch, P = env
    Ks, secs, ids, lens, offs, _ = small_trace(S=16, R=96, seed=48)
    x = workloads.signal(int(lens.sum()), seed=49)
    xd = torch.from_numpy(x).cuda()
    yd = torch.full_like(xd, float("nan"))
    srv = P.Server(tile=(512, 16), max_slots=32)
    sid = [srv.open(secs[s]) for s in range(len(Ks))]
    torch.cuda.synchronize()
    errors = []

    def run(part):
        try:
            tks = []
            for r in range(len(ids)):
                if ids[r] % 4 != part:
                    continue
                o, n = int(offs[r]), int(lens[r])
                tks.append(srv.push(sid[ids[r]], xd[o:o + n], yd[o:o + n])[0])
            for t in tks:
                srv.wait(t)
        except Exception as ex:   # reported below
            errors.append(ex)

    th = [threading.Thread(target=run, args=(p,)) for p in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    y = yd.cpu().numpy()
    yr, _, bnd = oracle_per_stream(Ks, secs, ids, lens, offs, x)
    for s in yr:
        assert rel_l2(gathered(y, ids, lens, offs, s), yr[s]) <= bnd[s][0], s
    srv.close()


def test_replay_poisson_load(env):
    """The native load driver: Poisson arrivals of chunks of 4096..65536
    samples over 64 streams of orders 2..16; outputs equal the oracle per
    stream and every chunk reports a latency."""
    torch, P = env
    Ks, secs, ids, lens, offs, arrival = workloads.serving_trace(
        S=64, R=256, rate_chunks_per_s=2e4, seed=50)
    x = workloads.signal(int(lens.sum()), seed=51)
    xd = torch.from_numpy(x).cuda()
    yd = torch.full_like(xd, float("nan"))
    srv = P.Server(tile=(512, 16), max_slots=256)
    sid = np.array([srv.open(secs[s]) for s in range(len(Ks))], dtype=np.int64)
    lat, wall = srv.replay(sid[ids], offs, lens, arrival, xd, yd)
    srv.close()
    assert (lat > 0).all() and wall > 0
    print("replay: %d chunks %.3f s wall, latency p50 %.1f us p99 %.1f us" %
          (len(ids), wall, 1e6 * np.percentile(lat, 50), 1e6 * np.percentile(lat, 99)))
    y = yd.cpu().numpy()
    yr, _, bnd = oracle_per_stream(Ks, secs, ids, lens, offs, x)
    for s in yr:
        assert rel_l2(gathered(y, ids, lens, offs, s), yr[s]) <= bnd[s][0], s


def test_device_errors_reach_their_chunks(env):
    """Device-side errors are per chunk and sticky per stream. A one-tick
    lookback bound, forced from the host, on long chunks of stream a yields
    SOS_ETIMEOUT (with NaN outputs from the failed group on) or SOS_OK; once a
    chunk of a failed, its later chunks and pushes report the same status and
    its state is not exported. Stream b's one-group chunks, which never wait
    and share steps with a's, stay SOS_OK and exact; so do the chunks of a
    stream opened after a was closed and reopened."""
    torch, P = env
    h = P.Handle(0, tile=(64, 16))
    h.set_timeout(1e-6)
    srv = P.Server(handle=h, max_slots=8)
    sos = workloads.sweep_sections(4, "random")
    a = srv.open(sos)
    b = srv.open(sos)
    x = torch.from_numpy(workloads.signal(1 << 18, seed=9)).cuda()
    xs = workloads.signal(500, seed=10)
    xsd = torch.from_numpy(xs).cuda()
    codes, ys, tks = [], [], []
    for _ in range(4):
        y = torch.empty_like(x)
        yb = torch.empty(500, device="cuda")
        try:
            tk, _ = srv.push(a, x, y)
        except P.SosError as e:                      # a already failed
            assert e.code == P.SOS_ETIMEOUT
            tk = None
        tks.append((tk, srv.push(b, xsd, yb)[0]))
        ys.append((y, yb))
    failed = False
    yb_all = []
    for (tka, tkb), (y, yb) in zip(tks, ys):
        code = P.SOS_ETIMEOUT
        if tka is not None:
            try:
                srv.wait(tka)
                code = P.SOS_OK
            except P.SosError as e:
                code = e.code
        assert code in (P.SOS_OK, P.SOS_ETIMEOUT)
        if failed:
            assert code == P.SOS_ETIMEOUT            # sticky after the first failure
        elif code == P.SOS_ETIMEOUT:
            assert bool(torch.isnan(y).any().item())
        else:
            assert not bool(torch.isnan(y).any().item())
        failed |= code == P.SOS_ETIMEOUT
        codes.append(code)
        srv.wait(tkb)                                # b's chunks are unaffected
        yb_all.append(yb.cpu().numpy())
    print("one-tick bound, stream a codes", codes)
    yr, _ = oracle.sosfilt(sos, np.tile(xs, 4))
    assert rel_l2(np.concatenate(yb_all), yr) <= 1e-5
    if failed:
        with pytest.raises(P.SosError) as ei:
            srv.push(a, x, torch.empty_like(x))
        assert ei.value.code == P.SOS_ETIMEOUT
        with pytest.raises(P.SosError) as ei:
            srv.state(a)
        assert ei.value.code == P.SOS_ETIMEOUT
    srv.close_stream(a)
    c = srv.open(sos)
    ys2 = torch.empty(500, device="cuda")
    tk, _ = srv.push(c, xsd, ys2)
    srv.wait(tk)
    yr, _ = oracle.sosfilt(sos, xs)
    assert rel_l2(ys2.cpu().numpy(), yr) <= 1e-5
    srv.close()


def test_large_steps_on_the_throughput_tile(env):
    """Steps of at least 2^22 samples run at the throughput tile (512, 32) with
    tables prepared for it at stream open; here 8 streams push 4 chunks of
    2^19 samples each at once, so steps carry up to 4.2e6 samples. Every
    stream against the oracle over its concatenated chunks, FP32 and FP64."""
    torch, P = env
    S, per, m = 8, 4, 1 << 19
    g = workloads.rng(47)
    Ks = g.integers(1, 9, size=S).astype(np.int32)
    secs = [workloads.random_stable_sos(int(k), g) for k in Ks]
    ids = np.tile(np.arange(S), per)
    lens = np.full(S * per, m, dtype=np.int64)
    offs = (np.arange(S * per) * m).astype(np.int64)
    x = workloads.signal(S * per * m, seed=48)
    xd = torch.from_numpy(x).cuda()
    y, states, _ = serve_all(torch, P, Ks, secs, ids, lens, offs, xd, max_slots=S)
    y64, states64, _ = serve_all(torch, P, Ks, secs, ids, lens, offs, xd, max_slots=S,
                                 precision=64)
    yr, zfr, bnd = oracle_per_stream(Ks, secs, ids, lens, offs, x)
    for s in yr:
        e = rel_l2(gathered(y, ids, lens, offs, s), yr[s])
        assert e <= bnd[s][0], (s, Ks[s], e, bnd[s])
        assert rel_l2(states[s], zfr[s]) <= bnd[s][1], s
        e64 = rel_l2(gathered(y64, ids, lens, offs, s), yr[s])
        assert e64 <= tol_for(int(Ks[s])), (s, Ks[s], e64)
