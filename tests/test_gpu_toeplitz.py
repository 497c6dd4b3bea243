"""GPU parity of the whole-cascade block-Toeplitz path (sos_toep.hip): the
multi-block split of Sec. II-B taken over the whole cascade (zero-state
output T x, column end states Gam x, column and tile scans, a 16-word
decoupled lookback per chunk of two, four or eight groups, y += O s), on the
matrix cores. Same FP64 oracle and bounds as the per-section kernels:
relative L2 error <= 1e-5 up to order 8 and <= 1e-4 at order 16 (or 10x the
sequential FP32 error, where that is larger), zf to the same bounds; exact,
ragged and one-group lengths at every chunk size, initial states, in place,
many groups per workgroup, the chunk size chosen from the length, and the
automatic choice."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, rel_l2, zf_bound

pytestmark = pytest.mark.gpu

CG = 16384   # samples per group of the block-Toeplitz kernel
CHUNK = 8 * CG   # samples per ticket (one lookback per chunk) at 8 groups per chunk


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


def run(torch, P, sos, x, zi=None, algorithm="toeplitz"):
    h = P.Handle(0, algorithm=algorithm)
    y, zf = P.sosfilt(dev(torch, x), dev(torch, np.asarray(sos, np.float32)),
                      None if zi is None else dev(torch, np.asarray(zi, np.float32)), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    return y.cpu().numpy(), zf.cpu().numpy()


def check(sos, x, zi, y, zf, label):
    K = sos.shape[0]
    ref, zref = oracle.sosfilt(np.asarray(sos, np.float64), np.asarray(x, np.float64),
                               None if zi is None else np.asarray(zi, np.float64))
    ref = np.asarray(ref)
    zref = np.asarray(zref).reshape(K, 2)
    by, bz = fp32_bounds(K, sos, x, zi, ref, zref)
    ey, ez = rel_l2(y, ref), rel_l2(zf, zref)
    print(label, "y", ey, "bound", by, "zf", ez)
    assert ey <= by, (label, ey, by)
    assert ez <= zf_bound(K, by, bz, ref, zref), (label, ez, bz)


@pytest.mark.parametrize("kind", ["butter", "random"])
@pytest.mark.parametrize("K", [1, 2, 4, 8])
@pytest.mark.parametrize("n", [5 * CG, 3 * CG + 1237, 100, 1])
def test_parity_with_initial_state(env, kind, K, n):
    torch, P = env
    sos = workloads.sweep_sections(K, kind)
    x = workloads.signal(n, 40 + K)
    zi = workloads.initial_state(K, workloads.rng(7 + K))
    y, zf = run(torch, P, sos, x, zi)
    check(sos, x, zi, y, zf, "%s K=%d n=%d" % (kind, K, n))


@pytest.mark.parametrize("n", [64, 1024, CG - 1, CG, CG + 1, 2 * CG + 64, CHUNK - 1, CHUNK,
                               CHUNK + 1, 7 * CG + 4097, 2 * CHUNK, 9 * CG + 5])
def test_lengths_across_column_tile_and_group_edges(env, monkeypatch, n):
    torch, P = env
    monkeypatch.setenv("SOS_TOEP_CHUNK", "8")
    sos = workloads.butterworth_sos(8)
    x = workloads.signal(n, n % 1000)
    y, zf = run(torch, P, sos, x)
    check(sos, x, None, y, zf, "edges n=%d" % n)


# signal lengths for a chunk of c samples
SMALL_CHUNK_LENGTHS = {
    "chunk-1": lambda c: c - 1,
    "chunk": lambda c: c,
    "chunk+1": lambda c: c + 1,
    "2chunks+5": lambda c: 2 * c + 5,
    "7groups+4097": lambda c: 7 * CG + 4097,
    "group-1": lambda c: CG - 1,
}


@pytest.mark.parametrize("ng", [2, 4])
@pytest.mark.parametrize("case", list(SMALL_CHUNK_LENGTHS))
def test_lengths_across_smaller_chunks(env, monkeypatch, ng, case):
    """Chunks of 2 and 4 groups: lengths on either side of a chunk edge,
    ragged ends inside later chunks, and a signal shorter than one group."""
    torch, P = env
    monkeypatch.setenv("SOS_TOEP_CHUNK", str(ng))
    n = SMALL_CHUNK_LENGTHS[case](ng * CG)
    K = 8 if ng == 2 else 5
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, n % 997)
    zi = workloads.initial_state(K, workloads.rng(n % 13))
    y, zf = run(torch, P, sos, x, zi)
    check(sos, x, zi, y, zf, "chunk %d n=%d" % (ng, n))


def test_in_place_with_ragged_end(env):
    """x == y: every tile is loaded before it is stored, and the final state of
    a ragged end reads its column's input before the tile is written."""
    torch, P = env
    K, n = 6, 4 * CG + 777
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, 11)
    zi = workloads.initial_state(K, workloads.rng(3))
    h = P.Handle(0, algorithm="toeplitz")
    xd = dev(torch, x)
    zf = torch.empty((K, 2), dtype=torch.float32, device="cuda")
    P.sosfilt_(xd, dev(torch, sos), y=xd, zi=dev(torch, zi), zf=zf, handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_OK
    check(sos, x, zi, xd.cpu().numpy(), zf.cpu().numpy(), "in place")


@pytest.mark.parametrize("ng", [2, 4, 8])
@pytest.mark.parametrize("grid", [1, 3])
def test_many_groups_per_workgroup(env, monkeypatch, grid, ng):
    """A persistent grid of 1 or 3 workgroups walks the 201 groups in chunks
    of 2, 4 or 8: the next group's samples are always in flight, and
    lookbacks find their predecessors already resolved."""
    torch, P = env
    monkeypatch.setenv("SOS_GRID", str(grid))
    monkeypatch.setenv("SOS_TOEP_CHUNK", str(ng))
    K, n = 8, 200 * CG + 3
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, 5)
    zi = workloads.initial_state(K, workloads.rng(5))
    y, zf = run(torch, P, sos, x, zi)
    check(sos, x, zi, y, zf, "grid %d" % grid)


@pytest.mark.parametrize("K,n,ng", [(4, 1 << 25, None), (8, 1 << 25, None),
                                    (8, (1 << 24) + 333, None), (8, 1 << 25, 8),
                                    (6, 1 << 23, 2)])
def test_full_device_lookback(env, monkeypatch, K, n, ng):
    """2^23 to 2^25 samples on the whole device, with the chunk size the
    length selects (or a forced one): every workgroup's lookback walks
    windows of in-flight predecessors."""
    torch, P = env
    if ng is None:
        monkeypatch.delenv("SOS_TOEP_CHUNK", raising=False)
    else:
        monkeypatch.setenv("SOS_TOEP_CHUNK", str(ng))
    sos = workloads.butterworth_sos(K)
    x = workloads.signal(n, 77)
    y, zf = run(torch, P, sos, x)
    check(sos, x, None, y, zf, "n=%d K=%d chunk %s" % (n, K, ng))


def test_automatic_choice_takes_the_toeplitz_path(env, monkeypatch):
    """The automatic solver runs orders 14-16 of at least 2^25 samples and
    order 12 of at least 2^26 through the block-Toeplitz kernel (its output
    equals an explicit block-Toeplitz handle's bit for bit, and differs from
    the per-section kernels'), lower orders and shorter signals through the
    per-section kernels. The check against the oracle uses a 2^20-sample
    prefix (causal: the same outputs)."""
    torch, P = env
    monkeypatch.delenv("SOS_ALG", raising=False)
    n = (1 << 27) + 12345
    x = workloads.signal(n, 8)
    sos = workloads.butterworth_sos(8)
    ya, _ = run(torch, P, sos, x, algorithm="auto")
    yt, _ = run(torch, P, sos, x, algorithm="toeplitz")
    yp, _ = run(torch, P, sos, x, algorithm="ph")
    assert np.array_equal(ya, yt)
    assert not np.array_equal(ya, yp)
    m = 1 << 20
    ref, _ = oracle.sosfilt(sos.astype(np.float64), x[:m].astype(np.float64))
    assert rel_l2(ya[:m], ref) <= 1e-4
    del ya, yt, yp
    sos6 = workloads.butterworth_sos(6)
    ya6, _ = run(torch, P, sos6, x, algorithm="auto")
    yt6, _ = run(torch, P, sos6, x, algorithm="toeplitz")
    assert np.array_equal(ya6, yt6)
    sos5 = workloads.butterworth_sos(5)
    ya5, _ = run(torch, P, sos5, x, algorithm="auto")
    yt5, _ = run(torch, P, sos5, x, algorithm="toeplitz")
    assert not np.array_equal(ya5, yt5)
    del ya6, yt6, ya5, yt5
    # each order at its threshold takes the block-Toeplitz kernel, one
    # sample less takes the section kernels: orders 16 and 14 at 2^25, order
    # 12 at 2^26
    sos7 = workloads.butterworth_sos(7)
    for cascade, lg in ((sos, 25), (sos7, 25), (sos6, 26)):
        for m, same in (((1 << lg), True), ((1 << lg) - 1, False)):
            ys, _ = run(torch, P, cascade, x[:m], algorithm="auto")
            yts, _ = run(torch, P, cascade, x[:m], algorithm="toeplitz")
            assert np.array_equal(ys, yts) == same, (cascade.shape[0], m)
            del ys, yts


@pytest.mark.parametrize("K", [6, 8])
def test_prepared_tables_serve_any_length(env, monkeypatch, K):
    """Tables from sos_prepare, whose signal length is unknown (8-group
    chunks), filter signals shorter than a group, ragged inside a chunk and
    across chunk edges, with zi and zf; the automatic choice's prepared
    tables give the same parity on lengths below its threshold."""
    torch, P = env
    monkeypatch.delenv("SOS_TOEP_CHUNK", raising=False)
    monkeypatch.delenv("SOS_ALG", raising=False)
    sos = workloads.sweep_sections(K, "random")
    for alg in ("toeplitz", "auto"):
        h = P.Handle(0, algorithm=alg)
        P.prepare(dev(torch, sos), handle=h)
        for n in (CG - 3, 3 * CG + 77, CHUNK + 1, 2 * CHUNK + 4097):
            x = workloads.signal(n, n % 101)
            zi = workloads.initial_state(K, workloads.rng(n % 7))
            xd = dev(torch, x)
            yd = torch.empty_like(xd)
            zf = torch.empty((K, 2), dtype=torch.float32, device="cuda")
            P.filter_prepared(xd, yd, zi=dev(torch, zi), zf=zf, handle=h)
            torch.cuda.synchronize()
            assert h.last_error() == P.SOS_OK
            check(sos, x, zi, yd.cpu().numpy(), zf.cpu().numpy(),
                  "prepared %s K=%d n=%d" % (alg, K, n))


def lightly_damped_sections(K=8, r=0.995, seed=9):
    sos = workloads.random_stable_sos(K, workloads.rng(seed), r_fixed=r)
    imp = np.zeros(40000)
    imp[0] = 1.0
    hr, _ = oracle.sosfilt(sos, imp)
    sos[0, :3] /= np.sqrt(np.sum(hr ** 2))
    return sos.astype(np.float32)


def test_gate_keeps_resonant_cascades_on_the_section_kernels(env, monkeypatch):
    """Poles at radius 0.995 (peak gains far above 128): the automatic choice
    leaves the cascade to the per-section kernels (the accurate layout, as an
    explicit PH handle), while an explicit block-Toeplitz handle filters it
    within the order-16 bound or 10x the sequential FP32 error."""
    torch, P = env
    monkeypatch.delenv("SOS_ALG", raising=False)
    sos = lightly_damped_sections()
    n = (1 << 27) + 5
    x = workloads.signal(n, 21)
    ya, _ = run(torch, P, sos, x, algorithm="auto")
    yp, _ = run(torch, P, sos, x, algorithm="ph")
    assert rel_l2(ya, yp) < 1e-6
    yt, _ = run(torch, P, sos, x, algorithm="toeplitz")
    assert not np.array_equal(yt, ya)
    del ya, yp, yt
    m = (1 << 20) + 5
    yt, zt = run(torch, P, sos, x[:m], algorithm="toeplitz")
    check(sos, x[:m], None, yt, zt, "damped16 toeplitz")


def test_unstable_section_is_reported(env):
    """A section on the stability boundary is never taken by the block-Toeplitz
    kernel: the per-section kernels run and report it."""
    torch, P = env
    sos = workloads.butterworth_sos(4).copy()
    sos[2, 5] = 1.0           # a2 = 1: poles on the unit circle
    x = workloads.signal(2 * CG, 1)
    h = P.Handle(0, algorithm="toeplitz")
    y, _ = P.sosfilt(dev(torch, x), dev(torch, sos), handle=h)
    torch.cuda.synchronize()
    assert h.last_error() == P.SOS_EUNSTABLE
    assert torch.isnan(y).all().item()


def test_misaligned_buffers(env):
    """Input and output at every 4-byte offset from a 16-byte boundary (the
    128-bit accesses at dword alignment), the two offsets differing, with a
    ragged end: results and zf as aligned, nothing written outside."""
    torch, P = env
    K, n = 8, 3 * CHUNK + 4097
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, 12)
    ref, zref = oracle.sosfilt(sos.astype(np.float64), x.astype(np.float64))
    zref = np.asarray(zref).reshape(K, 2)
    h = P.Handle(0, algorithm="toeplitz")
    sd = dev(torch, sos)
    zf = torch.empty((K, 2), dtype=torch.float32, device="cuda")
    for oi, oo in ((1, 1), (2, 3), (3, 2), (0, 1), (1, 0)):
        buf = torch.zeros(n + 4, device="cuda")
        buf[oi:oi + n] = dev(torch, x)
        out = torch.zeros(n + 4, device="cuda")
        P.sosfilt_(buf[oi:oi + n], sd, y=out[oo:oo + n], zf=zf, handle=h)
        torch.cuda.synchronize()
        assert h.last_error() == P.SOS_OK
        o = out.cpu().numpy()
        assert rel_l2(o[oo:oo + n], ref) <= 1e-4, (oi, oo)
        assert not o[:oo].any() and not o[oo + n:].any(), (oi, oo)
        assert rel_l2(zf.cpu().numpy(), zref) <= 1e-4, (oi, oo)


def test_captured_in_a_graph(env):
    """A block-Toeplitz call captured into a graph (both preparations, the arm
    step, the filter and the section kernels that leave at once), replayed
    three times with eager batched launches (which run PH on this handle and
    leave the ticket counter advanced) and eager plain calls in between: every
    replay and every eager call matches the oracle."""
    torch, P = env
    h = P.Handle(0, algorithm="toeplitz")
    K, n = 8, 2 * CHUNK + 777
    sos = workloads.sweep_sections(K, "random")
    sosd = dev(torch, sos)
    x = workloads.signal(n, 93)
    xd = dev(torch, x)
    yd = torch.empty_like(xd)
    yr, _ = oracle.sosfilt(sos.astype(np.float64), x.astype(np.float64))
    Ks, rows, sig_off, bzi = workloads.uneven_batch(B=16, log2_lo=4, log2_hi=15, seed=92)
    bx = workloads.batch_signal(int(sig_off[-1]), seed=94)
    bargs = (dev(torch, bx), dev(torch, rows), dev(torch, Ks.astype(np.int32)),
             dev(torch, sig_off.astype(np.int64)))
    so = np.r_[0, np.cumsum(Ks)]
    i = 5
    ybr, _ = oracle.sosfilt(rows[so[i]:so[i + 1]].astype(np.float64),
                            bx[sig_off[i]:sig_off[i + 1]].astype(np.float64),
                            bzi[so[i]:so[i + 1]].astype(np.float64))

    def batched():
        yb, _ = P.sosfilt_batched(*bargs, zi=dev(torch, bzi), handle=h)
        torch.cuda.synchronize()
        assert rel_l2(yb.cpu().numpy()[sig_off[i]:sig_off[i + 1]], ybr) <= 1e-4

    P.sosfilt_(xd, sosd, yd, handle=h)
    batched()
    P.sosfilt_(xd, sosd, yd, handle=h)
    torch.cuda.synchronize()
    assert rel_l2(yd.cpu().numpy(), yr) <= 1e-4
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        P.sosfilt_(xd, sosd, yd, handle=h)
    for rep in range(3):
        batched()
        yd.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= 1e-4, rep
        P.sosfilt_(xd, sosd, yd, handle=h)
        torch.cuda.synchronize()
        assert rel_l2(yd.cpu().numpy(), yr) <= 1e-4, rep
    assert h.last_error() == P.SOS_OK


def test_lookback_timeout_is_bounded_and_reported(env):
    """A one-tick bound on each chunk's lookback wait, forced from the host:
    the launch still ends (a chunk whose wait ran out publishes a NaN state,
    so its successors finish too), any NaN output comes with SOS_ETIMEOUT, and
    with the default bound restored the same handle is exact."""
    torch, P = env
    K, n = 8, 1 << 24
    sos = workloads.sweep_sections(K, "random")
    x = workloads.signal(n, 31)
    h = P.Handle(0, algorithm="toeplitz")
    xd, sd = dev(torch, x), dev(torch, sos)
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
    m = 1 << 20
    yr, _ = oracle.sosfilt(sos.astype(np.float64), x[:m].astype(np.float64))
    assert rel_l2(y.cpu().numpy()[:m], yr) <= 1e-4
    assert bool(torch.isfinite(y).all().item())
