"""GPU checks of the captured uneven batch (sos_graph_*) and of the
autotuner (sos_tune_batched): every graph replay, with new data written into
the captured buffers and eager work in between, equals the eager batched
call on the same data and the FP64 oracle; the tuner returns a compiled tile
whose result equals the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import fp32_bounds, rel_l2, zf_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2607_23763_amd as P

    P.lib()
    return torch, P


def check_vs_oracle(Ks, rows, sig_off, x, zi, y, zf):
    yr, zfr = oracle.sosfilt_batched(Ks, rows, sig_off, x, zi, nthreads=8)
    so = np.r_[0, np.cumsum(Ks)]
    for i in range(len(Ks)):
        a, b = sig_off[i], sig_off[i + 1]
        if b == a:
            continue
        by, bz = fp32_bounds(int(Ks[i]), rows[so[i]:so[i + 1]], x[a:b], zi[so[i]:so[i + 1]],
                             yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(y[a:b], yr[a:b]) <= by, (i, Ks[i], b - a)
        bz = zf_bound(int(Ks[i]), by, bz, yr[a:b], zfr[so[i]:so[i + 1]])
        assert rel_l2(zf[so[i]:so[i + 1]], zfr[so[i]:so[i + 1]]) <= bz, i


@pytest.mark.parametrize("tile", [(256, 16), (512, 64)])
def test_graph_replays_match_eager_and_oracle(env, tile):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=64, log2_lo=2, log2_hi=16, seed=61)
    total = int(sig_off[-1])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    xg = dev(workloads.batch_signal(total, seed=62))
    zig, rowsg = dev(zi), dev(rows)
    Kg, sg = dev(Ks.astype(np.int32)), dev(sig_off.astype(np.int64))
    h = P.Handle(0, tile=tile)
    gr = P.BatchGraph(xg, rowsg, Kg, sg, zi=zig, handle=h)
    he = P.Handle(0, tile=tile)
    for rep in range(3):
        x = workloads.batch_signal(total, seed=63 + rep)
        zi_r = workloads.initial_state(int(Ks.sum()), workloads.rng(70 + rep))
        so_r = sig_off.copy()
        if rep == 2:
            # new lengths, same bounds: the work table is rebuilt on the device
            lens = np.diff(sig_off)[::-1].copy()
            so_r[1:] = np.cumsum(lens)
            sg.copy_(dev(so_r))
        xg.copy_(dev(x))
        zig.copy_(dev(zi_r))
        gr.launch()
        torch.cuda.synchronize()
        assert gr.last_error() == P.SOS_OK
        y_graph, zf_graph = gr.y.cpu().numpy(), gr.zf.cpu().numpy()
        # eager work between replays, then the eager call on the same data
        ye, zfe = P.sosfilt_batched(dev(x), rowsg, Kg, dev(so_r), zi=dev(zi_r), handle=he)
        torch.cuda.synchronize()
        assert he.last_error() == P.SOS_OK
        ye, zfe = ye.cpu().numpy(), zfe.cpu().numpy()
        scale = max(np.abs(ye).max(), 1.0)
        print("replay", rep, "max |graph - eager| / scale", np.abs(y_graph - ye).max() / scale)
        assert np.abs(y_graph - ye).max() <= 1e-5 * scale
        check_vs_oracle(Ks, rows, so_r, x, zi_r, y_graph, zf_graph)
    gr.close()


def test_tuner_returns_a_compiled_tile_with_exact_output(env):
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=128, log2_lo=8, log2_hi=18, seed=64)
    x = workloads.batch_signal(int(sig_off[-1]), seed=65)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h = P.Handle(0)
    (L, N), ms, y, zf = P.tune_batched(dev(x), dev(rows), dev(Ks.astype(np.int32)),
                                       dev(sig_off.astype(np.int64)), zi=dev(zi), handle=h,
                                       reps=2)
    torch.cuda.synchronize()
    print("tuned tile", (L, N), h.algorithm(), "%.4f ms" % ms)
    assert h.last_error() == P.SOS_OK
    assert h.tile() == (L, N) and ms > 0
    assert h.algorithm() in ("auto", "ph")          # no solver set: both were timed
    assert (L, N) in {(64, 16), (64, 32), (64, 64), (256, 16), (256, 32), (256, 64),
                      (512, 16), (512, 32), (512, 64), (1024, 16), (1024, 32)}
    check_vs_oracle(Ks, rows, sig_off, x, zi, y.cpu().numpy(), zf.cpu().numpy())


def test_tuner_keeps_an_explicit_solver(env):
    """A handle with a solver set is tuned over tiles only, keeps its solver,
    and the cached tile is found again for the same request."""
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=32, log2_lo=8, log2_hi=14, seed=66)
    x = workloads.batch_signal(int(sig_off[-1]), seed=67)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for alg in ("dccr", "ph"):
        h = P.Handle(0, algorithm=alg)
        (L, N), ms, y, zf = P.tune_batched(dev(x), dev(rows), dev(Ks.astype(np.int32)),
                                           dev(sig_off.astype(np.int64)), zi=dev(zi), handle=h,
                                           reps=1)
        torch.cuda.synchronize()
        assert h.last_error() == P.SOS_OK
        assert h.algorithm() == alg and h.tile() == (L, N)
        Lc, Nc = P.ctypes.c_int(), P.ctypes.c_int()
        assert P.lib().sos_tune_lookup(h.ptr, len(Ks), int(Ks.max()), int(sig_off[-1]),
                                       P.ctypes.byref(Lc), P.ctypes.byref(Nc)) == P.SOS_OK
        assert (Lc.value, Nc.value) == (L, N)
        check_vs_oracle(Ks, rows, sig_off, x, zi, y.cpu().numpy(), zf.cpu().numpy())


def test_cost_model_residency_matches_the_runtime(env):
    """The tuner's model on MI355X's budgets, fed each compiled forward
    kernel's own register count, gives the resident workgroups per CU that
    the runtime's occupancy calculator reports, for every shape, both compute
    types and every kernel variant the launches use."""
    torch, P = env
    L = P.lib()
    d = P.model_device_gfx950()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert cus == d.sms
    checked = 0
    for bits in (32, 64):
        for alg in (0, 1, 4, 5):
            if bits == 64 and alg >= 4:
                continue
            for Lg in (64, 256, 512, 1024):
                for N in (16, 32, 64):
                    if not L.sos_fwd_shape_supported(Lg, N):
                        continue
                    regs, lds = P.fwd_kernel_attrs(bits, alg, Lg, N)
                    cap = L.sos_fwd_capacity(bits, alg, Lg, N)
                    assert regs > 0 and cap > 0 and lds >= 4 * Lg * (N + 4)
                    # the kernel's whole LDS (staging rows plus the wave
                    # exchange) as row padding
                    pad = -(-lds // (4 * Lg)) - N
                    c = P.model_config(d, Lg, N, pad=pad, regs=regs)
                    assert cap // cus == c.tbs_per_sm and cap % cus == 0, \
                        (bits, alg, Lg, N, regs, lds, cap // cus, c.tbs_per_sm, c.limit)
                    checked += 1
    assert checked >= 30


def test_tuner_rejects_filtering_in_place(env):
    """The tuner runs the batch many times, so it cannot filter in place: x
    as y (with samples) and zi as zf are rejected before anything runs."""
    torch, P = env
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=8, log2_lo=10, log2_hi=12, seed=95)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    x = dev(workloads.batch_signal(int(sig_off[-1]), seed=96))
    x0 = x.clone()
    zid = dev(zi)
    h = P.Handle(0)
    with pytest.raises(Exception) as e:
        P.tune_batched(x, dev(rows), dev(Ks.astype(np.int32)), dev(sig_off), zi=zid, y=x,
                       handle=h)
    assert getattr(e.value, "code", None) == P.SOS_EINVAL
    with pytest.raises(Exception) as e:
        P.tune_batched(x, dev(rows), dev(Ks.astype(np.int32)), dev(sig_off), zi=zid, zf=zid,
                       handle=h)
    assert getattr(e.value, "code", None) == P.SOS_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(x, x0)
