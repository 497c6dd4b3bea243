#!/usr/bin/env python3
"""Throughput benchmark of the single-kernel multi-block cascade filter on one MI355X.

Workload (the headline configuration): one FP32 signal of 2^28 i.i.d. N(0,1)
samples, zero initial state, cascades of K = 1, 2, 4, 8 sections (orders 2-16),
Butterworth low-pass at 0.2*Nyquist and random stable sections. The JSON
`value` is the order-2 (K = 1) Butterworth case: samples per second of one
whole step (coefficient preparation + filter kernel) with input and output
resident in HBM, in GS/s, with the divide-and-conquer cyclic-reduction
section solver (--alg ph: the PH solver). The other orders are reported under
"sweep", each timed with both solvers and with the library default (the
solver chosen per signal), and with the whole-cascade block-Toeplitz kernel
on the matrix cores ("toeplitz_*": its MFMA rate against the 157.3 TFLOP/s
dense FP32 MFMA peak); alu_roof_frac is against the unpacked FP32 rate
(78.6 TFLOP/s), which is what the per-section kernels are built for.

Timing: W untimed warm-up steps, then exactly K timed steps between
torch.cuda.synchronize() calls; two rotating input/output buffer pairs of
1 GiB each (beyond the 256 MB Infinity Cache). HIP events recorded on the
launch stream around every filter-kernel launch give the kernel's own average
duration for the roofline figure. "paper_protocol" times the same kernel the
paper's way (Sec. IV-F): 1000 warm-up launches, 20 batches of 200, the
20th-percentile batch mean beside the plain mean. "plateau" holds length
curves under that protocol (orders 2 and 16, 2^16..2^28 samples) and the
paper's plateau, the mean of the 2^24 and 2^25 points, for every order and
both section solvers (order 16 also with the default solver, which takes the
block-Toeplitz kernel from 2^25 samples, and with that kernel alone).

CPU legs (skipped with --no-cpu): "cpu_baseline" is the FP64 oracle on one
thread (one signal is one sequential recursion) over the whole headline
signal, median of 5; "cpu_baselines_multicore" runs the oracle on the host's
cores (at most 16 threads) over bounded samples of the batched, served and
differentiated workloads; "host" records nproc and the CPU model.

Beside the headline, on the same GPU (skipped with --quick):
* "batched": 4096 signals, lengths floor(2^U), U ~ U[10, 22], orders 2..16,
  random stable sections, random initial states, in one persistent launch
  captured in a HIP graph at the autotuned (L, N); GS/s over all samples (its
  parity at this size is a GPU test: tests/test_gpu_fullsize.py).
* "served": 1024 streams of orders 2..16, chunks of 4096..65536 samples,
  pushed by the library's native replay driver: first the saturated rate
  (100000 chunks queued at once), then Poisson arrivals at 0.1..1.2 times
  that rate, 100000 chunks per point; achieved GS/s and p50/p99 chunk
  latency (tile (256, 16), PH solver).
* "fwd_bwd": forward (keeping the section outputs) plus the adjoint, on one
  2^24-sample signal and on 256 signals of 2^16 samples, order 8, PH solver.
* "dtcr_bound": an upper bound for DTCR's gain on short signals: the tile
  with twice the lanes and half the samples per lane at the same group size
  (DTCR's extra waves without its per-section hand-off) against the base
  tile, 2^14..2^18 samples, orders 2 and 16, both solvers.

Prints one JSON line on stdout. `python bench.py --gpus N` with N > 1 exits:
this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E peak
METRIC = "GS/s & % HBM roof, orders 2-16; p50/p99 stream-chunk latency; fwd+bwd GS/s"
BYTES_PER_SAMPLE = 8            # 4 B FP32 in + 4 B FP32 out (Eq. (28))
# Algorithmic multiply/FMA operations per sample and section of each solver
# (2 flop each): DC-CR fold 5 + reduction 2 + back substitution 2; PH
# feed-forward 3 + recursion 2 + homogeneous correction 2 (Table III).
OPS_PER_SAMPLE_SECTION = {"dccr": 9, "ph": 7}
# The kernels are built without packed FP32 instructions, so their ALU roof is
# the unpacked rate: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz.
FP32_UNPACKED_PEAK_TFLOPS = 78.6
# Whole-cascade block-Toeplitz kernel: MFMA instructions (16x16x4 FP32, 2048
# flops each) per 1024 samples: 32 in the first sweep (Gam x, column scan), 56
# in the second (T x on the lower block triangle, O s), 1 for the tile scans;
# the same whatever the order (the state is padded to 16)
TOEP_MFMA_FLOPS_PER_SAMPLE = 89 * 2048 / 1024
FP32_MFMA_PEAK_TFLOPS = 157.3
FP32_PACKED_PEAK_TFLOPS = 157.3   # MI355X with packed FP32 (context only)
KERNEL_SOURCES = ("paper_2607_23763_amd/csrc/sos_fwd.hip", "paper_2607_23763_amd/csrc/sos_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sos_fwd_kernel_k1_2p28.json")


def kernel_sha() -> str:
    """Hash of the kernel sources' code: comments and blank space removed, so
    that a comment edit keeps counter data taken on the same code valid."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(torch, P, h, sos_d, xs, ys, steps, warmup):
    """Run warmup + steps whole steps (prepare + filter) rotating buffers.
    Returns (ms per step, mean filter-kernel ms from HIP events)."""
    nb = len(xs)
    for i in range(warmup):
        P.prepare(sos_d, handle=h)
        P.filter_prepared(xs[i % nb], ys[i % nb], handle=h)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        P.prepare(sos_d, handle=h)
        ev[i][0].record()
        P.filter_prepared(xs[i % nb], ys[i % nb], handle=h)
        ev[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = sum(a.elapsed_time(b) for a, b in ev) / steps
    return (t1 - t0) * 1e3 / steps, kern


def paper_protocol(torch, P, h, xs, ys, batches=20, per_batch=200, warmup=1000):
    """The paper's timing protocol (Sec. IV-F) for filter launches with the
    handle's prepared tables: `warmup` untimed launches, then `batches`
    batches of `per_batch` launches over the rotating buffers, each batch
    bracketed by HIP events on the launch stream. Returns the 20th-percentile
    batch mean and the plain mean (ms per launch), and the host time per
    launch call (us), which shows whether launches were issued faster than
    they ran."""
    import ctypes

    import numpy as np

    lib = P.lib()
    st = P._stream_ptr(xs[0].device)
    args = [(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.numel())
            for x, y in zip(xs, ys)]
    nb = len(args)
    f, hp = lib.sos_filter_prepared, h.ptr

    def launch(i):
        a = args[i % nb]
        rc = f(hp, a[0], a[1], a[2], None, None, st)
        if rc:
            raise RuntimeError("sos_filter_prepared returned %d" % rc)

    for i in range(warmup):
        launch(i)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(batches)]
    t0 = time.perf_counter()
    for b in range(batches):
        ev[b][0].record()
        for i in range(per_batch):
            launch(b * per_batch + i)
        ev[b][1].record()
    host = time.perf_counter() - t0
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(e) / per_batch for a, e in ev])
    return float(np.percentile(ms, 20)), float(ms.mean()), 1e6 * host / (batches * per_batch)


def length_curve(torch, P, h, sos_d, xs, ys, log2ns):
    """Kernel GS/s against the signal length under the paper's protocol:
    disjoint slices of the two 1 GiB buffer pairs rotate so that every cycle
    touches >= 512 MiB (beyond the 256 MB Infinity Cache). With no tile set,
    one sos_filter call per length prepares the tables at the shape sos_filter
    picks for that length."""
    n = xs[0].numel()
    pts = []
    for lg in log2ns:
        m = 1 << lg
        k = min(n // m, max(1, (1 << 29) // (8 * m)))
        sx = [xs[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
        sy = [ys[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
        P.sosfilt_(sx[0], sos_d, y=sy[0], handle=h)
        p20, mean, host_us = paper_protocol(torch, P, h, sx, sy)
        assert h.last_error() == P.SOS_OK
        pts.append({"log2n": lg, "kernel_GS_per_s": round(m / (p20 * 1e-3) / 1e9, 2),
                    "mean_GS_per_s": round(m / (mean * 1e-3) / 1e9, 2),
                    "ms_p20": round(p20, 5), "host_us_per_launch": round(host_us, 2)})
    return pts


def bench_dtcr_bound(torch, P, workloads, xs, ys, log):
    """What DTCR's extra waves could buy (Sec. IV-E): DTCR splits a group's
    two parity chains over two thread groups, doubling the waves per group at
    the same staging, and pays an LDS hand-off per section. The tile with
    twice the lanes and half the samples per lane at the same group size C
    has those waves and the half-length chains without the hand-off, so its
    gain bounds DTCR's. Short signals (2^14..2^18 samples), orders 2 and 16,
    both solvers, under the paper's protocol (200 warm-up launches, 20
    batches of 50)."""
    out = {}
    pairs = (((256, 32), (512, 16)), ((512, 32), (1024, 16)))
    for K in (1, 8):
        sos_d = torch.from_numpy(workloads.sweep_sections(K, "butter")).to(xs[0].device)
        for alg in ("dccr", "ph"):
            rows = []
            for base, wide in pairs:
                for lg in range(14, 19):
                    m = 1 << lg
                    k = min(xs[0].numel() // m, 64)
                    sx = [xs[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
                    sy = [ys[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
                    r = {"log2n": lg}
                    for name, tile in (("base", base), ("wide", wide)):
                        h = P.Handle(0, tile=tile, algorithm=alg)
                        P.sosfilt_(sx[0], sos_d, y=sy[0], handle=h)
                        p20, _, _ = paper_protocol(torch, P, h, sx, sy, batches=20, per_batch=50,
                                                   warmup=200)
                        assert h.last_error() == P.SOS_OK
                        h.close()
                        r[name] = {"tile_L_N": list(tile),
                                   "kernel_GS_per_s": round(m / (p20 * 1e-3) / 1e9, 2)}
                    r["wide_over_base"] = round(r["wide"]["kernel_GS_per_s"] /
                                                r["base"]["kernel_GS_per_s"], 3)
                    rows.append(r)
            out["order_%d_%s" % (2 * K, alg)] = rows
            log("dtcr bound", 2 * K, alg, [(r["log2n"], r["base"]["tile_L_N"], r["wide_over_base"])
                                            for r in rows])
    return out


def plateau_of(pts):
    """The paper's plateau of a length curve: the mean of its 2^24 and 2^25
    points (GS/s)."""
    v = [p["kernel_GS_per_s"] for p in pts if p["log2n"] in (24, 25)]
    return round(sum(v) / len(v), 2) if len(v) == 2 else None


def time_copy(torch, P, xs, ys, steps, warmup):
    for i in range(warmup):
        P.bench_copy(xs[i % 2], ys[i % 2])
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for i in range(steps):
        ev[i][0].record()
        P.bench_copy(xs[i % 2], ys[i % 2])
        ev[i][1].record()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in ev) / steps


def cpu_baseline(sos, x_host, reps=5):
    """The FP64 oracle (sequential, one thread) on the whole signal: GS/s and
    seconds, median of `reps` runs (the FP64 copy of the input is made before
    the timing; the oracle allocates its output in each run)."""
    import numpy as np

    import oracle

    xs = np.ascontiguousarray(x_host, dtype=np.float64)
    oracle.sosfilt(sos, xs[:1024])             # load / build outside the timing
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        oracle.sosfilt(sos, xs)
        ts.append(time.perf_counter() - t)
    ts.sort()
    return xs.size / ts[len(ts) // 2] / 1e9, ts[len(ts) // 2]


def host_info():
    """Host cores and CPU model, and the worker threads the CPU legs use (the
    cores this process may run on, at most 16)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "available": avail, "cpu_model": model,
            "threads": max(1, min(16, avail))}


def _median_time(fn, reps):
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    ts.sort()
    return ts[len(ts) // 2]


def cpu_baselines_multi(workloads, np, threads, log):
    """The FP64 oracle on the host's cores for the batched, served and
    differentiated workloads (bounded samples of each; median of 3 runs)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    out = {}
    g = np.random.default_rng(11)
    # uneven batch: the first signals of the benchmarked batch, >= 2^27 samples
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=4096, seed=3)
    S = int(np.searchsorted(sig_off, 1 << 27)) or 1
    sec = int(np.sum(Ks[:S]))
    x = g.standard_normal(int(sig_off[S]))
    run = lambda: oracle.sosfilt_batched(Ks[:S], rows[:sec], sig_off[:S + 1], x, zi[:sec],
                                         nthreads=threads)
    oracle.sosfilt_batched(Ks[:1], rows[:int(Ks[0])], sig_off[:2], x, zi[:int(Ks[0])])
    t = _median_time(run, 3)
    out["batched"] = {"value": round(x.size / t / 1e9, 4), "unit": "GS/s", "cores": threads,
                      "kind": "oracle", "seconds": round(t, 3),
                      "sample": "the first %d of the 4096 signals of the uneven batch (%d "
                                "samples), oracle_sosfilt_batched with %d threads (signals "
                                "dealt round-robin)" % (S, x.size, threads)}
    del x
    # serving: the first 5000 chunks of the trace; one stream's chunks in
    # arrival order, concatenated, give the outputs of chunk-by-chunk
    # filtering with the state carried (streams run in parallel)
    Ks_s, secs, ids, lens, offs, arrival = workloads.serving_trace(S=1024, R=20000,
                                                                   rate_chunks_per_s=1e9, seed=4)
    R = 5000
    per = np.bincount(ids[:R], minlength=len(Ks_s)).astype(np.int64)
    lens_s = np.zeros(len(Ks_s), np.int64)
    np.add.at(lens_s, ids[:R], lens[:R])
    keep = np.nonzero(per)[0]
    so = np.r_[0, np.cumsum(lens_s[keep])].astype(np.int64)
    rws = np.concatenate([secs[s] for s in keep])
    kk = np.array([secs[s].shape[0] for s in keep], np.int32)
    x = g.standard_normal(int(so[-1]))
    run = lambda: oracle.sosfilt_batched(kk, rws, so, x, None, nthreads=threads)
    t = _median_time(run, 3)
    out["served"] = {"value": round(x.size / t / 1e9, 4), "unit": "GS/s", "cores": threads,
                     "kind": "oracle", "seconds": round(t, 3),
                     "sample": "the first %d of the 20000 chunks (%d samples, %d streams), all "
                               "queued at once; each stream's chunks concatenated in arrival "
                               "order, streams on %d threads" % (R, x.size, keep.size, threads)}
    del x
    # differentiation: 256 signals of 2^16 samples, order-8 Butterworth
    sos = workloads.sweep_sections(4, "butter")
    B, m = 256, 1 << 16
    x = g.standard_normal(B * m)
    gy = g.standard_normal(B * m)
    K = sos.shape[0]
    rb = np.tile(sos, (B, 1))
    sob = np.arange(B + 1, dtype=np.int64) * m
    t_f = _median_time(lambda: oracle.sosfilt_batched(np.full(B, K, np.int32), rb, sob, x, None,
                                                      nthreads=threads), 3)

    def vjp_all():
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda i: oracle.sosfilt_vjp(sos, x[i * m:(i + 1) * m], None,
                                                     gy[i * m:(i + 1) * m], None), range(B)))

    t_b = _median_time(vjp_all, 3)
    x1 = g.standard_normal(1 << 24)
    g1 = g.standard_normal(1 << 24)
    t1 = _median_time(lambda: (oracle.sosfilt(sos, x1), oracle.sosfilt_vjp(sos, x1, None, g1)), 3)
    out["fwd_bwd"] = {"value": round(B * m / (t_f + t_b) / 1e9, 4), "unit": "GS/s",
                      "cores": threads, "kind": "oracle",
                      "fwd_GS_per_s": round(B * m / t_f / 1e9, 4),
                      "vjp_GS_per_s": round(B * m / t_b / 1e9, 4),
                      "one_signal_2p24_fwd_bwd_GS_per_s": round((1 << 24) / t1 / 1e9, 4),
                      "sample": "the whole 256 x 2^16 batch, order-8 Butterworth: "
                                "oracle_sosfilt_batched (forward) and one oracle_sosfilt_vjp "
                                "per signal on %d threads; one 2^24-sample signal forward + "
                                "VJP on one thread" % threads}
    log("cpu baselines", out)
    return out


def cpu_wavefront_rate(sos, x_host, n_sample, reps=3, node="serial"):
    """The paper's multi-core CPU method (wavefront over groups and sections,
    Sec. III-A, with serial or multi-block node kernels) on the first
    n_sample samples: GS/s, seconds, threads."""
    import numpy as np

    import cpu_wavefront

    xs = np.ascontiguousarray(x_host[:n_sample], dtype=np.float32)
    ys = np.empty_like(xs)
    threads = cpu_wavefront.default_threads()
    cpu_wavefront.sosfilt(sos, xs[:4096], threads=threads, node=node)   # load outside the timing
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        cpu_wavefront.sosfilt(sos, xs, threads=threads, out=ys, node=node)
        ts.append(time.perf_counter() - t)
    ts.sort()
    return n_sample / ts[len(ts) // 2] / 1e9, ts[len(ts) // 2], threads


def traffic_bytes(n):
    """HBM bytes per filter launch from the committed rocprofv3 counter runs,
    scaled by the same counters on the copy kernel; None if the counters were
    taken on a different kernel source or workload size."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha() or int(t.get("n", -1)) != n:
        return None
    fetch = t["fetch_kib"] * 1024.0 * t["copy_read_bytes"] / (t["copy_fetch_kib"] * 1024.0)
    write = t["write_kib"] * 1024.0 * t["copy_write_bytes"] / (t["copy_write_kib"] * 1024.0)
    return fetch + write


def bench_batched(torch, P, workloads, np, log):
    """Uneven batch (4096 signals) in one graph-captured persistent launch."""
    dev = torch.device("cuda", 0)
    Ks, rows, sig_off, zi = workloads.uneven_batch(B=4096, seed=3)
    total = int(sig_off[-1])
    gen = torch.Generator(device=dev).manual_seed(3)
    x = torch.randn(total, generator=gen, device=dev, dtype=torch.float32)
    y = torch.empty_like(x)
    Kd = torch.from_numpy(Ks.astype(np.int32)).to(dev)
    so = torch.from_numpy(sig_off.astype(np.int64)).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    zi_d = torch.from_numpy(zi).to(dev)
    zf = torch.empty_like(zi_d)

    def graph_ms(h):
        g = P.BatchGraph(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=h)
        for _ in range(2):
            g.launch()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        reps = 5
        ev[0].record()
        for _ in range(reps):
            g.launch()
        ev[1].record()
        torch.cuda.synchronize()
        assert g.last_error() == P.SOS_OK
        g.close()
        return ev[0].elapsed_time(ev[1]) / reps

    # the tuner as shipped: the cost model ranks every (tile, solver) pair and
    # only the best 6 are timed; then every pair the budgets admit, timed
    # (SOS_TUNE_EXHAUSTIVE), to check the ranking
    h = P.Handle(0)
    t0 = time.perf_counter()
    (L, N), tune_ms, _, _ = P.tune_batched(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=h,
                                           reps=2)
    tune_s = time.perf_counter() - t0
    log("batched: tuned tile", (L, N), h.algorithm(), "%.3f ms (%.2f s)" % (tune_ms, tune_s))
    hx = P.Handle(0)
    os.environ["SOS_TUNE_EXHAUSTIVE"] = "1"
    try:
        t0 = time.perf_counter()
        (Lx, Nx), _, _, _ = P.tune_batched(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=hx,
                                           reps=2)
        tune_xs = time.perf_counter() - t0
    finally:
        del os.environ["SOS_TUNE_EXHAUSTIVE"]
    ms = graph_ms(h)
    alg_x = hx.algorithm()
    msx = graph_ms(hx) if (Lx, Nx, alg_x) != (L, N, h.algorithm()) else ms
    log("batched: exhaustive tile", (Lx, Nx), alg_x, "%.3f ms vs %.3f ms" % (msx, ms))
    hx.close()
    gs = total / (ms * 1e-3) / 1e9
    out = {"workload": "4096 signals, lengths floor(2^U) U~U[10,22], K~U{1..8} random stable "
                       "SOS, zi~N(0,0.1)", "B": 4096, "samples": total,
           "tile_L_N": [L, N], "section_solver": h.algorithm(), "ms": round(ms, 4),
           "GS_per_s": round(gs, 2),
           "hbm_roof_frac": round(gs * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
           "graph": True,
           "tuner": {"timed_pairs": 6, "seconds": round(tune_s, 2),
                     "exhaustive_tile_L_N": [Lx, Nx], "exhaustive_solver": alg_x,
                     "exhaustive_ms": round(msx, 4), "exhaustive_seconds": round(tune_xs, 2),
                     "pick_vs_exhaustive": round(ms / msx, 4)}}
    log("batched", out)
    del x, y
    torch.cuda.empty_cache()
    return out


SERVED_LOADS = (0.1, 0.25, 0.5, 0.75, 0.9, 1.0, 1.2)


def bench_served(torch, P, workloads, np, log, loads=SERVED_LOADS, R=100000, tile=(256, 16),
                 alg="ph", rates=None):
    """1024 streams. First the saturated rate: all R chunks queued at t = 0
    (after a short warm-up replay); then Poisson arrivals at each fraction of
    that rate (`loads`), R chunks per point; or, with `rates`, at those
    aggregate rates in chunks/s (0 = all at t = 0)."""
    dev = torch.device("cuda", 0)
    gen = torch.Generator(device=dev).manual_seed(4)
    buf = {}

    def run(rate, RR):
        Ks, secs, ids, lens, offs, arrival = workloads.serving_trace(
            S=1024, R=RR, rate_chunks_per_s=rate if rate > 0 else 1e9, seed=4)
        if rate <= 0:
            arrival = np.zeros_like(arrival)
        total = int(lens.sum())
        if buf.get("n", 0) < total:
            buf.clear()
            buf["x"] = torch.randn(total, generator=gen, device=dev, dtype=torch.float32)
            buf["y"] = torch.empty_like(buf["x"])
            buf["n"] = total
        srv = P.Server(handle=P.Handle(0, tile=tile, algorithm=alg), max_slots=1024,
                       budget=1 << 30)
        sid = np.array([srv.open(secs[s]) for s in range(len(Ks))], dtype=np.int64)
        lat, wall = srv.replay(sid[ids], offs, lens, arrival, buf["x"], buf["y"])
        srv.close()
        return total, wall, lat, float(lens.mean())

    def point(rate, RR, label, load=None):
        total, wall, lat, mean_len = run(rate, RR)
        r = {"rate_chunks_per_s": round(rate, 1) if rate > 0 else "all at t=0",
             "offered_GS_per_s": round(rate * mean_len / 1e9, 3) if rate > 0 else None,
             "GS_per_s": round(total / wall / 1e9, 3),
             "p50_us": round(1e6 * float(np.percentile(lat, 50)), 1),
             "p99_us": round(1e6 * float(np.percentile(lat, 99)), 1), "chunks": RR}
        if load is not None:
            r["load"] = load
        log("served", label, r)
        return r, RR / wall

    run(0.0, 2000)                                       # warm-up
    res = []
    if rates is not None:
        for rate in rates:
            res.append(point(rate, R, "rate")[0])
        capacity = None
    else:
        sat, cap_cps = point(0.0, R, "saturated")
        capacity = {"GS_per_s": sat["GS_per_s"], "chunks_per_s": round(cap_cps, 1)}
        res.append(sat)
        for f in loads:
            res.append(point(f * cap_cps, R, "load %.2f" % f, load=f)[0])
    buf.clear()
    torch.cuda.empty_cache()
    return {"workload": "1024 streams, K~U{1..8} random stable SOS, chunks floor(2^U) samples "
                        "U~U[12,16], Poisson arrivals at fractions of the saturated rate, state "
                        "on device, FIFO per stream, two step lanes",
            "tile_L_N": list(tile), "section_solver": alg, "saturated": capacity,
            "points": res}


def bench_fwd_bwd(torch, P, workloads, np, log):
    """Forward with saved section outputs plus the adjoint, order 8 Butterworth."""
    dev = torch.device("cuda", 0)
    sos = torch.from_numpy(workloads.sweep_sections(4, "butter")).to(dev)
    out = {}
    gen = torch.Generator(device=dev).manual_seed(5)
    # one long signal
    n = 1 << 24
    x = torch.randn(n, generator=gen, device=dev)
    gy = torch.randn(n, generator=gen, device=dev)
    h = P.Handle(0, algorithm="ph")
    for _ in range(2):
        yv, zf, saved = P.sosfilt_train(x, sos, None, handle=h)
        P.sosfilt_vjp(sos, x, yv, saved, gy, None, handle=h)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = 5
    tf = tb = 0.0
    for _ in range(reps):
        ev[0].record()
        yv, zf, saved = P.sosfilt_train(x, sos, None, handle=h)
        ev[1].record()
        P.sosfilt_vjp(sos, x, yv, saved, gy, None, handle=h)
        ev[2].record()
        torch.cuda.synchronize()
        tf += ev[0].elapsed_time(ev[1])
        tb += ev[1].elapsed_time(ev[2])
    assert h.last_error() == P.SOS_OK
    tf, tb = tf / reps, tb / reps
    out["section_solver"] = "ph"
    out["one_signal_2p24"] = {"fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                              "fwd_bwd_GS_per_s": round(n / ((tf + tb) * 1e-3) / 1e9, 2),
                              "fwd_GS_per_s": round(n / (tf * 1e-3) / 1e9, 2)}
    # 256 signals of 2^16 sharing the cascade: batched forward (keeping the
    # section outputs) + one batched adjoint launch for the whole batch
    B, m = 256, 1 << 16
    xb = torch.randn(B * m, generator=gen, device=dev)
    gb = torch.randn(B * m, generator=gen, device=dev)
    K = sos.shape[0]
    rows = sos.repeat(B, 1).contiguous()
    Kd = torch.full((B,), K, dtype=torch.int32, device=dev)
    so = torch.arange(B + 1, dtype=torch.int64, device=dev) * m
    for _ in range(2):
        yv, zf, saved = P.sosfilt_train_batched(xb, rows, Kd, so, handle=h)
        P.sosfilt_vjp_batched(rows, Kd, so, xb, yv, saved, gb, None, handle=h)
    torch.cuda.synchronize()
    tf = tb = 0.0
    for _ in range(reps):
        ev[0].record()
        yv, zf, saved = P.sosfilt_train_batched(xb, rows, Kd, so, handle=h)
        ev[1].record()
        P.sosfilt_vjp_batched(rows, Kd, so, xb, yv, saved, gb, None, handle=h)
        ev[2].record()
        torch.cuda.synchronize()
        tf += ev[0].elapsed_time(ev[1])
        tb += ev[1].elapsed_time(ev[2])
    assert h.last_error() == P.SOS_OK
    tf, tb = tf / reps, tb / reps
    out["batch_256x2p16"] = {"fwd_ms": round(tf, 4), "bwd_ms": round(tb, 4),
                             "fwd_bwd_GS_per_s": round(B * m / ((tf + tb) * 1e-3) / 1e9, 2),
                             "note": "one batched forward and one batched adjoint launch"}
    log("fwd_bwd", out)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--tile", default="", help="group shape 'L,N' (lanes per group, samples per lane); default: library default")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-k", type=int, default=0, help="profile helper: only this K, Butterworth")
    ap.add_argument("--quick", action="store_true", help="headline and sweep only")
    ap.add_argument("--only-fwd-bwd", action="store_true",
                    help="profile helper: only the forward + adjoint leg, printed as its own JSON")
    ap.add_argument("--only-served", default="",
                    help="profile helper: only the serving leg, as its own JSON: 'loads' (the "
                         "default sweep) or comma-separated aggregate rates in chunks/s "
                         "(0 = all chunks at t=0)")
    ap.add_argument("--served-tile", default="256,16",
                    help="profile helper: the server's tile with --only-served")
    ap.add_argument("--only-batched", action="store_true",
                    help="profile helper: only the uneven-batch leg, printed as its own JSON")
    ap.add_argument("--alg", default="dccr", choices=("dccr", "ph", "toeplitz"),
                    help="section solver of the headline (the sweep times all); "
                         "toeplitz: with --only-k only (profile helper)")
    args = ap.parse_args()
    if args.alg == "toeplitz" and not args.only_k:
        ap.error("--alg toeplitz is a profile helper: give --only-k")

    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU split is a design note only)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_23763_amd as P
    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    P.lib()
    if args.only_fwd_bwd:
        print(json.dumps({"fwd_bwd": bench_fwd_bwd(torch, P, workloads, np, log)}), flush=True)
        return
    if args.only_served:
        st = tuple(int(v) for v in args.served_tile.split(","))
        rates = None if args.only_served == "loads" else \
            tuple(float(v) for v in args.only_served.split(","))
        print(json.dumps({"served": bench_served(torch, P, workloads, np, log, rates=rates,
                                                 tile=st)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": bench_batched(torch, P, workloads, np, log)}), flush=True)
        return
    dev = torch.device("cuda", 0)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    h = P.Handle(0, tile=tile, algorithm=args.alg)
    L, N = h.tile()
    n = 1 << args.log2n
    log("generating %d samples" % n)
    x_host = workloads.signal(n, seed=2)
    x0 = torch.from_numpy(x_host).to(dev)
    xs = [x0, x0.clone()]
    ys = [torch.empty_like(x0), torch.empty_like(x0)]
    torch.cuda.synchronize()

    def gss(ms):
        return n / (ms * 1e-3) / 1e9

    # --- headline: K = 1 Butterworth
    K1 = args.only_k or 1
    sos1 = workloads.sweep_sections(K1, "butter")
    sos1_d = torch.from_numpy(sos1).to(dev)
    ms_step, ms_kern = time_steps(torch, P, h, sos1_d, xs, ys, args.steps, args.warmup)
    assert h.last_error() == P.SOS_OK
    log("K=%d step %.4f ms (%.1f GS/s), kernel %.4f ms" % (K1, ms_step, gss(ms_step), ms_kern))
    # the same kernel under the paper's protocol (Sec. IV-F)
    paper_stat = None
    if not args.quick and not args.only_k:
        P.prepare(sos1_d, handle=h)
        p20, pmean, host_us = paper_protocol(torch, P, h, xs, ys)
        assert h.last_error() == P.SOS_OK
        paper_stat = {"protocol": "1000 warm-up launches, 20 batches of 200 launches, "
                                  "20th-percentile batch mean (Sec. IV-F)",
                      "kernel_ms_p20": round(p20, 4), "kernel_GS_per_s": round(gss(p20), 2),
                      "kernel_ms_mean": round(pmean, 4), "mean_GS_per_s": round(gss(pmean), 2),
                      "hbm_roof_frac": round(gss(p20) * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
                      "host_us_per_launch": round(host_us, 2)}
        log("paper protocol", paper_stat)

    result_sweep = {}
    if not args.no_sweep and not args.only_k:
        other = "ph" if args.alg == "dccr" else "dccr"
        h2 = P.Handle(0, tile=tile, algorithm=other)
        h3 = P.Handle(0, tile=tile)         # the library default: per-signal choice
        h4 = P.Handle(0, tile=tile, algorithm="toeplitz")   # whole-cascade MFMA form
        for kind in ("butter", "random"):
            result_sweep[kind] = {}
            for K in (1, 2, 4, 8):
                sos_d = torch.from_numpy(workloads.sweep_sections(K, kind)).to(dev)
                ms, mk = time_steps(torch, P, h, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h.last_error() == P.SOS_OK
                ms2, mk2 = time_steps(torch, P, h2, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h2.last_error() == P.SOS_OK
                ms3, mk3 = time_steps(torch, P, h3, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h3.last_error() == P.SOS_OK
                ms4, mk4 = time_steps(torch, P, h4, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h4.last_error() == P.SOS_OK
                mf = gss(mk4) * TOEP_MFMA_FLOPS_PER_SAMPLE / 1e3
                tf = gss(mk) * 2 * OPS_PER_SAMPLE_SECTION[args.alg] * K / 1e3
                tf2 = gss(mk2) * 2 * OPS_PER_SAMPLE_SECTION[other] * K / 1e3
                result_sweep[kind][str(K)] = {
                    "order": 2 * K, "GS_per_s": round(gss(ms), 2),
                    "kernel_GS_per_s": round(gss(mk), 2),
                    "hbm_roof_frac": round(gss(mk) * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
                    "alu_TFLOPs": round(tf, 2),
                    "alu_roof_frac": round(tf / FP32_UNPACKED_PEAK_TFLOPS, 4),
                    "alu_packed_roof_frac": round(tf / FP32_PACKED_PEAK_TFLOPS, 4),
                    other + "_GS_per_s": round(gss(ms2), 2),
                    other + "_kernel_GS_per_s": round(gss(mk2), 2),
                    other + "_alu_roof_frac": round(tf2 / FP32_UNPACKED_PEAK_TFLOPS, 4),
                    "auto_GS_per_s": round(gss(ms3), 2),
                    "auto_kernel_GS_per_s": round(gss(mk3), 2),
                    "toeplitz_GS_per_s": round(gss(ms4), 2),
                    "toeplitz_kernel_GS_per_s": round(gss(mk4), 2),
                    "toeplitz_mfma_TFLOPs": round(mf, 2),
                    "toeplitz_mfma_roof_frac": round(mf / FP32_MFMA_PEAK_TFLOPS, 4)}
                log(kind, K, result_sweep[kind][str(K)])
        h2.close()
        h3.close()
        h4.close()

    # length curves and the paper's plateau (mean of the 2^24 and 2^25
    # points), Butterworth, under the paper's protocol: orders 2 and 16 over
    # 2^16..2^28 samples with the headline solver, the plateau points of
    # every order with both solvers
    plateau = {}
    if not args.no_sweep and not args.only_k and args.log2n == 28 and not args.quick:
        hp = P.Handle(0, tile=tile, algorithm="ph" if args.alg == "dccr" else "dccr")
        for K in (1, 2, 4, 8):
            sos_d = torch.from_numpy(workloads.sweep_sections(K, "butter")).to(dev)
            lgs = range(16, 29) if K in (1, 8) else (24, 25)
            pts = length_curve(torch, P, h, sos_d, xs, ys, lgs)
            pts2 = length_curve(torch, P, hp, sos_d, xs, ys, (24, 25))
            plateau["order_%d" % (2 * K)] = {
                "plateau_GS_per_s": plateau_of(pts),
                "plateau_hbm_roof_frac": round(plateau_of(pts) * BYTES_PER_SAMPLE / HBM_PEAK_GBS,
                                               4),
                hp.algorithm() + "_plateau_GS_per_s": plateau_of(pts2),
                "curve": pts}
            if K == 8:
                # order 16: the default (automatic) solver, which takes the
                # block-Toeplitz kernel from 2^25 samples, and that kernel
                # alone
                for alg in ("auto", "toeplitz"):
                    ha = P.Handle(0, tile=tile, algorithm=alg)
                    pa = length_curve(torch, P, ha, sos_d, xs, ys, (24, 25))
                    ha.close()
                    plateau["order_16"][alg + "_plateau_GS_per_s"] = plateau_of(pa)
                    plateau["order_16"][alg + "_points"] = pa
            log("plateau", 2 * K, plateau["order_%d" % (2 * K)])
        hp.close()
        extra_dtcr = bench_dtcr_bound(torch, P, workloads, xs, ys, log)
    else:
        extra_dtcr = None

    copy_ms = time_copy(torch, P, xs, ys, 20, 3)
    copy_gbs = n * BYTES_PER_SAMPLE / (copy_ms * 1e-3) / 1e9
    log("copy %.4f ms = %.0f GB/s" % (copy_ms, copy_gbs))

    achieved_gbs = n * BYTES_PER_SAMPLE / (ms_kern * 1e-3) / 1e9
    # the committed counter runs are of the order-2 DC-CR forward kernel; the
    # profile helper's other cascades and solvers report no traffic
    headline_kernel = K1 == 1 and args.alg == "dccr"
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic_bytes(n) if headline_kernel else None,
                "kernel": "sos_toep_kernel" if args.alg == "toeplitz" else "sos_fwd_kernel",
                "kernel_ms": round(ms_kern, 4),
                "copy_roof_GBs": round(copy_gbs, 1),
                "frac_of_copy_roof": round(achieved_gbs / copy_gbs, 4)}

    extra = {}
    if not args.quick and not args.only_k:
        del xs, ys, x0
        torch.cuda.empty_cache()
        extra["batched"] = bench_batched(torch, P, workloads, np, log)
        extra["served"] = bench_served(torch, P, workloads, np, log)
        extra["fwd_bwd"] = bench_fwd_bwd(torch, P, workloads, np, log)

    cpu = None
    cpu_extra = None
    cpu_multi = None
    host = host_info()
    if not args.no_cpu:
        v, secs = cpu_baseline(sos1, x_host)
        cpu = {"value": round(v, 4), "unit": "GS/s", "cores": 1, "kind": "oracle",
               "sample": "FP64 sequential oracle, one thread (one signal is one sequential "
                         "recursion), the whole 2^%d-sample K=%d Butterworth signal, median of "
                         "5 runs (%.2f s each)" % (args.log2n, K1, secs),
               "nproc": host["nproc"], "cpu_model": host["cpu_model"]}
        log("cpu", cpu)
        if not args.quick and not args.only_k:
            cpu_multi = cpu_baselines_multi(workloads, np, host["threads"], log)
        # the paper's multi-core CPU method, beside the oracle (not the baseline)
        wf = {}
        for node in ("serial", "multiblock"):
            for K in (K1, 8):
                v, secs, thr = cpu_wavefront_rate(workloads.sweep_sections(K, "butter"), x_host,
                                                  min(n, 1 << 26), node=node)
                wf["%s_order_%d" % (node, 2 * K)] = {"value": round(v, 4), "unit": "GS/s",
                                                    "threads": thr, "seconds": round(secs, 3)}
        cpu_extra = {"kind": "wavefront over groups of 2^16 samples and sections, FP32, "
                             "pthreads (Sec. III-A); nodes: the serial filter, or the "
                             "multi-block node kernel (32 lanes x 64 samples per block, 8-wide "
                             "AVX2 vectors, PH per section); first 2^26 samples, median of 3",
                     **wf}
        log("cpu wavefront", cpu_extra)

    out = {
        "metric": METRIC,
        "value": round(gss(ms_step), 2),
        "unit": "GS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one FP32 signal of 2^%d N(0,1) samples, order-%d Butterworth "
                               "low-pass at 0.2*Nyquist (K=%d SOS), zi=0" % (args.log2n, 2 * K1, K1),
                   "n": n, "K": K1, "lanes_per_group_L": L, "samples_per_lane_N": N,
                   "group_C": L * N, "section_solver": args.alg},
        "hbm_roof_frac_step": round(gss(ms_step) * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baselines_multicore": cpu_multi,
        "host": host,
        "cpu_wavefront": cpu_extra,
        "paper_protocol": paper_stat,
        "dtcr_bound": extra_dtcr,
        "sweep": result_sweep,
        "plateau": plateau,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
