#!/usr/bin/env python3
"""Throughput benchmark of the single-kernel multi-block cascade filter on one MI355X.

Workload (the headline configuration): one FP32 signal of 2^28 i.i.d. N(0,1)
samples, zero initial state, cascades of K = 1, 2, 4, 8 sections (orders 2-16),
Butterworth low-pass at 0.2*Nyquist and random stable sections. The JSON
`value` is the order-2 (K = 1) Butterworth case: samples per second of one
whole step (coefficient preparation + filter kernel) with input and output
resident in HBM, in GS/s, with the divide-and-conquer cyclic-reduction
section solver (--alg ph: the PH solver). The other orders are reported under
"sweep", each timed with both solvers; "plateau" gives the kernel rate against
the signal length, 2^24..2^28 samples, at orders 2 and 16.

Timing: W untimed warm-up steps, then exactly K timed steps between
torch.cuda.synchronize() calls; two rotating input/output buffer pairs of
1 GiB each (beyond the 256 MB Infinity Cache). HIP events recorded on the
launch stream around every filter-kernel launch give the kernel's own average
duration for the roofline figure.

Beside the headline, on the same GPU (skipped with --quick):
* "batched": 4096 signals, lengths floor(2^U), U ~ U[10, 22], orders 2..16,
  random stable sections, random initial states, in one persistent launch
  captured in a HIP graph at the autotuned (L, N); GS/s over all samples (its
  parity at this size is a GPU test: tests/test_gpu_batched.py).
* "served": 1024 streams of orders 2..16, chunks of 4096..65536 samples
  arriving as a Poisson process at swept aggregate rates, pushed by the
  library's native replay driver; achieved GS/s and p50/p99 chunk latency
  (tile (256, 16), PH solver: 10-13 % lower latency than DC-CR there).
* "fwd_bwd": forward (keeping the section outputs) plus the adjoint, on one
  2^24-sample signal and on 256 signals of 2^16 samples, order 8, PH solver.
* "toeplitz_mfma_bound": a lower bound for a block-Toeplitz (matrix-core)
  form of the whole cascade, not part of the filter: the FP32 library GEMM
  that maps every 64-sample chunk of a 2^28-sample signal through a 64 x 64
  lower-triangular operator (the zero-state response), and through 80 x 64
  (plus the 16 terminal states of an order-16 cascade), beside the order-16
  filter kernel.

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
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X, packed FP32
FP32_UNPACKED_PEAK_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
KERNEL_SOURCES = ("paper_2607_23763_amd/csrc/sos_fwd.hip", "paper_2607_23763_amd/csrc/sos_device.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sos_fwd_kernel_k1_2p28.json")


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
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


def bench_toeplitz_bound(torch, n, order16_kernel_gss, log):
    """Chunk-by-operator products of a whole block-Toeplitz cascade form, as
    FP32 library GEMMs (matrix cores), timed with HIP events: a lower bound
    for that design's zero-state stage, with nothing fused."""
    prev = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    g = torch.Generator(device="cuda").manual_seed(7)
    x = [torch.randn(n, device="cuda", generator=g) for _ in range(2)]
    out = {"chunk": 64, "n": n, "order16_filter_kernel_GS_per_s": order16_kernel_gss}
    for rows in (64, 80):
        op = torch.randn(rows, 64, device="cuda", generator=g)
        if rows == 64:
            op = op.tril()
        opt = op.t().contiguous()
        ys = [torch.empty(n // 64, rows, device="cuda") for _ in range(2)]
        xv = [v.view(-1, 64) for v in x]
        for i in range(5):
            torch.mm(xv[i % 2], opt, out=ys[i % 2])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(20):
            torch.mm(xv[i % 2], opt, out=ys[i % 2])
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        out["rows_%d" % rows] = {"ms": round(ms, 4), "GS_per_s": round(n / (ms * 1e-3) / 1e9, 1),
                                 "TFLOP_per_s": round(2.0 * n * rows / (ms * 1e-3) / 1e12, 1)}
        del ys
    torch.backends.cuda.matmul.allow_tf32 = prev
    del x
    torch.cuda.empty_cache()
    log("toeplitz_mfma_bound", out)
    return out


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


def cpu_baseline(sos, x_host, n_sample, reps=3):
    """The FP64 oracle (sequential, one thread) on the first n_sample samples."""
    import numpy as np

    import oracle

    xs = np.ascontiguousarray(x_host[:n_sample], dtype=np.float64)
    oracle.sosfilt(sos, xs[:1024])             # load / build outside the timing
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        oracle.sosfilt(sos, xs)
        ts.append(time.perf_counter() - t)
    ts.sort()
    return n_sample / ts[len(ts) // 2] / 1e9, ts[len(ts) // 2]


def cpu_wavefront_rate(sos, x_host, n_sample, reps=3):
    """The paper's multi-core CPU method (wavefront over groups and sections,
    Sec. III-A) on the first n_sample samples: GS/s, seconds, threads."""
    import numpy as np

    import cpu_wavefront

    xs = np.ascontiguousarray(x_host[:n_sample], dtype=np.float32)
    ys = np.empty_like(xs)
    threads = cpu_wavefront.default_threads()
    cpu_wavefront.sosfilt(sos, xs[:4096], threads=threads)     # load outside the timing
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        cpu_wavefront.sosfilt(sos, xs, threads=threads, out=ys)
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
    h = P.Handle(0)
    (L, N), tune_ms, _, _ = P.tune_batched(x, rows_d, Kd, so, zi=zi_d, y=y, zf=zf, handle=h,
                                           reps=2)
    log("batched: tuned tile", (L, N), h.algorithm(), "%.3f ms" % tune_ms)
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
    ms = ev[0].elapsed_time(ev[1]) / reps
    gs = total / (ms * 1e-3) / 1e9
    out = {"workload": "4096 signals, lengths floor(2^U) U~U[10,22], K~U{1..8} random stable "
                       "SOS, zi~N(0,0.1)", "B": 4096, "samples": total,
           "tile_L_N": [L, N], "section_solver": h.algorithm(), "ms": round(ms, 4),
           "GS_per_s": round(gs, 2),
           "hbm_roof_frac": round(gs * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
           "graph": True}
    log("batched", out)
    g.close()
    del x, y
    torch.cuda.empty_cache()
    return out


def bench_served(torch, P, workloads, np, log, rates=(5e4, 1e5, 2e5, 4e5, 8e5, 0.0), R=20000):
    """1024 streams, Poisson chunk arrivals at each aggregate rate (0 = all at once)."""
    dev = torch.device("cuda", 0)
    res = []
    for rate in rates:
        Ks, secs, ids, lens, offs, arrival = workloads.serving_trace(
            S=1024, R=R, rate_chunks_per_s=rate if rate > 0 else 1e9, seed=4)
        if rate <= 0:
            arrival = np.zeros_like(arrival)
        total = int(lens.sum())
        gen = torch.Generator(device=dev).manual_seed(4)
        x = torch.randn(total, generator=gen, device=dev, dtype=torch.float32)
        y = torch.empty_like(x)
        srv = P.Server(handle=P.Handle(0, tile=(256, 16), algorithm="ph"), max_slots=1024,
                       budget=1 << 30)
        sid = np.array([srv.open(secs[s]) for s in range(len(Ks))], dtype=np.int64)
        lat, wall = srv.replay(sid[ids], offs, lens, arrival, x, y)
        srv.close()
        gs = total / wall / 1e9
        offered = rate * float(lens.mean()) / 1e9 if rate > 0 else None
        r = {"rate_chunks_per_s": rate if rate > 0 else "all at t=0",
             "offered_GS_per_s": None if offered is None else round(offered, 3),
             "GS_per_s": round(gs, 3), "p50_us": round(1e6 * float(np.percentile(lat, 50)), 1),
             "p99_us": round(1e6 * float(np.percentile(lat, 99)), 1), "chunks": R}
        log("served", r)
        res.append(r)
        del x, y
    torch.cuda.empty_cache()
    return {"workload": "1024 streams, K~U{1..8} random stable SOS, chunks floor(2^U) samples "
                        "U~U[12,16], Poisson arrivals, state on device, FIFO per stream",
            "tile_L_N": [256, 16], "section_solver": "ph", "points": res}


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
    ap.add_argument("--only-batched", action="store_true",
                    help="profile helper: only the uneven-batch leg, printed as its own JSON")
    ap.add_argument("--alg", default="dccr", choices=("dccr", "ph"),
                    help="section solver of the headline (the sweep times both)")
    args = ap.parse_args()

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

    result_sweep = {}
    if not args.no_sweep and not args.only_k:
        other = "ph" if args.alg == "dccr" else "dccr"
        h2 = P.Handle(0, tile=tile, algorithm=other)
        for kind in ("butter", "random"):
            result_sweep[kind] = {}
            for K in (1, 2, 4, 8):
                sos_d = torch.from_numpy(workloads.sweep_sections(K, kind)).to(dev)
                ms, mk = time_steps(torch, P, h, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h.last_error() == P.SOS_OK
                ms2, mk2 = time_steps(torch, P, h2, sos_d, xs, ys, max(10, args.steps // 2), 3)
                assert h2.last_error() == P.SOS_OK
                tf = gss(mk) * 2 * OPS_PER_SAMPLE_SECTION[args.alg] * K / 1e3
                tf2 = gss(mk2) * 2 * OPS_PER_SAMPLE_SECTION[other] * K / 1e3
                result_sweep[kind][str(K)] = {
                    "order": 2 * K, "GS_per_s": round(gss(ms), 2),
                    "kernel_GS_per_s": round(gss(mk), 2),
                    "hbm_roof_frac": round(gss(mk) * BYTES_PER_SAMPLE / HBM_PEAK_GBS, 4),
                    "alu_TFLOPs": round(tf, 2),
                    "alu_roof_frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
                    "alu_unpacked_roof_frac": round(tf / FP32_UNPACKED_PEAK_TFLOPS, 4),
                    other + "_GS_per_s": round(gss(ms2), 2),
                    other + "_kernel_GS_per_s": round(gss(mk2), 2),
                    other + "_alu_roof_frac": round(tf2 / FP32_VECTOR_PEAK_TFLOPS, 4)}
                log(kind, K, result_sweep[kind][str(K)])
        h2.close()

    # plateau: kernel GS/s against the signal length (disjoint slices of the
    # two 1 GiB buffer pairs, rotated so that >= 512 MiB is touched per cycle,
    # beyond the 256 MB Infinity Cache)
    plateau = {}
    if not args.no_sweep and not args.only_k and args.log2n == 28:
        for K in (1, 8):
            sos_d = torch.from_numpy(workloads.sweep_sections(K, "butter")).to(dev)
            pts = []
            for lg in (24, 25, 26, 27, 28):
                m = 1 << lg
                k = min(8, n // m)
                sx = [xs[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
                sy = [ys[b][j * m:(j + 1) * m] for j in range(k) for b in (0, 1)]
                _, mk = time_steps(torch, P, h, sos_d, sx, sy, 20, 4)
                assert h.last_error() == P.SOS_OK
                pts.append({"log2n": lg, "kernel_GS_per_s": round(m / (mk * 1e-3) / 1e9, 2)})
            plateau["order_%d" % (2 * K)] = pts
            log("plateau", K, pts)

    copy_ms = time_copy(torch, P, xs, ys, 20, 3)
    copy_gbs = n * BYTES_PER_SAMPLE / (copy_ms * 1e-3) / 1e9
    log("copy %.4f ms = %.0f GB/s" % (copy_ms, copy_gbs))

    achieved_gbs = n * BYTES_PER_SAMPLE / (ms_kern * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": traffic_bytes(n),
                "kernel": "sos_fwd_kernel", "kernel_ms": round(ms_kern, 4),
                "copy_roof_GBs": round(copy_gbs, 1),
                "frac_of_copy_roof": round(achieved_gbs / copy_gbs, 4)}

    extra = {}
    if not args.quick and not args.only_k:
        del xs, ys, x0
        torch.cuda.empty_cache()
        extra["batched"] = bench_batched(torch, P, workloads, np, log)
        extra["served"] = bench_served(torch, P, workloads, np, log)
        extra["fwd_bwd"] = bench_fwd_bwd(torch, P, workloads, np, log)
        k16 = (result_sweep or {}).get("butter", {}).get("8", {}).get("kernel_GS_per_s")
        extra["toeplitz_mfma_bound"] = bench_toeplitz_bound(torch, n, k16, log)

    cpu = None
    cpu_extra = None
    if not args.no_cpu:
        n_cpu = min(n, 1 << 27)
        v, secs = cpu_baseline(sos1, x_host, n_cpu)
        cpu = {"value": round(v, 4), "unit": "GS/s", "cores": 1, "kind": "oracle",
               "sample": "FP64 sequential oracle, one thread, first 2^%d samples of the same "
                         "K=%d Butterworth signal, median of 3 runs (%.2f s each)"
                         % (n_cpu.bit_length() - 1, K1, secs)}
        log("cpu", cpu)
        # the paper's multi-core CPU method, beside the oracle (not the baseline)
        wf = {}
        for K in (K1, 8):
            v, secs, thr = cpu_wavefront_rate(workloads.sweep_sections(K, "butter"), x_host,
                                              min(n, 1 << 26))
            wf["order_%d" % (2 * K)] = {"value": round(v, 4), "unit": "GS/s", "threads": thr,
                                        "seconds": round(secs, 3)}
        cpu_extra = {"kind": "wavefront over groups of 2^16 samples and sections, FP32, "
                             "pthreads (Sec. III-A); first 2^26 samples, median of 3 runs",
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
        "cpu_wavefront": cpu_extra,
        "sweep": result_sweep,
        "plateau": plateau,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
