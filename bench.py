#!/usr/bin/env python3
"""Benchmark of the gfx950 coherent beamformer on one GPU.

One step = one bf_run over one synthetic block of the paper-scale workload
(BEST-2-like 4x8 array, 1024 channels over 16 MHz at 408 MHz, 128 beams,
65536 samples, integration 16), i.e. the whole hot path: int8 voltages in
HBM -> per-channel complex GEMM on MFMA -> |B|^2 -> integration -> FP32
power in HBM.  Inputs are resident in HBM before timing starts.  Prints one
JSON line (see ``main``).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--precision fp32|fp16|bf16] [--workload paper|small|precision]
                       [--no-cpu-baseline] [--no-extra]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "fp16": 2516.6, "bf16": 2516.6}  # MI355X dense MFMA
PEAK_HBM_GBS = 8000.0
DTYPE = {"fp32": "f32", "fp16": "f16 (f32 accumulate)", "bf16": "bf16 (f32 accumulate)"}


def progress(msg: str) -> None:
    """One line on stderr per finished phase (the JSON result stays the only
    line on stdout), so a long default run shows that it is alive."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "bf16"])
    ap.add_argument("--input-bits", type=int, default=8, choices=[8, 4],
                    help="voltage format: int8 pairs, or 4-bit pairs packed one per byte")
    ap.add_argument("--output", default="power", choices=["power", "complex"],
                    help="detected integrated power, or complex FP16 beams (integration 1)")
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "small", "precision", "large", "serve", "batch", "tracking"])
    ap.add_argument("--blocks", type=int, default=200, help="serve: blocks to stream")
    ap.add_argument("--pace", type=float, default=10.0,
                    help="serve: replay speed-up over real time for the latency run "
                         "(Poisson block arrivals with mean gap block_period / pace)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other-precision legs")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--retune", action="store_true", help="re-run the autotuner")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0,
                    help="serve: HBM budget for admitted requests")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES (counter calibration)")
    ap.add_argument("--library-gemm", action="store_true",
                    help="only time the vendor GEMM (torch.matmul, random data) at a few sizes: "
                         "the device's practical dense rate, for context")
    return ap.parse_args()


def library_gemm(reps: int = 30) -> None:
    """Median TFLOP/s of torch.matmul (hipBLASLt on ROCm) on random data:
    the practical dense-GEMM rate of this device under sustained load."""
    import torch
    dev = torch.device("cuda:0")
    rows = []
    for dtype, (m, n, k) in ((torch.float16, (8192, 8192, 8192)), (torch.float16, (16384, 16384, 8192)),
                             (torch.bfloat16, (8192, 8192, 8192)), (torch.float32, (8192, 8192, 8192))):
        a = torch.randn(m, k, device=dev, dtype=dtype)
        b = torch.randn(k, n, device=dev, dtype=dtype)
        for _ in range(3):
            a @ b
        torch.cuda.synchronize()
        r = reps if dtype != torch.float32 else 10
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(r + 1)]
        ev[0].record()
        for i in range(r):
            a @ b
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(r))
        rows.append({"dtype": str(dtype).split(".")[-1], "m": m, "n": n, "k": k,
                     "median_ms": round(ms[r // 2], 4),
                     "tflops_median": round(2.0 * m * n * k / ms[r // 2] / 1e9, 1),
                     "tflops_best": round(2.0 * m * n * k / ms[0] / 1e9, 1)})
        del a, b
    print(json.dumps({"library_gemm": rows}), flush=True)


def copy_calibration(nbytes: int, reps: int = 3) -> None:
    """A plain copy kernel of known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings: each dispatch reads and writes nbytes."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(7)
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def workload(name):
    from paper_1412_4907_amd import synth
    return {"paper": synth.paper, "small": synth.small, "precision": synth.precision,
            "large": synth.large}[name]()


def algorithmic_bytes(w, prec, output="power") -> float:
    """Bytes one launch must move at minimum: every voltage once, every
    weight once, every output window (or complex FP16 sample) once."""
    es = 4 if prec == "fp32" else 2
    x = w.n_chan * w.n_samples * w.n_ant * (1 if w.input_bits == 4 else 2)
    wt = w.n_chan * w.n_beams * w.n_ant * 2 * es
    p = w.n_chan * w.n_beams * (w.n_samples // w.integration) * 4  # f32 power or 2 x f16
    return float(x + wt + p)


def time_plan(plan, xd, p, steps, warmup, torch):
    """Per-step HIP events on torch's current stream (the stream bf_run is
    given); returns per-step ms and the whole timed region in ms.  xd and p
    may be lists of equally shaped buffers, used in turn (so that a small
    workload cannot be served from the 256 MB last-level cache)."""
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    xs = xd if isinstance(xd, (list, tuple)) else [xd]
    ps = p if isinstance(p, (list, tuple)) else [p]
    bufs = [(x.data_ptr(), q.data_ptr()) for x, q in zip(xs, ps)]
    for i in range(warmup):
        plan.run_ptr(*bufs[i % len(bufs)], sp)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        plan.run_ptr(*bufs[i % len(bufs)], sp)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]
    total = ev[0].elapsed_time(ev[steps])
    return per, total


def cpu_baseline(w, budget_s: float) -> dict:
    """The FP64 oracle, as it stands, on a bounded channel sample of the same
    workload (all beams, all samples of each sampled channel): compute-only
    wall time, best of 3 runs sharing the budget."""
    import oracle
    g = np.random.default_rng(4907)
    order = g.permutation(w.n_chan)
    W = oracle.weights(w.pos, w.dirs, w.freqs[order[:1]])
    x1 = w.voltages(channels=order[:1])
    four = w.input_bits == 4
    t = time.perf_counter()
    oracle.beamform(W, oracle.unpack4(x1) if four else x1, w.integration)
    t1 = time.perf_counter() - t
    n = int(max(1, min(w.n_chan - 1, budget_s / 3 / max(t1, 1e-3))))
    chans = order[1:1 + n]
    W = oracle.weights(w.pos, w.dirs, w.freqs[chans])
    x = w.voltages(channels=chans, workers=8)
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        oracle.beamform(W, oracle.unpack4(x) if four else x, w.integration)
        runs.append(time.perf_counter() - t)
    dt = min(runs)
    flops = 8.0 * len(chans) * w.n_beams * w.n_samples * w.n_ant
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{len(chans)} of {w.n_chan} channels (seeded), all {w.n_beams} beams x "
                      f"{w.n_samples} samples x {w.n_ant} antennas, I={w.integration}"
                      f"{', 4-bit input decoded in the timed region' if four else ''}; "
                      f"best of 3 runs, {dt:.1f} s FP64 on the host"}


def precision_report(torch, dev, n_chan_check: int = 5) -> dict:
    """Power error of each precision form against the FP64 oracle on the
    512-beam precision workload (small array and voltages, I=1): per-beam
    normwise error max/median over a seeded channel sample, plus the
    accumulation-only error (oracle run on the GPU's own rounded weights)."""
    import oracle
    from paper_1412_4907_amd import bf, synth
    w = synth.precision()
    x = w.voltages()
    chans = sorted(synth.rng("precision", "check").choice(w.n_chan, n_chan_check, replace=False))
    ref = oracle.beamform(oracle.weights(w.pos, w.dirs, w.freqs[chans]), x[chans], 1)
    xd = torch.from_numpy(x).to(dev)
    rep = {"workload": "precision: N=32 line, C=128, B=512, T=4096, I=1",
           "channels_checked": [int(c) for c in chans]}
    for prec in ("fp32", "fp16", "bf16"):
        plan = bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, 1, precision=prec)
        plan.set_weights(w.pos, w.dirs, w.freqs)
        p = torch.empty((w.n_chan, w.n_beams, w.n_samples), device=dev)
        plan.run(xd, p)
        torch.cuda.synchronize()
        got = p[chans].cpu().numpy().astype(np.float64)
        wq = plan.get_weights()[chans]
        plan.destroy()
        refq = oracle.beamform(wq, x[chans], 1)
        e = np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)
        eq = np.linalg.norm(got - refq, axis=-1) / np.linalg.norm(refq, axis=-1)
        rep[prec] = {"power_err_max": float(e.max()), "power_err_median": float(np.median(e)),
                     "accumulation_err_max": float(eq.max())}
    return rep


def roofline(tflops: float, peak: float, abytes: float, ms: float, flops: float, traffic) -> dict:
    """The bounding roofline of the workload: MFMA when its arithmetic
    intensity (flop per algorithmic byte) is above the ridge peak / 8 TB/s,
    else HBM; achieved and peak in that roofline's unit."""
    gbs = abytes / (ms * 1e-3) / 1e9
    ridge = peak * 1e12 / (PEAK_HBM_GBS * 1e9)
    common = {"traffic": traffic, "algorithmic_bytes": abytes, "intensity_flop_per_byte":
              round(flops / abytes, 1), "ridge_flop_per_byte": round(ridge, 1)}
    if flops / abytes >= ridge:
        return {"bound": "mfma", "achieved": round(tflops, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tflops / peak, 4), **common,
                "algorithmic_hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)}
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4), **common,
            "mfma_tflops": round(tflops, 3), "mfma_frac": round(tflops / peak, 4)}


def load_traffic(kernel_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel build (else null)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except Exception:
        return None
    e = d.get(kernel_key)
    if not e:
        return None
    from paper_1412_4907_amd import build as pbuild
    if e.get("source_hash") != pbuild.source_hash():
        return None
    return e.get("bytes_per_launch")


# HBM ring slots of the serving form: up to this many blocks in flight, so the
# host's admission work for a new request (plan creation, weight generation)
# overlaps the blocks already queued
SERVE_RING_SLOTS = 3


def serve_bench(a, torch, dev, emit=True):
    """Serving form: 256-antenna 16x16 array, blocks of 1024 channels x 8192
    samples (524.288 ms each), FP16, I=64, seeded Poisson beam-set requests
    (64..2048 beams, mean ~512 concurrently active) admitted by HBM footprint,
    one batched launch per block replayed as a hipGraph.  Runs:
    * throughput: blocks pre-staged in an HBM ring (the NIC-to-GPU case),
      released as soon as a ring slot frees -> real-time factor;
    * paced: seeded Poisson block arrivals at ``--pace``x real time -> block
      latency p50/p99 from arrival to completion;
    * h2d: as throughput, but every block first copied from pinned host
      memory on a second stream, overlapped with the previous block's compute
      (PCIe-bound context, never the headline value);
    * load curve: real-time factor against the mean number of concurrently
      active beams (shorter runs)."""
    from paper_1412_4907_amd import serve, synth
    prec = "fp16" if a.precision == "fp32" else a.precision
    pos = synth.serve_array()
    C, T, I = 1024, 8192, 64
    freqs = synth.channel_freqs(C, 400e6, 16e6)
    period = T / (16e6 / 1024)
    t0 = time.perf_counter()
    ring = []
    for k in range(SERVE_RING_SLOTS):
        blk = synth.serve_block(k)
        if a.input_bits == 4:
            blk = synth.four_bit(blk)
        ring.append(torch.from_numpy(blk.voltages(workers=16)).to(dev))
    gen_s = time.perf_counter() - t0
    fp = lambda r: serve.footprint_bytes(r.n_beams, 256, C, T, I, prec,  # noqa: E731
                                         out_buffers=len(ring))
    budget = int(a.serve_budget_gb * (1 << 30))
    out = {"metric": "beamforming TFLOP/s (8 flop/cMAC) + % MFMA peak; real-time factor, "
                     "p99 block ms", "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
           "config": {"workload": "serve: N=256 (16x16 grid, 10 m), C=1024, T=8192 per block "
                                  "(524.288 ms), I=64, Poisson beam-set requests 64..2048 beams",
                      "precision": prec, "input_bits": a.input_bits,
                      "hbm_budget_gb": a.serve_budget_gb,
                      "ring_slots": len(ring), "blocks": a.blocks,
                      "paced_arrivals": f"seeded Poisson, mean gap {period / a.pace * 1e3:.3f} ms "
                                        f"({a.pace:g}x real time)"}}

    def run(reqs_spec, n_blocks, arrivals=None, host_blocks=None):
        reqs = [serve.Request(i, d, lifetime=life, arrival_block=arr_b)
                for i, (arr_b, nb, life, d) in enumerate(reqs_spec)]
        ex = serve.GpuExecutor(pos, freqs, T, I, prec, ring=ring, host_blocks=host_blocks,
                               input_bits=a.input_bits)
        sch = serve.Scheduler(budget, fp)
        recs = serve.serve(ex, sch, reqs, n_blocks=n_blocks, block_period_s=period,
                           arrivals=arrivals)
        ex.close()
        st = serve.summarize(recs, period)
        beams = sum(r.beams for r in recs)
        st["tflops"] = 8.0 * C * T * 256 * beams / st["wall_s"] / 1e12 if st["wall_s"] else None
        st["graph_replays"] = ex.graph_replays
        st["eager_launches"] = ex.eager_launches
        st["requests_finished"] = len(sch.finished)
        if host_blocks is not None:
            st["h2d_gb_s"] = ex.h2d_bytes / st["wall_s"] / 1e9 if st["wall_s"] else None
        return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}

    reqs_spec = synth.serve_requests(64)
    out["throughput"] = run(reqs_spec, a.blocks)
    progress(f"serve throughput: real-time factor {out['throughput']['rtf']}")
    out["paced"] = run(reqs_spec, a.blocks, arrivals=synth.serve_block_arrivals(a.blocks, period,
                                                                                 a.pace))
    host = []
    for r in ring:
        h = torch.empty(r.shape, dtype=r.dtype, pin_memory=True)
        h.copy_(r)
        host.append(h)
    progress(f"serve paced: p99 {out['paced']['p99_block_ms']} ms")
    out["h2d"] = run(reqs_spec, min(a.blocks, 60), host_blocks=host)
    progress(f"serve PCIe-fed: real-time factor {out['h2d']['rtf']}")
    del host
    curve = []
    for load in (128, 256, 512, 1024, 2048):
        st = run(synth.serve_requests(64, mean_concurrent_beams=float(load)), min(a.blocks, 100))
        curve.append({"mean_concurrent_beams": load, "mean_active_beams": st["mean_active_beams"],
                      "rtf": st["rtf"], "tflops": st["tflops"], "p99_block_ms": st["p99_block_ms"]})
    out["rtf_vs_load"] = curve
    thr = out["throughput"]
    out["value"] = round(thr["tflops"], 3)
    out["mfma_peak_frac"] = round(thr["tflops"] / PEAK_TFLOPS[prec], 4)
    out["real_time_factor"] = thr["rtf"]
    out["p50_block_ms"] = out["paced"]["p50_block_ms"]
    out["p99_block_ms"] = out["paced"]["p99_block_ms"]
    out["block_period_ms"] = round(period * 1e3, 3)
    out["input_gen_s"] = round(gen_s, 1)
    if emit:
        print(json.dumps(out), flush=True)
    return out


def tracking_bench(a, torch, dev):
    """Tracking beams: a 512-beam set on the serving array (N=256, 1024
    channels x 8192 samples, I=64) whose pointing changes every block.  Per
    block time with static weights, with the refresh enqueued on the run
    stream before each block, and with the refresh generated on a side stream
    (bf_set_weights_async) while the previous block runs."""
    from paper_1412_4907_amd import bf, synth, tune
    blk = synth.serve_block(0)
    B, steps = 512, max(a.steps, 8)
    g = synth.rng("serve", "tracking")
    base = synth.random_dirs(B, g, 25.0)

    def pointing(k):
        ang = np.deg2rad(0.05 * k)
        rot = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]])
        d = base @ rot.T
        return d / np.linalg.norm(d, axis=1, keepdims=True)

    x = torch.from_numpy(blk.voltages(workers=16)).to(dev)
    plan = bf.Plan(blk.n_ant, blk.n_chan, B, blk.n_samples, blk.integration, precision=a.precision)
    p = torch.empty(plan.p_shape, dtype=plan.p_dtype, device=dev)
    run_s, side_s = torch.cuda.Stream(), torch.cuda.Stream()
    plan.set_weights(blk.pos, pointing(0), blk.freqs, stream=run_s)
    if tune.apply_cached(plan) is None:
        with torch.cuda.stream(run_s):
            tune.tune(plan, x, p, reps=3)

    def leg(mode):
        for k in range(a.warmup):
            plan.run(x, p, stream=run_s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(run_s)
        for k in range(steps):
            if mode == "sync":
                plan.set_weights(blk.pos, pointing(k + 1), blk.freqs, stream=run_s)
            elif mode == "async":
                plan.set_weights_async(blk.pos, pointing(k + 1), blk.freqs, stream=side_s)
            plan.run(x, p, stream=run_s)
        e1.record(run_s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    static = leg("static")
    sync = leg("sync")
    asyn = leg("async")
    # the weight generation alone
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(run_s)
    for k in range(steps):
        plan.set_weights(blk.pos, pointing(k), blk.freqs, stream=run_s)
    e1.record(run_s)
    torch.cuda.synchronize()
    gen = e0.elapsed_time(e1) / steps
    flops = 8.0 * blk.n_chan * B * blk.n_samples * blk.n_ant
    period = blk.n_samples / (16e6 / 1024)
    out = {"metric": "tracking beams: block time with per-block weight refresh", "value":
           round(flops / (asyn * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": steps,
           "warmup": a.warmup, "ms_per_step": round(asyn, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[a.precision], "data": "synthetic",
           "config": {"workload": f"tracking: N={blk.n_ant} (16x16 grid), C={blk.n_chan}, B={B}, "
                                  f"T={blk.n_samples}, I={blk.integration}, new pointing per block",
                      "precision": a.precision, "tile": list(plan.tile())},
           "static_ms": round(static, 4), "sync_refresh_ms": round(sync, 4),
           "async_refresh_ms": round(asyn, 4), "weight_generation_ms": round(gen, 4),
           "hidden_fraction": round((sync - asyn) / max(sync - static, 1e-9), 3),
           "real_time_factor": round(period / (asyn * 1e-3), 1)}
    plan.destroy()
    print(json.dumps(out), flush=True)


def batch_bench(a, torch, dev, emit=True):
    """Batching form: the 12 seeded beam sets of uneven N, C, B, T in one
    persistent launch (tiles from the autotuner cache or each set's default)."""
    from paper_1412_4907_amd import bf, synth, tune
    prec = a.precision
    sets = synth.batch_sets()
    plans, xs, ps = [], [], []
    t0 = time.perf_counter()
    flops = 0.0
    abytes = 0.0
    for w in sets:
        plan = bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, w.integration, precision=prec)
        plan.set_weights(w.pos, w.dirs, w.freqs)
        plans.append(plan)
        xs.append(torch.from_numpy(w.voltages(workers=16)).to(dev))
        ps.append(torch.empty((w.n_chan, w.n_beams, w.n_samples // w.integration), device=dev))
        # per-set tile from the autotuner, among the batching kernel's variants
        if a.retune or tune.apply_cached(plan, batch=True) is None:
            tune.tune(plan, xs[-1], ps[-1], reps=2, batch=True)
        flops += w.flops
        abytes += algorithmic_bytes(w, prec)
    gen_s = time.perf_counter() - t0
    batch = bf.Batch(plans)
    stream = torch.cuda.current_stream()
    for _ in range(a.warmup):
        batch.run(xs, ps)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    ev[0].record(stream)
    for i in range(a.steps):
        batch.run(xs, ps)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(a.steps)]
    ms = ev[0].elapsed_time(ev[a.steps]) / a.steps
    # per-set solo time, for the batched-vs-sum comparison
    solo_ms = 0.0
    for plan, x, p in zip(plans, xs, ps):
        s_per, s_total = time_plan(plan, x, p, 3, 1, torch)
        solo_ms += s_total / 3
    value = flops / (ms * 1e-3) / 1e12
    # roofline fraction: sum over sets of max(flop/peak, bytes/bandwidth) / time
    ideal = 0.0
    for w in sets:
        ideal += max(w.flops / (PEAK_TFLOPS[prec] * 1e12), algorithmic_bytes(w, prec) / (PEAK_HBM_GBS * 1e9))
    out = {"metric": "beamforming TFLOP/s (8 flop/cMAC) + % MFMA peak; real-time factor, "
                     "p99 block ms", "value": round(value, 3), "unit": "TFLOP/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPE[prec], "data": "synthetic",
           "config": {"workload": "batch: 12 seeded beam sets, N in {16..256}, C in "
                                  "{256,512,1024}, B in {16..1024}, T in [8192,32768], I=16",
                      "sets": [[w.n_ant, w.n_chan, w.n_beams, w.n_samples] for w in sets]},
           "roofline_frac": round(ideal * 1e3 / ms, 4),
           "tiles": [list(p.tile()) for p in plans],
           "sum_of_solo_ms": round(solo_ms, 4),
           "p99_block_ms": round(float(np.percentile(per, 99)), 4),
           "input_gen_s": round(gen_s, 1)}
    batch.destroy()
    for p in plans:
        p.destroy()
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.library_gemm:
        library_gemm()
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(channel-sharded multi-GPU operation is a design note only)"}))
        sys.exit(2)
    import torch
    from paper_1412_4907_amd import bf, tune

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.workload == "serve":
        return serve_bench(a, torch, dev)
    if a.workload == "batch":
        return batch_bench(a, torch, dev)
    if a.workload == "tracking":
        return tracking_bench(a, torch, dev)
    w = workload(a.workload)
    if a.input_bits == 4:
        from paper_1412_4907_amd import synth
        w = synth.four_bit(w)
    if a.output == "complex":
        import dataclasses
        w = dataclasses.replace(w, name=w.name + "_complex", integration=1)
    t0 = time.perf_counter()
    x = w.voltages(workers=16)
    gen_s = time.perf_counter() - t0
    xd = torch.from_numpy(x).to(dev)
    del x
    windows = w.n_samples // w.integration

    def leg(prec, steps, warmup):
        plan = bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, w.integration, precision=prec,
                       input_bits=w.input_bits, output=a.output)
        plan.set_weights(w.pos, w.dirs, w.freqs)
        if a.output == "complex":
            plan.set_output_scale(1.0 / np.sqrt(w.n_ant))
        p = torch.empty(plan.p_shape, dtype=plan.p_dtype, device=dev)
        # tile shape from the autotuner's cache, else tuned now (untimed)
        if a.retune or tune.apply_cached(plan) is None:
            tune.tune(plan, xd, p, reps=3)
        hot = None
        if xd.numel() + p.numel() * 4 < (1 << 30):
            # small footprint: 16 distinct input/output buffers in turn, so
            # the timed figure is not served from the last-level cache; the
            # single-buffer ("hot") figure is reported beside it
            xs = [xd] + [xd.clone() for _ in range(15)]
            ps = [p] + [torch.empty_like(p) for _ in range(15)]
            per, total = time_plan(plan, xs, ps, steps, warmup, torch)
            _, hot_total = time_plan(plan, xd, p, steps, warmup, torch)
            hot = hot_total / steps
            del xs, ps
        else:
            per, total = time_plan(plan, xd, p, steps, warmup, torch)
        info = plan.info()
        info["hot_ms"] = hot
        plan.destroy()
        del p
        return per, total, info

    per, total, info = leg(a.precision, a.steps, a.warmup)
    progress(f"{w.name} {a.precision}: {total / a.steps:.3f} ms per block")
    ms = total / a.steps
    flops = w.flops
    value = flops / (ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[a.precision]
    abytes = algorithmic_bytes(w, a.precision, a.output)
    chan_rate = 16e6 / 1024  # channel sample rate of every workload here
    block_s = w.n_samples / chan_rate
    kernel_key = f"beamform/{w.name}/{a.precision}"
    out = {
        "metric": "beamforming TFLOP/s (8 flop/cMAC) + % MFMA peak; real-time factor, p99 block ms",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: N={w.n_ant} antennas, C={w.n_chan} channels, "
                               f"B={w.n_beams} beams, T={w.n_samples} samples, I={w.integration}",
                   "precision": a.precision, "input_bits": w.input_bits, "output": a.output,
                   "n_antennas": w.n_ant, "n_channels": w.n_chan,
                   "n_beams": w.n_beams, "n_samples": w.n_samples, "integration": w.integration,
                   "tile": {"mt": info["tile_mt"], "nbt": info["tile_nbt"],
                            "nbp": info["tile_nbp"], "kres": info["tile_kres"],
                            "sg_per_wave": info["sg_per_wave"]},
                   "work_units": info["work_units"]},
        "mfma_peak_frac": round(value / peak, 4),
        "real_time_factor": round(block_s / (ms * 1e-3), 1),
        "p10_block_ms": round(float(np.percentile(per, 10)), 4),
        "p50_block_ms": round(float(np.percentile(per, 50)), 4),
        "p90_block_ms": round(float(np.percentile(per, 90)), 4),
        "p99_block_ms": round(float(np.percentile(per, 99)), 4),
        "block_period_ms": round(block_s * 1e3, 3),
        "roofline": roofline(value, peak, abytes, ms, flops, load_traffic(kernel_key)),
        "input_gen_s": round(gen_s, 1),
    }
    if info.get("hot_ms") is not None:
        out["buffers_rotated"] = 16
        out["hot_ms_per_step"] = round(info["hot_ms"], 4)
    if not a.no_extra:
        extra = {}
        for prec in ("fp32", "fp16", "bf16"):
            if prec == a.precision:
                continue
            per2, total2, _ = leg(prec, a.steps, a.warmup)
            ms2 = total2 / a.steps
            progress(f"{w.name} {prec}: {ms2:.3f} ms per block")
            v2 = flops / (ms2 * 1e-3) / 1e12
            ab2 = algorithmic_bytes(w, prec, a.output)
            extra[prec] = {"tflops": round(v2, 3), "ms_per_step": round(ms2, 4),
                           "mfma_peak_frac": round(v2 / PEAK_TFLOPS[prec], 4),
                           "hbm_frac": round(ab2 / (ms2 * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                           "p99_block_ms": round(float(np.percentile(per2, 99)), 4)}
        out["other_precisions"] = extra
    del xd
    if not a.no_extra:
        out["precision_forms"] = precision_report(torch, dev)
        progress("precision forms against the oracle")
    if not a.no_extra and a.workload == "paper" and w.input_bits == 8 and a.output == "power":
        # the batching and serving forms, in FP16 at their own workloads, so
        # that the default run also records them (summaries of
        # --workload batch / --workload serve)
        import argparse
        sub = argparse.Namespace(**vars(a))
        sub.precision = "fp16"
        b = batch_bench(sub, torch, dev, emit=False)
        progress(f"batch fp16: {b['ms_per_step']} ms per batch")
        sv = serve_bench(sub, torch, dev, emit=False)
        progress(f"serve fp16: real-time factor {sv['real_time_factor']}")
        out["other_workloads"] = {
            "batch_fp16": {"workload": b["config"]["workload"], "ms_per_step": b["ms_per_step"],
                           "tflops": b["value"], "roofline_frac": b["roofline_frac"],
                           "sum_of_solo_ms": b["sum_of_solo_ms"]},
            "serve_fp16": {"workload": sv["config"]["workload"], "tflops": sv["value"],
                           "real_time_factor": sv["real_time_factor"],
                           "mean_active_beams": sv["throughput"]["mean_active_beams"],
                           "deadline_misses": sv["throughput"]["deadline_misses"],
                           "paced_p50_block_ms": sv["p50_block_ms"],
                           "paced_p99_block_ms": sv["p99_block_ms"],
                           "blocks": sv["throughput"]["blocks"]}}
    if not a.no_cpu_baseline:
        progress("CPU baseline (FP64 oracle)")
        cb = cpu_baseline(w, a.cpu_seconds)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = round(value / cb["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
