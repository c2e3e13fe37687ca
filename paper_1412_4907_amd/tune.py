"""Autotuner for the beamform kernel's tile shape.

Sec. 2.2 tunes two parameters of the K20 kernel (accumulators per thread and
threads per block) by sweeping them on the target device.  The tunables
here are the gfx950 kernel's compiled tile variants -- (MT row tiles per
wave step, NBT beam tiles per workgroup, NBP beam tiles per pass, KRES K
chunks in registers; KRES -1 streams weights from device memory, -2 is the
eight-wave streamed form) -- and the work-unit length (store groups per
wave).
Each candidate is timed with HIP events on the caller's inputs; the fastest
is applied with ``bf_plan_set_tile`` and remembered in a JSON cache keyed by
device and problem shape.  The tile never changes the results (same K
order and window sums), only the speed.

Cache: ``$BF_TUNE_CACHE`` or ``tune_cache.json`` next to this file.
"""
from __future__ import annotations

import json
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path() -> str:
    return os.environ.get("BF_TUNE_CACHE", os.path.join(HERE, "tune_cache.json"))


def shape_key(plan, batch: bool = False) -> str:
    """The library's own cache key for the plan (``bf_tune_key``): precision,
    input and output form, N and I exactly; B, C and T bucketed to the
    largest power of two not above them (they act on the best tile through
    the number of work units)."""
    return plan.tune_key(batch)


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except Exception:
        return {}


def save_cache(d: dict) -> None:
    path = cache_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def sgw_options(plan, tile) -> list:
    """Store groups per wave per unit: multiples of the smallest legal value
    (sgw * tiles-per-store-group must be a multiple of MT)."""
    from math import gcd
    I = plan.I
    G = 1 if I == 1 else 2 if I == 2 else 4 * ((I + 3) // 4)
    base = tile[0] // gcd(tile[0], G)
    sg_total = -(-(plan.T // I) // 16)
    waves = 8 if tile[3] == -2 else 4   # waves sharing one work unit
    opts = []
    k = 1
    while True:
        s = base * k
        if s * G > 1024 or (k > 1 and (s - base) * waves >= sg_total):
            break
        opts.append(s)
        k *= 2
    return opts or [base]


def apply_cached(plan, batch: bool = False) -> Optional[tuple]:
    """Apply the cached tile for the plan's shape through the library
    (``bf_plan_apply_tuned``); None if the cache has no usable entry."""
    return plan.tile() if plan.apply_tuned(batch) else None


def lds_bytes(plan, tile) -> int:
    """Dynamic LDS a tile stages for this plan (its beam range's weight rows
    for all K; none when the weights are read from device memory)."""
    if tile[3] == -1:
        return 0
    es = 4 if plan.precision == 0 else 2
    kpad = -(-2 * plan.N // 64) * 64
    return 2 * 16 * tile[1] * (kpad * es + 16)


def tune(plan, x, p, reps: int = 3, max_candidates: Optional[int] = None, save: bool = True,
         verbose: bool = False, batch: bool = False, lds_limit: Optional[int] = None) -> dict:
    """Time every (tile, sgw) candidate on device tensors x, p; apply and
    return the fastest.  ``p`` is overwritten.  ``batch``: only the variants
    the persistent batching kernel carries (cached under a separate key);
    ``lds_limit``: only tiles staging at most that many LDS bytes (the table
    kernel's fixed LDS size)."""
    import torch
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    xp, pp = x.data_ptr(), p.data_ptr()
    results = []
    cands = plan.tile_candidates(batch=batch) or plan.tile_candidates()
    if lds_limit is not None:
        cands = [t for t in cands if lds_bytes(plan, t) <= lds_limit] or cands
    if max_candidates:
        cands = cands[:max_candidates]
    for t in cands:
        for s in sgw_options(plan, t):
            try:
                plan.set_tile(*t, s)
            except Exception:
                continue
            plan.run_ptr(xp, pp, sp)  # warm-up
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
            ev[0].record(stream)
            for i in range(reps):
                plan.run_ptr(xp, pp, sp)
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
            results.append((ms, t + (s,)))
            if verbose:
                print(f"  tile {t} sgw {s}: {ms:.4f} ms", flush=True)
    results.sort()
    best_ms, best = results[0]
    plan.set_tile(*best)
    out = {"tile": list(best), "ms": best_ms, "candidates": len(results)}
    if save:
        d = load_cache()
        d[shape_key(plan, batch)] = out
        save_cache(d)
        from . import bf
        bf.tune_load(cache_path())
    return out


def _tune_workloads(what: str, verbose: bool) -> list:
    """Tune the cache entries of a named workload family on the device:
    ``paper`` -- the paper-scale block in every precision, int8 and 4-bit
    input (single-run kernel); ``serve`` -- the serving shape (256 antennas,
    1024 channels x 8192 samples, I = 64, FP16) at every power-of-two beam
    count from 64 to 2048 (the batching kernel's variants, for the table
    kernel the serving loop replays)."""
    import torch
    import numpy as np
    from . import bf, synth
    dev = torch.device("cuda:0")
    out = []
    if what == "paper":
        for bits in (8, 4):
            w = synth.paper() if bits == 8 else synth.four_bit(synth.paper())
            x = torch.from_numpy(w.voltages(workers=16)).to(dev)
            for prec in ("fp32", "fp16", "bf16"):
                plan = bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, w.integration,
                               precision=prec, input_bits=bits)
                plan.set_weights(w.pos, w.dirs, w.freqs)
                p = torch.empty(plan.p_shape, dtype=plan.p_dtype, device=dev)
                r = tune(plan, x, p, reps=3, verbose=verbose)
                out.append((plan.tune_key(), r))
                print(f"{plan.tune_key()}: {r}", flush=True)
                plan.destroy()
            del x
    elif what == "serve":
        blk = synth.serve_block(0)
        x = torch.from_numpy(blk.voltages(workers=16)).to(dev)
        for B in (64, 128, 256, 512, 1024, 2048):
            plan = bf.Plan(blk.n_ant, blk.n_chan, B, blk.n_samples, blk.integration,
                           precision="fp16")
            plan.set_weights(blk.pos, synth.random_dirs(B, np.random.default_rng(B)), blk.freqs)
            p = torch.empty(plan.p_shape, dtype=plan.p_dtype, device=dev)
            # the table kernel keeps two workgroups per CU: 80 KB of LDS
            r = tune(plan, x, p, reps=3, batch=True, verbose=verbose, lds_limit=80 * 1024)
            out.append((plan.tune_key(batch=True), r))
            print(f"{plan.tune_key(batch=True)}: {r}", flush=True)
            plan.destroy()
            del p
    else:
        raise ValueError(what)
    return out


def main(argv=None) -> None:
    """python -m paper_1412_4907_amd.tune {paper,serve} [--out PATH] [-v]:
    tune a workload family on the GPU and merge the results into the cache
    (PATH, started from the package's cache if it does not exist yet)."""
    import argparse
    import shutil
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["paper", "serve"])
    ap.add_argument("--out", default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args(argv)
    if a.out:
        if not os.path.exists(a.out):
            shutil.copyfile(cache_path(), a.out)
        os.environ["BF_TUNE_CACHE"] = os.path.abspath(a.out)
    _tune_workloads(a.what, a.v)


if __name__ == "__main__":
    main()
