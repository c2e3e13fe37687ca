"""Autotuner for the beamform kernel's tile shape.

Sec. 2.2 tunes two parameters of the K20 kernel (accumulators per thread and
threads per block) by sweeping them on the target device.  The tunables
here are the gfx950 kernel's compiled tile variants -- (MT row tiles per
wave step, NBT beam tiles per workgroup, NBP beam tiles per pass, KRES K
chunks in registers) -- and the work-unit length (store groups per wave).
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


def shape_key(plan, arch: str = "gfx950") -> str:
    """Tile choice depends on precision, input and output form, N, B, I and the block
    length; C and T enter through the number of work units (bucketed by
    powers of 2)."""
    import math
    cb = 1 << int(math.log2(max(1, plan.C)))
    tb = 1 << int(math.log2(max(1, plan.T)))
    fmt = "/in4" if getattr(plan, "input_bits", 8) == 4 else ""
    fmt += "/cx" if getattr(plan, "output", "power") == "complex" else ""
    return f"{arch}/p{plan.precision}/N{plan.N}/B{plan.B}/I{plan.I}/C~{cb}/T~{tb}{fmt}"


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
    opts = []
    k = 1
    while True:
        s = base * k
        if s * G > 1024 or (k > 1 and (s - base) * 4 >= sg_total):
            break
        opts.append(s)
        k *= 2
    return opts or [base]


def apply_cached(plan, batch: bool = False) -> Optional[tuple]:
    e = load_cache().get(shape_key(plan) + ("/batch" if batch else ""))
    if not e:
        return None
    try:
        plan.set_tile(*e["tile"])
        return tuple(e["tile"])
    except Exception:
        return None


def tune(plan, x, p, reps: int = 3, max_candidates: Optional[int] = None, save: bool = True,
         verbose: bool = False, batch: bool = False) -> dict:
    """Time every (tile, sgw) candidate on device tensors x, p; apply and
    return the fastest.  ``p`` is overwritten.  ``batch``: only the variants
    the persistent batching kernel carries (cached under a separate key)."""
    import torch
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    xp, pp = x.data_ptr(), p.data_ptr()
    results = []
    cands = plan.tile_candidates(batch=batch) or plan.tile_candidates()
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
        d[shape_key(plan) + ("/batch" if batch else "")] = out
        save_cache(d)
    return out
