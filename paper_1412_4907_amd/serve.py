"""Streaming serve loop: continuous batching of beam-set requests over a
stream of voltage blocks, one batched launch per block, captured as a
hipGraph.

Sec. 2.2 observes that a beamforming pipeline spends half its time waiting
for voltages over PCIe and proposes overlapping copies with compute on a
second stream; Sec. 3.2 recomputes weights while the previous iteration runs
and keeps beams on the device for downstream stages.  The serving form here
builds those ideas on one MI355X:

* blocks (C channels x T samples x N antennas, int8) land in a ring of HBM
  slots (pre-staged: the NIC-to-GPU assumption; or copied from pinned host
  memory on a copy stream, the PCIe-bound variant);
* beam-set requests (a set of pointings, a lifetime in blocks) arrive at any
  time; at each block boundary the scheduler retires finished requests and
  admits waiting ones while their HBM footprint (weights + one output
  buffer per ring slot) fits the budget -- requests arriving while others run join the
  next block's launch (continuous batching, not a queue of whole jobs);
* each admitted request owns a plan (weights generated on the device once,
  at admission) and one output buffer per ring slot (block k writes buffer
  k mod slots, so a block's output stays intact while the later blocks that
  can be in flight run); integration state never leaves HBM;
* the per-block work -- one queue-reset kernel and one persistent beamform
  launch over every active request -- reads its set table (which requests,
  which ring slot, which output buffers) from device memory, so it is
  captured once as a hipGraph and replayed for every block; before each
  replay a one-workgroup kernel stores that block's table;
* per block: arrival time, completion time (stamped by a watcher thread as
  soon as the block's completion event fires), latency, deadline misses
  (completion later than arrival + one block period) and the real-time
  factor (block period / processing time) are recorded;
* a retired request's plan is freed once the last block that used it has
  completed (its completion event), without synchronising the device.

A request's output is bitwise the same whether it runs alone or in a mix
(each work unit depends only on its own set's voltages and weights).

The scheduler (``Scheduler``) is pure Python and is unit-tested on the CPU
with a fake executor; ``GpuExecutor`` runs the C ABI.
"""
from __future__ import annotations

import queue
import threading
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    """A beam-set request: ``dirs`` [B][3] unit pointings, alive for
    ``lifetime`` blocks from admission (None = until cancelled)."""
    rid: int
    dirs: np.ndarray
    lifetime: Optional[int] = None
    arrival_block: int = 0
    # filled by the scheduler
    admitted_block: Optional[int] = None
    finished_block: Optional[int] = None
    blocks_done: int = 0
    failed: Optional[str] = None

    @property
    def n_beams(self) -> int:
        return int(self.dirs.shape[0])


def footprint_bytes(n_beams: int, n_ant: int, n_chan: int, n_samples: int, integration: int,
                    precision: str, out_buffers: int = 2) -> int:
    """Device bytes one admitted request holds: its weight buffer in the
    MFMA operand layout plus ``out_buffers`` integrated-power outputs."""
    es = 4 if precision == "fp32" else 2
    bpad = -(-n_beams // 16) * 16
    kpad = -(-2 * n_ant // 64) * 64
    w = n_chan * bpad * 2 * kpad * es
    p = n_chan * n_beams * (n_samples // integration) * 4
    return int(w + out_buffers * p)


@dataclass
class BlockRecord:
    block: int
    active: List[int]
    beams: int
    arrival_s: float
    done_s: float = 0.0

    @property
    def latency_ms(self) -> float:
        return (self.done_s - self.arrival_s) * 1e3


class CompletionWatcher:
    """Stamps each block's completion time as soon as it completes: a thread
    waits on the blocks' completion events in enqueue order (one stream
    completes its work in order), so a block's stamp never waits for the
    host's own pacing or ring-slot waits."""

    def __init__(self, t0: float):
        self.t0 = t0
        self.q: "queue.Queue" = queue.Queue()
        self.err: Optional[BaseException] = None
        self.thread = threading.Thread(target=self._run, name="block-completion", daemon=True)
        self.thread.start()

    def add(self, ev, rec: "BlockRecord") -> None:
        self.q.put((ev, rec))

    def _run(self) -> None:
        while True:
            item = self.q.get()
            if item is None:
                return
            ev, rec = item
            try:
                ev.synchronize()
            except BaseException as e:  # reported by close()
                self.err = e
            rec.done_s = time.perf_counter() - self.t0

    def close(self) -> None:
        """Waits until every added block is stamped."""
        self.q.put(None)
        self.thread.join()
        if self.err is not None:
            raise self.err


class Scheduler:
    """Admission, retirement and footprint accounting (no device work)."""

    def __init__(self, budget_bytes: int, fp: Callable[[Request], int], max_active: int = 16):
        self.budget = int(budget_bytes)
        self.fp = fp
        self.max_active = max_active
        self.waiting: List[Request] = []
        self.active: Dict[int, Request] = {}
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.used = 0

    def submit(self, r: Request) -> None:
        if self.fp(r) > self.budget:
            r.failed = "footprint exceeds the whole budget"
            self.rejected.append(r)
            return
        self.waiting.append(r)

    def cancel(self, rid: int) -> None:
        if rid in self.active:
            self.active[rid].lifetime = self.active[rid].blocks_done
        self.waiting = [r for r in self.waiting if r.rid != rid]

    def fail(self, rid: int, why: str, block: int) -> None:
        r = self.active.pop(rid, None)
        if r is not None:
            r.failed = why
            r.finished_block = block
            self.used -= self.fp(r)
            self.finished.append(r)

    def step(self, block: int):
        """At a block boundary: retire finished requests, admit waiting ones
        in arrival order while they fit.  Returns (admitted, retired)."""
        retired = []
        for rid in list(self.active):
            r = self.active[rid]
            if r.lifetime is not None and r.blocks_done >= r.lifetime:
                r.finished_block = block
                self.used -= self.fp(r)
                retired.append(self.active.pop(rid))
        self.finished.extend(retired)
        admitted = []
        still = []
        for r in self.waiting:
            if r.arrival_block > block:
                still.append(r)
                continue
            f = self.fp(r)
            if len(self.active) < self.max_active and self.used + f <= self.budget:
                r.admitted_block = block
                self.active[r.rid] = r
                self.used += f
                admitted.append(r)
            else:
                still.append(r)
        self.waiting = still
        return admitted, retired

    def block_done(self, block: int) -> None:
        for r in self.active.values():
            r.blocks_done += 1


class GpuExecutor:
    """Runs the per-block batched launch through the C ABI: a table batch
    whose launch is captured once as a hipGraph and replayed for every
    block, whatever the active set."""

    def __init__(self, pos: np.ndarray, freqs: np.ndarray, n_samples: int, integration: int,
                 precision: str = "fp16", ring: Sequence = (), use_graphs: bool = True,
                 host_blocks: Optional[Sequence] = None, input_bits: int = 8):
        import torch
        from . import bf, tune
        self.torch, self.bf, self.tune = torch, bf, tune
        self.pos, self.freqs = pos, freqs
        self.N, self.C = pos.shape[0], freqs.shape[0]
        self.T, self.I = n_samples, integration
        self.precision = precision
        self.input_bits = input_bits     # 8: int8 [C][T][N][2] blocks; 4: packed uint8 [C][T][N]
        self.ring = list(ring)           # device voltage blocks
        # output buffers per request: one per block that can be in flight
        # (a block's output is written while up to len(ring) - 1 later
        # blocks are queued behind it)
        self.n_out = max(2, len(self.ring))
        self.use_graphs = use_graphs
        self.stream = torch.cuda.Stream()
        # PCIe-fed variant: every block is first copied from pinned host memory
        # (host_blocks[slot]) into its ring slot on a copy stream; the copy of
        # a block overlaps the previous block's compute, and a slot is
        # overwritten only after the compute that read it has finished
        self.host_blocks = list(host_blocks) if host_blocks is not None else None
        self.copy_stream = torch.cuda.Stream() if host_blocks is not None else None
        self.slot_free = [None] * len(self.ring)
        self.h2d_bytes = 0
        self.plans: Dict[int, object] = {}
        self.outs: Dict[int, List] = {}
        self.table = bf.Table(self.N, self.I, precision, input_bits=input_bits)
        self.graph = None
        # retired requests whose last block may still be running:
        # (that block's completion event, plan, outputs)
        self.retiring: List = []
        self.last_use: Dict[int, object] = {}
        self.eager_launches = 0
        self.graph_replays = 0
        self.tuned_admissions = 0

    def admit(self, r: Request) -> None:
        torch = self.torch
        plan = self.bf.Plan(self.N, self.C, r.n_beams, self.T, self.I, precision=self.precision,
                            input_bits=self.input_bits)
        with torch.cuda.stream(self.stream):
            plan.set_weights(self.pos, r.dirs, self.freqs, stream=self.stream)
            self.outs[r.rid] = [torch.empty((self.C, r.n_beams, self.T // self.I),
                                            dtype=torch.float32, device="cuda")
                                for _ in range(self.n_out)]
        # the table kernel's own tuned tile for this shape (B bucketed), if
        # the tile cache has one; else the plan keeps its creation tile
        if plan.apply_tuned(batch=True):
            self.tuned_admissions += 1
        self.plans[r.rid] = plan

    def retire(self, r: Request) -> None:
        """Drop a request: it is left out of every later table, and its plan
        and outputs are freed once the last block that read them has
        completed (checked at every later block; never a device-wide
        synchronisation)."""
        outs = self.outs.pop(r.rid, None)
        p = self.plans.pop(r.rid, None)
        if p is not None:
            self.retiring.append((self.last_use.pop(r.rid, None), p, outs))
        self.reap()

    def reap(self, wait: bool = False) -> None:
        """Free retired requests whose last block has completed (all of them,
        waiting for each, if ``wait``)."""
        keep = []
        for ev, p, outs in self.retiring:
            if ev is None or wait or ev.query():
                if ev is not None:
                    ev.synchronize()
                p.destroy()  # waits only for the plan's own weight generation
            else:
                keep.append((ev, p, outs))
        self.retiring = keep

    def run_block(self, ids: Sequence[int], slot: int, out_slot: int):
        """Enqueue one block's work on the serve stream (voltages from ring
        slot ``slot``, each request's output into its buffer ``out_slot``);
        returns an event recorded after it."""
        torch = self.torch
        ids = tuple(sorted(ids))
        if self.host_blocks is not None:
            cs = self.copy_stream
            if self.slot_free[slot] is not None:
                cs.wait_event(self.slot_free[slot])
            with torch.cuda.stream(cs):
                self.ring[slot].copy_(self.host_blocks[slot], non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(cs)
            self.stream.wait_event(copied)
            self.h2d_bytes += self.ring[slot].numel()
        if ids:
            self.table.set([self.plans[i] for i in ids], [self.ring[slot]] * len(ids),
                           [self.outs[i][out_slot] for i in ids], stream=self.stream)
            if self.graph is None or not self.use_graphs:
                # first block: run eagerly (also the warm-up that keeps
                # one-time runtime calls out of the capture), then capture
                # the same launch for every later block
                self.table.run(stream=self.stream)
                self.eager_launches += 1
                if self.use_graphs:
                    g = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g, stream=self.stream):
                        self.table.run(stream=self.stream)
                    self.graph = g
            else:
                with torch.cuda.stream(self.stream):
                    self.graph.replay()
                self.graph_replays += 1
        ev = torch.cuda.Event()
        ev.record(self.stream)
        self.slot_free[slot] = ev
        for i in ids:
            self.last_use[i] = ev
        return ev

    def output(self, rid: int, out_slot: int):
        return self.outs[rid][out_slot]

    def close(self) -> None:
        self.stream.synchronize()
        self.graph = None
        self.table.destroy()
        for p in self.plans.values():
            p.destroy()
        self.plans.clear()
        self.outs.clear()
        self.reap(wait=True)


def serve(executor, scheduler: Scheduler, requests: Sequence[Request], n_blocks: int,
          block_period_s: float, pace: float = 0.0, on_block=None,
          arrivals: Optional[Sequence[float]] = None) -> List[BlockRecord]:
    """Run ``n_blocks`` blocks.  ``arrivals`` (seconds from the start, e.g.
    a Poisson process) releases block k at arrivals[k]; else ``pace`` > 0
    releases it at k * block_period_s / pace (a replay ``pace`` times faster
    than real time), and 0 releases each block as soon as its ring slot is
    free.  Returns one record per block (latency = release -> completion, so
    a block that arrives while earlier ones still run includes its wait); a
    watcher thread stamps each completion when the block's event fires."""
    pending = sorted(requests, key=lambda r: r.arrival_block)
    pi = 0
    records: List[BlockRecord] = []
    inflight = []  # (event, record)
    n_slots = max(1, len(getattr(executor, "ring", [None])))
    n_out = max(2, getattr(executor, "n_out", 2))
    t0 = time.perf_counter()
    watcher = CompletionWatcher(t0)
    for k in range(n_blocks):
        while pi < len(pending) and pending[pi].arrival_block <= k:
            scheduler.submit(pending[pi])
            pi += 1
        admitted, retired = scheduler.step(k)
        for r in retired:
            executor.retire(r)
        for r in admitted:
            try:
                executor.admit(r)
            except Exception as e:  # a request that cannot start fails alone
                scheduler.fail(r.rid, f"admission failed: {e}", k)
        # ring slot k % n_slots must be free: wait for block k - n_slots
        while len(inflight) >= n_slots:
            ev, rec = inflight.pop(0)
            ev.synchronize()
        release = None
        if arrivals is not None:
            release = float(arrivals[k])
        elif pace > 0:
            release = k * block_period_s / pace
        now = time.perf_counter() - t0
        if release is not None and release > now:
            time.sleep(release - now)
        # latency counts from the block's arrival (it may have waited for a
        # ring slot behind earlier blocks)
        arrived = release if release is not None else time.perf_counter() - t0
        rec = BlockRecord(k, sorted(scheduler.active), sum(r.n_beams for r in scheduler.active.values()),
                          arrived)
        ev = executor.run_block(rec.active, k % n_slots, k % n_out)
        watcher.add(ev, rec)
        inflight.append((ev, rec))
        records.append(rec)
        scheduler.block_done(k)
        if on_block is not None:
            on_block(k, rec)
    watcher.close()
    for r in list(scheduler.active.values()):
        executor.retire(r)
    return records


def summarize(records: Sequence[BlockRecord], block_period_s: float,
              deadline_s: Optional[float] = None) -> dict:
    """Throughput and latency of a run.  A block misses its deadline when it
    completes later than ``deadline_s`` (default: one block period) after
    its arrival, i.e. a real-time pipeline would have fallen behind."""
    lat = np.array([r.latency_ms for r in records])
    wall = records[-1].done_s - records[0].arrival_s if records else 0.0
    dl_ms = (block_period_s if deadline_s is None else deadline_s) * 1e3
    misses = int(np.count_nonzero(lat > dl_ms)) if len(lat) else 0
    return {"blocks": len(records),
            "deadline_ms": dl_ms,
            "deadline_misses": misses,
            "deadline_miss_frac": (misses / len(records)) if records else 0.0,
            "rtf": (len(records) * block_period_s / wall) if wall > 0 else None,
            "p50_block_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_block_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "max_block_ms": float(lat.max()) if len(lat) else None,
            "mean_active_beams": float(np.mean([r.beams for r in records])) if records else 0.0,
            "wall_s": wall}
