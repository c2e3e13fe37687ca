"""Serving-form scheduler on the CPU with fake executors: admission by HBM
footprint, retirement, cancellation, a failing request that does not stop
the others, per-request results computed by the oracle on tiny shapes
(alone == in the mix), block latency stamped at completion (not at the
host's next wait), and deadline-miss accounting."""
import time

import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import serve, synth


class FakeEvent:
    def synchronize(self):
        pass


class FakeExecutor:
    """Oracle-backed executor on tiny shapes: block k's voltages are
    regenerated from the seed; each active request's output is the oracle's
    power for its own pointings."""

    def __init__(self, pos, freqs, T, I, fail_ids=()):
        self.pos, self.freqs, self.T, self.I = pos, freqs, T, I
        self.ring = [None, None]
        self.W = {}
        self.out = {}
        self.fail_ids = set(fail_ids)
        self.launches = []

    def admit(self, r):
        if r.rid in self.fail_ids:
            raise RuntimeError("simulated device allocation failure")
        self.W[r.rid] = oracle.weights(self.pos, r.dirs, self.freqs)
        self.out[r.rid] = {}

    def retire(self, r):
        self.W.pop(r.rid, None)

    def run_block(self, ids, slot, parity):
        self.launches.append(tuple(ids))
        w = synth.Workload("t", 77, self.pos.shape[0], len(self.freqs), 0, self.T, self.I,
                           self.pos, np.zeros((0, 3)), self.freqs)
        x = np.stack([synth.channel_voltages(500 + len(self.launches), c, self.T, self.pos,
                                             self.freqs[c]) for c in range(len(self.freqs))])
        for i in ids:
            self.out[i][len(self.launches) - 1] = oracle.beamform(self.W[i], x, self.I)
        return FakeEvent()


def _reqs(n, g, nb=(3, 5, 8)):
    out = []
    for i in range(n):
        out.append(serve.Request(i, synth.random_dirs(int(g.choice(nb)), g),
                                 lifetime=int(g.integers(1, 4)), arrival_block=int(g.integers(0, 6))))
    return out


def test_footprint_accounting_and_admission():
    fp = lambda r: 100 * r.n_beams  # noqa: E731
    s = serve.Scheduler(budget_bytes=1000, fp=fp)
    a = serve.Request(0, np.zeros((6, 3)), lifetime=2)
    b = serve.Request(1, np.zeros((5, 3)), lifetime=1)
    c = serve.Request(2, np.zeros((4, 3)), lifetime=1)
    huge = serve.Request(3, np.zeros((11, 3)), lifetime=1)
    for r in (a, b, c, huge):
        s.submit(r)
    assert huge in s.rejected
    adm, ret = s.step(0)
    assert [r.rid for r in adm] == [0, 2] and s.used == 1000  # b (500) does not fit after a (600)
    s.block_done(0)
    adm, ret = s.step(1)        # c done (lifetime 1) -> b still does not fit next to a
    assert [r.rid for r in ret] == [2] and [r.rid for r in adm] == []
    s.block_done(1)
    adm, ret = s.step(2)        # a done -> b admitted
    assert sorted(r.rid for r in ret) == [0] and [r.rid for r in adm] == [1]
    assert s.used == 500
    s.cancel(1)
    adm, ret = s.step(3)
    assert [r.rid for r in ret] == [1] and s.used == 0


def test_serve_loop_alone_equals_mix_with_failure():
    g = np.random.default_rng(3)
    pos = synth.disc_positions(5, 50.0, g)
    freqs = np.array([401e6, 409e6])
    T, I = 16, 4
    reqs = _reqs(7, g)
    fp = lambda r: serve.footprint_bytes(r.n_beams, 5, 2, T, I, "fp32")  # noqa: E731
    budget = 3 * fp(serve.Request(0, np.zeros((8, 3))))
    ex = FakeExecutor(pos, freqs, T, I, fail_ids={4})
    sch = serve.Scheduler(budget, fp)
    recs = serve.serve(ex, sch, reqs, n_blocks=12, block_period_s=0.0)
    assert len(recs) == 12
    st = serve.summarize(recs, 0.5)
    assert st["blocks"] == 12
    # request 4 failed alone; the others ran their full lifetime
    r4 = [r for r in sch.finished if r.rid == 4][0]
    assert r4.failed and "admission" in r4.failed
    for r in sch.finished:
        if r.rid != 4:
            assert r.failed is None and r.blocks_done == r.lifetime
    # footprint never exceeded the budget at any block
    for rec in recs:
        assert sum(fp(r) for r in reqs if r.rid in rec.active) <= budget
    # each request's per-block output equals the request run alone on that block
    for r in reqs:
        if r.rid == 4:
            continue
        W = oracle.weights(pos, r.dirs, freqs)
        for k, got in ex.out[r.rid].items():
            w = synth.Workload("t", 77, 5, 2, 0, T, I, pos, np.zeros((0, 3)), freqs)
            x = np.stack([synth.channel_voltages(500 + k + 1, c, T, pos, freqs[c]) for c in range(2)])
            assert np.array_equal(got, oracle.beamform(W, x, I))


def test_footprint_formula():
    # FP16, N=256, C=1024, 2048 beams, T=8192, I=64: 4 GiB of weights + 2 x 1 GiB outputs
    f = serve.footprint_bytes(2048, 256, 1024, 8192, 64, "fp16")
    assert f == 1024 * 2048 * 2 * 512 * 2 + 2 * 1024 * 2048 * 128 * 4


def test_poisson_block_arrivals_release_and_latency():
    """Blocks are released no earlier than their (seeded Poisson) arrival
    times and latency is measured from arrival."""
    period = 0.524288
    arr = synth.serve_block_arrivals(12, period, pace=400.0)
    assert np.all(np.diff(arr) > 0) and arr[0] > 0
    # same seed, same times; the mean gap follows period / pace
    assert np.array_equal(arr, synth.serve_block_arrivals(12, period, pace=400.0))
    long = synth.serve_block_arrivals(4000, period, pace=1.0)
    assert abs(np.mean(np.diff(long)) / period - 1.0) < 0.06
    pos = synth.line_positions(4, 10.0)
    freqs = np.array([401e6, 405e6])
    ex = FakeExecutor(pos, freqs, 32, 4)
    sch = serve.Scheduler(1 << 30, lambda r: 1)
    reqs = [serve.Request(0, synth.random_dirs(3, np.random.default_rng(2)), lifetime=None)]
    recs = serve.serve(ex, sch, reqs, n_blocks=12, block_period_s=period, arrivals=arr)
    for rec, a in zip(recs, arr):
        assert rec.arrival_s == pytest.approx(a)
        assert rec.done_s >= rec.arrival_s
    assert len(ex.launches) == 12


class TimedEvent:
    """Completes at a known host time (perf_counter seconds)."""

    def __init__(self, done_at):
        self.done_at = done_at

    def query(self):
        return time.perf_counter() >= self.done_at

    def synchronize(self):
        dt = self.done_at - time.perf_counter()
        if dt > 0:
            time.sleep(dt)


class TimedExecutor:
    """A device that runs blocks one after another, block k taking work_s[k]
    seconds from when it is enqueued or the previous block ends."""

    def __init__(self, work_s):
        self.ring = [None, None]
        self.work_s = list(work_s)
        self.busy_until = 0.0
        self.k = 0

    def admit(self, r):
        pass

    def retire(self, r):
        pass

    def run_block(self, ids, slot, parity):
        start = max(time.perf_counter(), self.busy_until)
        self.busy_until = start + self.work_s[self.k]
        self.k += 1
        return TimedEvent(self.busy_until)


def _timed_run(work_s, gap_s):
    ex = TimedExecutor(work_s)
    sch = serve.Scheduler(1 << 30, lambda r: 1)
    reqs = [serve.Request(0, np.zeros((4, 3)), lifetime=None)]
    arrivals = [gap_s * (k + 1) for k in range(len(work_s))]
    recs = serve.serve(ex, sch, reqs, n_blocks=len(work_s), block_period_s=gap_s,
                       arrivals=arrivals)
    return recs


def test_latency_is_completion_minus_arrival():
    """A 5 ms block arriving every 50 ms has about 5 ms of latency: the
    completion is stamped when the block ends, not when the host next waits
    for its ring slot (which comes only after the next arrival)."""
    recs = _timed_run([0.005] * 8, 0.05)
    lat = np.array([r.latency_ms for r in recs])
    assert np.all(lat >= 4.5), lat
    assert np.median(lat) < 20.0, lat
    st = serve.summarize(recs, 0.05)
    assert st["deadline_misses"] == 0 and st["deadline_ms"] == pytest.approx(50.0)


def test_deadline_misses_counted():
    """One 120 ms block among 5 ms ones (50 ms period): it misses its
    deadline, so does the next block (queued behind it), the one after
    recovers."""
    recs = _timed_run([0.005, 0.005, 0.120, 0.005, 0.005, 0.005], 0.05)
    lat = [r.latency_ms for r in recs]
    st = serve.summarize(recs, 0.05)
    assert st["deadline_misses"] == 2, lat
    assert lat[2] > 110 and lat[3] > 50 and lat[4] < 45, lat
    assert st["deadline_miss_frac"] == pytest.approx(2 / 6)


def test_summarize_deadline_from_records():
    recs = [serve.BlockRecord(k, [0], 4, arrival_s=0.1 * k, done_s=0.1 * k + d)
            for k, d in enumerate([0.01, 0.2, 0.05, 0.3])]
    st = serve.summarize(recs, 0.1)
    assert st["deadline_misses"] == 2
    st = serve.summarize(recs, 0.1, deadline_s=0.25)
    assert st["deadline_misses"] == 1
    assert st["p50_block_ms"] == pytest.approx(125.0)


class RingExecutor(TimedExecutor):
    """TimedExecutor with a ring of `slots` voltage slots and as many output
    buffers per request; records which slot and output buffer each block used
    and how many blocks were in flight when it was enqueued."""

    def __init__(self, work_s, slots):
        super().__init__(work_s)
        self.ring = [None] * slots
        self.n_out = slots
        self.used = []
        self.events = []

    def run_block(self, ids, slot, out_slot):
        now = time.perf_counter()
        in_flight = sum(1 for e in self.events if e.done_at > now)
        self.used.append((slot, out_slot, in_flight))
        ev = super().run_block(ids, slot, out_slot)
        self.events.append(ev)
        return ev


@pytest.mark.parametrize("slots", [2, 3])
def test_ring_slots_bound_blocks_in_flight_and_output_buffers(slots):
    """Block k reads ring slot k % slots and writes each request's output
    buffer k % slots; blocks released at once never have more than `slots`
    in flight (the host waits for block k - slots before enqueuing block k),
    so no block overwrites a slot or an output buffer still in use."""
    ex = RingExecutor([0.01] * 9, slots)
    sch = serve.Scheduler(1 << 30, lambda r: 1)
    reqs = [serve.Request(0, np.zeros((4, 3)), lifetime=None)]
    serve.serve(ex, sch, reqs, n_blocks=9, block_period_s=0.5)
    assert [(s, o) for s, o, _ in ex.used] == [(k % slots, k % slots) for k in range(9)]
    assert max(n for _, _, n in ex.used) <= slots - 1
    assert max(n for _, _, n in ex.used) == slots - 1  # the ring is used in full
