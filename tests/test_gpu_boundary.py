"""The C ABI's handle lifetime, argument checks and tile cache on the GPU:
destroying a plan, batch or table never waits for another stream's work, and
a handle's memory outlives its own queued work; bf_run rejects overlapping voltage and
output buffers, and plans take their tile from the loaded tile cache at
creation (bf_tune_load, bf_tune_key, bf_plan_apply_tuned)."""
import json

import numpy as np
import pytest

from paper_1412_4907_amd import bf, synth, tune

pytestmark = pytest.mark.gpu


def _busy_plan(torch, gpu, stream):
    """A large FP32 plan (about 16 ms per run) with its buffers, set up and
    warmed on `stream` before any timing-sensitive check."""
    N, C, B, T, I = 32, 1024, 128, 65536, 16
    plan = bf.Plan(N, C, B, T, I)
    w = synth.paper()
    plan.set_weights(w.pos, w.dirs, w.freqs, stream=stream)
    with torch.cuda.stream(stream):
        x = torch.randint(-128, 128, (C, T, N, 2), dtype=torch.int8, device=gpu)
        p = torch.empty((C, B, T // I), dtype=torch.float32, device=gpu)
    plan.run(x, p, stream=stream)
    stream.synchronize()
    return plan, (x, p)


def _busy_stream_work(torch, stream, plan, bufs, runs=24):
    """Enqueue about 0.4 s of beamforming on `stream` and return the event
    recorded after it.  Nothing here allocates, so no implicit device-wide
    synchronisation can drain the stream early."""
    for _ in range(runs):
        plan.run(*bufs, stream=stream)
    ev = torch.cuda.Event()
    ev.record(stream)
    return ev


def _small(gpu, torch, stream):
    g = np.random.default_rng(5)
    N, C, B, T, I = 16, 4, 20, 256, 4
    plan = bf.Plan(N, C, B, T, I, precision="fp16")
    plan.set_weights(synth.disc_positions(N, 50.0, g), synth.random_dirs(B, g),
                     np.linspace(401e6, 409e6, C), stream=stream)
    with torch.cuda.stream(stream):
        x = torch.randint(-128, 128, (C, T, N, 2), dtype=torch.int8, device=gpu)
        p = torch.empty((C, B, T // I), dtype=torch.float32, device=gpu)
    return plan, x, p


def test_destroy_does_not_wait_for_other_streams(gpu):
    """Handles whose own work has completed are destroyed while about 0.4 s
    of another stream's work is queued: every destroy returns with that work
    still pending.  (The handles' own runs finish before the other work is
    enqueued, since two streams may share one hardware queue.)"""
    import torch
    print("destroy vs another stream's work", flush=True)
    busy, own = torch.cuda.Stream(), torch.cuda.Stream()
    big, bufs = _busy_plan(torch, gpu, busy)
    plan, x, p = _small(gpu, torch, own)
    p2, x2, o2 = _small(gpu, torch, own)
    batch = bf.Batch([p2])
    tab = bf.Table(16, 4, "fp16")
    tab.set([p2], [x2], [o2], stream=own)
    plan.run(x, p, stream=own)
    batch.run([x2], [o2], stream=own)
    tab.run(stream=own)
    torch.cuda.synchronize()

    busy_done = _busy_stream_work(torch, busy, big, bufs)
    plan.destroy()
    assert not busy_done.query(), "bf_plan_destroy waited for another stream's work"
    batch.destroy()
    tab.destroy()
    p2.destroy()
    assert not busy_done.query(), "a batch or table destroy waited for another stream's work"
    torch.cuda.synchronize()
    big.destroy()
    del bufs


def test_destroy_keeps_memory_until_own_work_is_done(gpu):
    """A plan destroyed while its run is still queued: the run must still read
    the plan's weights, so its output equals the same run made earlier, even
    though a new plan of the same size is created and given other weights
    before that run executes."""
    import torch
    print("destroy with the plan's own run still queued", flush=True)
    busy, side = torch.cuda.Stream(), torch.cuda.Stream()
    big, bufs = _busy_plan(torch, gpu, busy)
    plan, x, p = _small(gpu, torch, busy)
    plan.run(x, p, stream=busy)
    torch.cuda.synchronize()
    ref = p.cpu().numpy()
    p.fill_(float("nan"))
    torch.cuda.synchronize()
    _busy_stream_work(torch, busy, big, bufs)
    plan.run(x, p, stream=busy)  # queued behind the long work
    ran = torch.cuda.Event()
    ran.record(busy)
    assert not ran.query()
    plan.destroy()
    other, _, _ = _small(gpu, torch, side)
    g = np.random.default_rng(9)
    other.set_weights(synth.disc_positions(16, 50.0, g), synth.random_dirs(20, g),
                      np.linspace(401e6, 409e6, 4), stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    assert np.array_equal(p.cpu().numpy(), ref), "the destroyed plan's queued run lost its weights"
    other.destroy()
    big.destroy()
    del bufs


def test_run_rejects_overlapping_buffers(gpu):
    import torch
    print("overlapping X / P rejected", flush=True)
    N, C, B, T, I = 8, 2, 16, 64, 1
    g = np.random.default_rng(1)
    with bf.Plan(N, C, B, T, I) as plan:
        plan.set_weights(synth.disc_positions(N, 30.0, g), synth.random_dirs(B, g),
                         np.array([401e6, 402e6]))
        xbytes, pbytes = C * T * N * 2, C * B * T * 4
        buf = torch.zeros(xbytes + pbytes + 64, dtype=torch.uint8, device=gpu)
        base = buf.data_ptr()
        s = torch.cuda.current_stream().cuda_stream
        # output starting inside the voltages, and voltages inside the output
        for xo, po in ((0, xbytes - 16), (pbytes - 16, 0), (0, 0)):
            with pytest.raises(bf.BfError) as e:
                plan.run_ptr(base + xo, base + po, s)
            assert e.value.status == bf.ERR_INVALID_ARG
        # adjacent ranges are fine
        plan.run_ptr(base, base + xbytes, s)
        torch.cuda.synchronize()
        # the batch form checks every set's output against every set's input
        x = buf[:xbytes].view(torch.int8).view(C, T, N, 2)
        pa = buf[16:16 + pbytes].view(torch.float32).view(C, B, T)
        batch = bf.Batch([plan])
        with pytest.raises(bf.BfError) as e:
            batch.run([x], [pa])
        assert e.value.status == bf.ERR_INVALID_ARG
        batch.destroy()


def test_tile_cache_applied_at_creation(gpu, tmp_path):
    print("tile cache at plan creation", flush=True)
    N, C, B, T, I = 32, 64, 40, 4096, 16
    with bf.Plan(N, C, B, T, I, precision="fp16") as plan:
        key = plan.tune_key()
        assert key == "gfx950/p1/N32/B~32/I16/C~64/T~4096"
        assert plan.tune_key(batch=True) == key + "/batch"
        default = plan.tile()
        assert plan.info()["tile_tuned"] == 0
    # a cache naming another legal tile for this shape (and one for the batch kernel)
    alt = (4, 4, 2, 0, 8) if default[:4] != (4, 4, 2, 0) else (4, 2, 2, 0, 8)
    path = tmp_path / "cache.json"
    path.write_text(json.dumps({key: {"tile": list(alt), "ms": 1.0},
                                key + "/batch": {"tile": [4, 1, 1, 0, 4]},
                                "gfx950/junk": {"tile": "bad"}}))
    try:
        assert bf.tune_load(str(path)) == 2
        with bf.Plan(N, C, B, T, I, precision="fp16") as plan:
            assert plan.tile() == alt and plan.info()["tile_tuned"] == 1
            plan.set_tile(*default)
            assert plan.info()["tile_tuned"] == 0
            assert plan.apply_tuned(batch=True) and plan.tile() == (4, 1, 1, 0, 4)
            assert plan.apply_tuned() and plan.tile() == alt
        # a shape the cache does not cover keeps the built-in choice
        with bf.Plan(N, C, B + 200, T, I, precision="fp16") as other:
            assert other.info()["tile_tuned"] == 0 and not other.apply_tuned()
        with pytest.raises(bf.BfError):
            bf.tune_load(str(tmp_path / "missing.json"))
        (tmp_path / "broken.json").write_text("{\"a\": [1, 2")
        with pytest.raises(bf.BfError):
            bf.tune_load(str(tmp_path / "broken.json"))
    finally:
        bf.tune_load(tune.cache_path())
