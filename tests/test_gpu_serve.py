"""Serving form on the GPU (scaled-down serve shapes: the 16x16 array, FP16,
I=64): requests arriving and leaving while others run share each block's
launch (replayed as hipGraphs); every request's output for every block is
bitwise equal to that request run alone on the same block."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, serve, synth
from tests.gpu_util import assert_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("input_bits", [8, 4])
def test_serve_alone_equals_mix(gpu, input_bits):
    import torch
    print(f"serve mix, {input_bits}-bit blocks", flush=True)
    pos = synth.serve_array()
    C, T, I = 16, 2048, 64
    freqs = synth.channel_freqs(C, 400e6, 16e6)
    sigma = synth.SIGMA4 if input_bits == 4 else synth.SIGMA
    blocks = [synth.Workload(f"b{k}", 2000 + k, 256, C, 0, T, I, pos, np.zeros((0, 3)),
                             freqs, sigma=sigma, input_bits=input_bits).voltages()
              for k in range(2)]
    ring = [torch.from_numpy(b).to(gpu) for b in blocks]
    g = np.random.default_rng(5)
    reqs = [serve.Request(i, synth.random_dirs(int(nb), g), lifetime=int(life), arrival_block=int(a))
            for i, (nb, life, a) in enumerate([(64, 4, 0), (20, 2, 0), (100, 3, 1), (33, 5, 2),
                                                (16, 1, 3), (48, 3, 3)])]
    fp = lambda r: serve.footprint_bytes(r.n_beams, 256, C, T, I, "fp16")  # noqa: E731
    budget = fp(reqs[0]) + fp(reqs[2]) + fp(reqs[1])  # forces some requests to wait
    ex = serve.GpuExecutor(pos, freqs, T, I, "fp16", ring=ring, input_bits=input_bits)
    sch = serve.Scheduler(budget, fp)
    snaps = {}

    def grab(k, rec):
        with torch.cuda.stream(ex.stream):
            for rid in rec.active:
                snaps[(rid, k)] = ex.output(rid, k & 1).clone()

    recs = serve.serve(ex, sch, reqs, n_blocks=10, block_period_s=0.524288, on_block=grab)
    torch.cuda.synchronize()
    assert ex.graph_replays > 0 and ex.eager_launches > 0
    assert any(len(r.active) >= 2 for r in recs)
    for rec in recs:
        assert sum(fp(r) for r in reqs if r.rid in rec.active) <= budget
    assert all(r.failed is None for r in sch.finished)
    # every request ran its full lifetime
    for r in reqs:
        assert r.blocks_done == r.lifetime, (r.rid, r.blocks_done, r.lifetime)
    # alone == in the mix, bitwise, for every (request, block)
    solo = {}
    for r in reqs:
        plan = bf.Plan(256, C, r.n_beams, T, I, precision="fp16", input_bits=input_bits)
        plan.set_weights(pos, r.dirs, freqs)
        for slot in range(2):
            p = torch.empty((C, r.n_beams, T // I), device=gpu)
            plan.run(ring[slot], p)
            torch.cuda.synchronize()
            solo[(r.rid, slot)] = p.cpu().numpy()
        plan.destroy()
    for (rid, k), t in snaps.items():
        assert np.array_equal(t.cpu().numpy(), solo[(rid, k % 2)]), (rid, k)
    # and one request against the oracle on two channels
    r = reqs[2]
    x1 = oracle.unpack4(blocks[1][:2]) if input_bits == 4 else blocks[1][:2]
    ref = oracle.beamform(oracle.weights(pos, r.dirs, freqs[:2]), x1, I)
    assert_parity(solo[(r.rid, 1)][:2], ref, 2e-3, "serve fp16 vs oracle")
    ex.close()
    st = serve.summarize(recs, 0.524288)
    print(st, flush=True)


def test_serve_pcie_fed_equals_prestaged(gpu):
    """The PCIe-fed variant (every block copied from pinned host memory into
    its ring slot on a second stream, overlapped with compute) gives every
    request the same output, bitwise, as the plan run alone on that block."""
    import torch
    print("serve pcie-fed", flush=True)
    pos = synth.serve_array()
    C, T, I = 8, 1024, 64
    freqs = synth.channel_freqs(C, 400e6, 16e6)
    blocks = [synth.Workload(f"h{k}", 2100 + k, 256, C, 0, T, I, pos, np.zeros((0, 3)),
                             freqs).voltages() for k in range(2)]
    host = [torch.from_numpy(b).pin_memory() for b in blocks]
    # ring slots start as garbage: every block must arrive through the copy
    ring = [torch.full(b.shape, 77, dtype=torch.int8, device=gpu) for b in blocks]
    g = np.random.default_rng(9)
    reqs = [serve.Request(i, synth.random_dirs(nb, g), lifetime=life, arrival_block=a)
            for i, (nb, life, a) in enumerate([(40, 5, 0), (17, 3, 1), (64, 2, 2)])]
    ex = serve.GpuExecutor(pos, freqs, T, I, "fp16", ring=ring, host_blocks=host)
    sch = serve.Scheduler(1 << 34, lambda r: 1)
    snaps = {}

    def grab(k, rec):
        with torch.cuda.stream(ex.stream):
            for rid in rec.active:
                snaps[(rid, k)] = ex.output(rid, k & 1).clone()

    serve.serve(ex, sch, reqs, n_blocks=6, block_period_s=0.524288, on_block=grab)
    torch.cuda.synchronize()
    assert ex.h2d_bytes == 6 * blocks[0].nbytes
    solo = {}
    for r in reqs:
        plan = bf.Plan(256, C, r.n_beams, T, I, precision="fp16")
        plan.set_weights(pos, r.dirs, freqs)
        for slot in range(2):
            p = torch.empty((C, r.n_beams, T // I), device=gpu)
            plan.run(torch.from_numpy(blocks[slot]).to(gpu), p)
            torch.cuda.synchronize()
            solo[(r.rid, slot)] = p.cpu().numpy()
        plan.destroy()
    assert len(snaps) >= 6
    for (rid, k), t in snaps.items():
        assert np.array_equal(t.cpu().numpy(), solo[(rid, k % 2)]), (rid, k)
    # and what arrived through the copy stream against the FP64 oracle: the
    # first request's output on its first block (slot 0), two channels
    r = reqs[0]
    ref = oracle.beamform(oracle.weights(pos, r.dirs, freqs[:2]), blocks[0][:2], I)
    assert_parity(snaps[(r.rid, 0)].cpu().numpy()[:2], ref, 2e-3, "pcie-fed serve vs oracle")
    ex.close()


@pytest.mark.slow
def test_serve_real_shape(gpu):
    """The serving workload at its real shape: the 256-antenna 16x16 grid,
    blocks of 1024 channels x 8192 samples, I = 64, FP16, the first requests
    of the seeded request stream (arrivals compressed so that they overlap),
    the table kernel replayed from a captured graph, tiles from the tile cache
    where it has them.  Every request's output on every block equals the plan
    run alone on that block (bitwise, compared on the device), and one
    request's sampled channels match the FP64 oracle."""
    import torch
    from paper_1412_4907_amd import tune
    C, T, I = 1024, 8192, 64
    pos = synth.serve_array()
    freqs = synth.channel_freqs(C, 400e6, 16e6)
    print("serve real shape: generating 2 blocks of 4.29 GB", flush=True)
    blocks = [synth.serve_block(k).voltages(workers=16) for k in range(2)]
    ring = [torch.from_numpy(b).to(gpu) for b in blocks]
    spec = synth.serve_requests(64)[:4]
    reqs = [serve.Request(i, d, lifetime=max(1, min(int(life), 3)), arrival_block=i // 2)
            for i, (_, nb, life, d) in enumerate(spec)]
    print("requests (beams, lifetime, arrival):",
          [(r.n_beams, r.lifetime, r.arrival_block) for r in reqs], flush=True)
    ex = serve.GpuExecutor(pos, freqs, T, I, "fp16", ring=ring)
    sch = serve.Scheduler(200 << 30, lambda r: serve.footprint_bytes(r.n_beams, 256, C, T, I,
                                                                        "fp16"))
    snaps = {}

    def grab(k, rec):
        with torch.cuda.stream(ex.stream):
            for rid in rec.active:
                snaps[(rid, k)] = ex.output(rid, k & 1).clone()

    recs = serve.serve(ex, sch, reqs, n_blocks=5, block_period_s=0.524288, on_block=grab)
    torch.cuda.synchronize()
    st = serve.summarize(recs, 0.524288)
    print({k: st[k] for k in ("rtf", "p50_block_ms", "p99_block_ms", "deadline_misses")},
          f"replays {ex.graph_replays}, tuned admissions {ex.tuned_admissions}", flush=True)
    assert ex.graph_replays > 0 and ex.eager_launches == 1
    assert any(len(r.active) >= 2 for r in recs)
    assert all(r.failed is None for r in sch.finished)
    for r in reqs:
        assert r.blocks_done == r.lifetime, (r.rid, r.blocks_done, r.lifetime)
    # every admission that the tile cache covers ran the cached batching tile
    cache = tune.load_cache()
    covered = 0
    for r in reqs:
        with bf.Plan(256, C, r.n_beams, T, I, precision="fp16") as probe:
            covered += probe.tune_key(batch=True) in cache
    assert ex.tuned_admissions == covered
    # alone == in the mix, bitwise, on the device
    for r in reqs:
        plan = bf.Plan(256, C, r.n_beams, T, I, precision="fp16")
        plan.set_weights(pos, r.dirs, freqs)
        solo = []
        for slot in range(2):
            p = torch.empty((C, r.n_beams, T // I), device=gpu)
            plan.run(ring[slot], p)
            solo.append(p)
        torch.cuda.synchronize()
        for (rid, k), t in snaps.items():
            if rid == r.rid:
                assert torch.equal(t, solo[k % 2]), (rid, k)
        if r.rid == min(reqs, key=lambda q: q.n_beams).rid:
            chans = [3, 700]
            ref = oracle.beamform(oracle.weights(pos, r.dirs, freqs[chans]), blocks[0][chans], I)
            assert_parity(solo[0][chans].cpu().numpy(), ref, 2e-3, "serve real shape vs oracle")
            print(f"request {r.rid} ({r.n_beams} beams) matches the oracle on channels {chans}",
                  flush=True)
        del solo
        plan.destroy()
    ex.close()
