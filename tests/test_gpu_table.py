"""Table batch on the GPU: one hipGraph captured around bf_table_run,
replayed while the set table stored before each replay changes (which plans,
which voltage and output buffers).  Every replay's output must equal each
plan run alone, bit for bit; eager work and synchronisations run between
the replays, and outputs are poisoned before each one."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity

pytestmark = pytest.mark.gpu


def _setup(gpu, prec, shapes, N=32, I=16):
    import torch
    g = np.random.default_rng(31)
    pos = synth.grid_positions(4, 8, 10.0, 20.0) if N == 32 else synth.disc_positions(N, 150.0, g)
    plans, xs, solo, freqs_all, dirs_all, xh = [], [], [], [], [], []
    for C, B, T in shapes:
        dirs = synth.random_dirs(B, g)
        freqs = np.linspace(402e6, 414e6, C)
        x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
        plan = bf.Plan(N, C, B, T, I, precision=prec)
        plan.set_weights(pos, dirs, freqs)
        xd = torch.from_numpy(x).to(gpu)
        p = torch.empty((C, B, T // I), device=gpu)
        plan.run(xd, p)
        torch.cuda.synchronize()
        plans.append(plan); xs.append(xd); solo.append(p.cpu().numpy())
        freqs_all.append(freqs); dirs_all.append(dirs); xh.append(x)
    return pos, plans, xs, solo, freqs_all, dirs_all, xh


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_table_graph_replays_follow_the_table(gpu, prec):
    import torch
    print(f"table graph {prec}", flush=True)
    shapes = [(8, 128, 2048), (5, 40, 1024), (3, 300, 4096), (6, 16, 512)]
    pos, plans, xs, solo, freqs, dirs, xh = _setup(gpu, prec, shapes)
    outs = [[torch.empty((C, B, T // 16), device=gpu) for _ in range(2)] for C, B, T in shapes]
    table = bf.Table(32, 16, prec)
    s = torch.cuda.Stream()
    sets = [[0, 1], [2], [3, 1, 0, 2], [1], [2, 0], []]
    graph = None
    with torch.cuda.stream(s):
        for k, ids in enumerate(sets):
            par = k & 1
            for i in range(len(plans)):
                outs[i][par].fill_(float("nan"))
            table.set([plans[i] for i in ids], [xs[i] for i in ids],
                      [outs[i][par] for i in ids], stream=s)
            if graph is None:
                table.run(stream=s)  # eager first run, then capture the same launch
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=s):
                    table.run(stream=s)
            else:
                graph.replay()
            s.synchronize()
            # eager work between replays
            junk = torch.randn(1 << 20, device=gpu, dtype=torch.float32).sum()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for i in ids:
                got = outs[i][par].cpu().numpy()
                assert np.array_equal(got, solo[i]), (k, i)
            for i in set(range(len(plans))) - set(ids):
                assert torch.isnan(outs[i][par]).all(), (k, i)  # not in this table: untouched
    # one set against the oracle on two channels
    i = 2
    ref = oracle.beamform(oracle.weights(pos, dirs[i], freqs[i][:2]), xh[i][:2], 16)
    assert_parity(solo[i][:2], ref, 2e-3 if prec == "fp16" else 1e-5, "table set vs oracle")
    table.destroy()
    for p in plans:
        p.destroy()


def test_table_rejects_mismatched_plans(gpu):
    import torch
    table = bf.Table(32, 16, "fp16")
    plan = bf.Plan(32, 2, 16, 256, 8, precision="fp16")  # another integration
    plan.set_weights(synth.grid_positions(4, 8, 10.0, 20.0),
                     synth.random_dirs(16, np.random.default_rng(1)), np.array([401e6, 402e6]))
    x = torch.zeros((2, 256, 32, 2), dtype=torch.int8, device=gpu)
    p = torch.empty((2, 16, 32), device=gpu)
    with pytest.raises(bf.BfError) as e:
        table.set([plan], [x], [p])
    assert e.value.status == bf.ERR_UNSUPPORTED
    table.destroy()
    plan.destroy()


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_eight_wave_table_sets_sharing_one_block(gpu, prec):
    """Sets that read one voltage block (the serving case) run the
    eight-wave table kernel, whose queues then go channel by channel over
    all sets; the block is short (8 store groups per channel), so each set's
    store groups per wave are capped to reach all eight waves.  Each set's
    output equals the set run alone, bit for bit, whether the sets share the
    block or not; one set is checked against the oracle."""
    import torch
    print(f"eight-wave table, shared block, {prec}", flush=True)
    N, C, T, I = 160, 9, 8192, 64  # K = 320: five chunks, eight-wave form
    g = np.random.default_rng(47)
    pos = synth.disc_positions(N, 150.0, g)
    freqs = np.linspace(402e6, 414e6, C)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    xd = torch.from_numpy(x).to(gpu)
    x2 = torch.from_numpy(g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)).to(gpu)
    beams = [75, 16, 130, 33]
    plans, dirs, solo = [], [], []
    for b in beams:
        d = synth.random_dirs(b, g)
        p = bf.Plan(N, C, b, T, I, precision=prec)
        p.set_weights(pos, d, freqs)
        plans.append(p)
        dirs.append(d)
    for xin, tag in ((xd, "shared"), (x2, "shared, other block")):
        solo = []
        for p, b in zip(plans, beams):
            out = torch.empty((C, b, T // I), device=gpu)
            p.run(xin, out)
            solo.append(out)
        torch.cuda.synchronize()
        table = bf.Table(N, I, prec)
        outs = [torch.full((C, b, T // I), float("nan"), device=gpu) for b in beams]
        table.set(plans, [xin] * len(plans), outs)
        table.run()
        torch.cuda.synchronize()
        for i in range(len(plans)):
            assert torch.equal(outs[i], solo[i]), (tag, i)
        table.destroy()
    # sets on different blocks: the set-major queue order
    table = bf.Table(N, I, prec)
    xs = [xd, x2, xd, x2]
    outs = [torch.full((C, b, T // I), float("nan"), device=gpu) for b in beams]
    table.set(plans, xs, outs)
    table.run()
    torch.cuda.synchronize()
    for i, (p, b) in enumerate(zip(plans, beams)):
        ref = torch.empty((C, b, T // I), device=gpu)
        p.run(xs[i], ref)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], ref), ("mixed blocks", i)
    # one set against the oracle on two channels
    ref = oracle.beamform(oracle.weights(pos, dirs[0], freqs[:2]), x[:2], I)
    assert_parity(outs[0][:2].cpu().numpy(), ref, 2e-3 if prec == "fp16" else 1e-2,
                  "eight-wave table set vs oracle")
    table.destroy()
    for p in plans:
        p.destroy()
