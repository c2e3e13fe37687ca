"""4-bit complex input (Sec. 2.1: the F-engine emits 4-bit two's complement
components, one antenna sample per byte) on the GPU.

The 4-bit plan must give, bit for bit, what the int8 plan gives on the same
samples widened to int8 pairs (the kernel widens the nibbles to int8 values
scaled by 16 and scales the power back by 1/256, both exact), and match the
FP64 oracle on its own decoding of the bytes to the precision form's
tolerance.  Covers every integration mode, register-resident and streamed K,
ragged beams and windows, every compiled tile, and the batching and table
forms."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity, run_plan

pytestmark = pytest.mark.gpu
TOL = {"fp32": 1e-5, "fp16": 2e-3, "bf16": 1e-2}

SHAPES = [  # N, C, B, T, I
    (32, 2, 128, 1024, 1), (32, 2, 130, 2048, 16), (8, 3, 40, 512, 2), (16, 2, 33, 960, 3),
    (64, 2, 136, 2048, 64), (24, 2, 200, 768, 1), (256, 1, 40, 512, 16), (128, 2, 24, 640, 5),
    (40, 1, 9, 96, 4), (32, 1, 3, 48, 48),
]


def _case(shape, seed):
    N, C, B, T, I = shape
    g = np.random.default_rng(seed)
    pos = synth.disc_positions(N, 200.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.linspace(400e6, 416e6, C)
    x4 = g.integers(0, 256, (C, T, N)).astype(np.uint8)
    return pos, dirs, freqs, x4


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}C{s[1]}B{s[2]}T{s[3]}I{s[4]}" for s in SHAPES])
def test_4bit_equals_int8_and_oracle(gpu, shape, prec):
    N, C, B, T, I = shape
    print(f"4-bit {shape} {prec}", flush=True)
    pos, dirs, freqs, x4 = _case(shape, sum(shape) + len(prec))
    x8 = oracle.unpack4(x4)
    with bf.Plan(N, C, B, T, I, precision=prec, input_bits=4) as p4, \
            bf.Plan(N, C, B, T, I, precision=prec) as p8:
        p4.set_weights(pos, dirs, freqs)
        p8.set_weights(pos, dirs, freqs)
        got = run_plan(p4, x4, gpu)
        t4 = p4.tile()
        p8.set_tile(*t4)  # the same tile, so the same summation order
        wide = run_plan(p8, x8, gpu)
    assert np.array_equal(got, wide), (shape, prec, t4)
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), x8, I)
    assert_parity(got, ref, TOL[prec], f"4-bit {shape} {prec}")


@pytest.mark.parametrize("prec", ["fp16", "fp32"])
def test_4bit_every_tile_and_rails(gpu, prec):
    """Every compiled 4-bit tile gives the same bits; rail values (-8) on
    every antenna are converted exactly."""
    print(f"4-bit tiles {prec}", flush=True)
    N, C, B, T, I = 32, 2, 128, 2048, 16
    pos, dirs, freqs, x4 = _case((N, C, B, T, I), 77)
    x4[:, :64] = 0x88  # (-8, -8) on every antenna for 64 samples
    with bf.Plan(N, C, B, T, I, precision=prec, input_bits=4) as plan:
        plan.set_weights(pos, dirs, freqs)
        base = run_plan(plan, x4, gpu)
        cands = plan.tile_candidates()
        assert len(cands) >= 6
        for i, t in enumerate(cands):
            plan.set_tile(*t, [1, 2, 3, 4][i % 4])
            assert np.array_equal(base, run_plan(plan, x4, gpu)), t
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), oracle.unpack4(x4), I)
    assert_parity(base, ref, TOL[prec], f"4-bit tiles {prec}")


def test_4bit_integer_weights_bitwise(gpu):
    """Weights in {1, -1, i, -i}: every precision form is exact."""
    g = np.random.default_rng(5)
    N, C, B, T, I = 64, 2, 48, 1024, 8
    units = np.array([1, -1, 1j, -1j])
    W = units[g.integers(0, 4, (C, B, N))]
    x4 = g.integers(0, 256, (C, T, N)).astype(np.uint8)
    ref = oracle.beamform(W, oracle.unpack4(x4), I)
    for prec in ("fp32", "fp16", "bf16"):
        with bf.Plan(N, C, B, T, I, precision=prec, input_bits=4) as plan:
            plan.set_weights_raw(W)
            got = run_plan(plan, x4, gpu)
        assert np.array_equal(got.astype(np.float64), ref), prec


def test_4bit_batch_and_table(gpu):
    import torch
    print("4-bit batch + table", flush=True)
    shapes = [(32, 3, 64, 1024), (32, 2, 130, 2048), (32, 4, 16, 512)]
    plans, xs, solo, host = [], [], [], []
    for i, (N, C, B, T) in enumerate(shapes):
        pos, dirs, freqs, x4 = _case((N, C, B, T, 16), 300 + i)
        plan = bf.Plan(N, C, B, T, 16, precision="fp16", input_bits=4)
        plan.set_weights(pos, dirs, freqs)
        plans.append(plan)
        host.append(x4)
        xs.append(torch.from_numpy(x4).to(gpu))
        solo.append(run_plan(plan, x4, gpu))
    ps = [torch.full((p.C, p.B, p.windows), float("nan"), device=gpu) for p in plans]
    batch = bf.Batch(plans)
    batch.run(xs, ps)
    torch.cuda.synchronize()
    for s, p in zip(solo, ps):
        assert np.array_equal(s, p.cpu().numpy())
    batch.destroy()
    table = bf.Table(32, 16, "fp16", input_bits=4)
    for ids in ([0, 2], [1], [2, 1, 0]):
        for p in ps:
            p.fill_(float("nan"))
        table.set([plans[i] for i in ids], [xs[i] for i in ids], [ps[i] for i in ids])
        table.run()
        torch.cuda.synchronize()
        for i in ids:
            assert np.array_equal(solo[i], ps[i].cpu().numpy()), (ids, i)
    # an int8 plan does not fit a 4-bit table, nor a 4-bit plan an int8 batch
    with bf.Plan(32, 2, 16, 512, 16, precision="fp16") as p8:
        p8.set_weights(synth.grid_positions(4, 8, 10.0, 20.0),
                       synth.random_dirs(16, np.random.default_rng(1)), np.array([401e6, 402e6]))
        x8 = torch.zeros((2, 512, 32, 2), dtype=torch.int8, device=gpu)
        out = torch.empty((2, 16, 32), device=gpu)
        with pytest.raises(bf.BfError) as e:
            table.set([p8], [x8], [out])
        assert e.value.status == bf.ERR_UNSUPPORTED
        with pytest.raises(bf.BfError) as e:
            bf.Batch([plans[0], p8])
        assert e.value.status == bf.ERR_UNSUPPORTED
    table.destroy()
    for p in plans:
        p.destroy()


def test_4bit_input_checks(gpu):
    import torch
    with pytest.raises(bf.BfError) as e:
        bf.Plan(12, 1, 4, 64, 1, input_bits=4)
    assert e.value.status == bf.ERR_UNSUPPORTED
    with bf.Plan(16, 1, 4, 64, 1, input_bits=4) as plan:
        plan.set_weights(synth.line_positions(16), synth.random_dirs(4, np.random.default_rng(2)),
                         [401e6])
        p = torch.empty((1, 4, 64), device=gpu)
        with pytest.raises(ValueError):
            plan.run(torch.zeros((1, 64, 16, 2), dtype=torch.int8, device=gpu), p)
        x = torch.zeros((1, 64, 16), dtype=torch.uint8, device=gpu)
        plan.run(x, p)
        torch.cuda.synchronize()
        assert float(p.abs().sum()) == 0.0


def test_4bit_accumulate(gpu):
    """Integration across blocks (BF_ACCUMULATE) with 4-bit input: the second
    block adds into the first's output, exactly as the int8 plan does."""
    import torch
    N, C, B, T, I = 32, 2, 40, 512, 16
    pos, dirs, freqs, x4a = _case((N, C, B, T, I), 90)
    x4b = np.random.default_rng(91).integers(0, 256, (C, T, N)).astype(np.uint8)
    with bf.Plan(N, C, B, T, I, input_bits=4) as a, \
            bf.Plan(N, C, B, T, I, input_bits=4, accumulate=True) as acc, \
            bf.Plan(N, C, B, T, I, accumulate=True) as acc8:
        for p in (a, acc, acc8):
            p.set_weights(pos, dirs, freqs)
        p1 = run_plan(a, x4a, gpu)
        out = torch.from_numpy(p1).to(gpu)
        acc.run(torch.from_numpy(x4b).to(gpu), out)
        out8 = torch.from_numpy(p1).to(gpu)
        acc8.run(torch.from_numpy(oracle.unpack4(x4b)).to(gpu), out8)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, out8.cpu().numpy())
    # window w of the result is window w of block a plus window w of block b
    W = oracle.weights(pos, dirs, freqs)
    ra = oracle.beamform(W, oracle.unpack4(x4a), I)
    rb = oracle.beamform(W, oracle.unpack4(x4b), I)
    assert_parity(got, ra + rb, 1e-5, "4-bit accumulate")
