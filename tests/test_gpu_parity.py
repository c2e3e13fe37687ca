"""GPU parity: the HIP path through the C ABI against the FP64 oracle on
the same seeded inputs.

Tolerances (power, per-beam normwise and element-wise with near-null
samples scaled by their beam's mean power): FP32 path 1e-5, FP16 path 2e-3
(the stated targets); BF16 is measured against 1e-2 (its 8-bit significand
puts weight rounding alone near 2e-3).  Integer-exact inputs must match
bit for bit in every precision.
"""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity, round_to, run_plan

pytestmark = pytest.mark.gpu
TOL = {"fp32": 1e-5, "fp16": 2e-3, "bf16": 1e-2}


def _announce(msg):
    print(msg, flush=True)


# --- weights ---------------------------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_weights_match_rounded_oracle(gpu, prec):
    _announce(f"weights {prec}")
    g = np.random.default_rng(11)
    cases = [synth.small(),
             synth.Workload("wide", 0, 48, 8, 37, 16, 1, synth.disc_positions(48, 250.0, g),
                            synth.random_dirs(37, g), np.linspace(400e6, 416e6, 8))]
    for w in cases:
        plan = bf.Plan(w.n_ant, w.n_chan, w.n_beams, 16, 1, precision=prec)
        plan.set_weights(w.pos, w.dirs, w.freqs)
        got = plan.get_weights()
        ref = round_to(oracle.weights(w.pos, w.dirs, w.freqs), prec)
        ulp = {"fp32": 2.0 ** -23, "fp16": 2.0 ** -10, "bf16": 2.0 ** -7}[prec]
        d = np.maximum(np.abs(got.real - ref.real), np.abs(got.imag - ref.imag))
        # at most one unit in the last place (phase rounding of ~1e-12 rad can
        # move a value across a rounding boundary), and almost always equal
        assert d.max() <= ulp, (prec, d.max())
        assert np.mean(d == 0) > 0.999, (prec, np.mean(d == 0))
        plan.destroy()


# --- the small configuration, full size -------------------------------------

def test_small_fp32_full(gpu):
    _announce("small fp32 full")
    w = synth.small()
    x = w.voltages()
    with bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, w.integration) as plan:
        plan.set_weights(w.pos, w.dirs, w.freqs)
        got = run_plan(plan, x, gpu)
    ref = oracle.beamform(oracle.weights(w.pos, w.dirs, w.freqs), x, 1)
    st = assert_parity(got, ref, TOL["fp32"], "small fp32")
    _announce(f"  {st}")
    # beam 0 is steered at the tone: mean power N^2 |s|^2 + N * 2 sigma^2
    # (coherent tone plus incoherent noise) = 32^2 * 32^2 + 32 * 512
    expect = 32 ** 2 * 32 ** 2 + 32 * 2 * 16 ** 2
    assert abs(got[:, 0].mean() / expect - 1) < 0.02


# --- precision forms (512 beams) --------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_precision_forms(gpu, prec):
    _announce(f"precision form {prec}")
    w = synth.precision()
    chans = [0, 17, 64, 101, 127]
    x = w.voltages()
    with bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, 1, precision=prec) as plan:
        plan.set_weights(w.pos, w.dirs, w.freqs)
        got = run_plan(plan, x, gpu)[chans]
        wq = plan.get_weights()[chans]
    W64 = oracle.weights(w.pos, w.dirs, w.freqs[chans])
    ref = oracle.beamform(W64, x[chans], 1)
    st = assert_parity(got, ref, TOL[prec], f"precision {prec}")
    _announce(f"  vs FP64 oracle: {st}")
    # with the same rounded weights only FP32 accumulation differs
    ref_q = oracle.beamform(wq, x[chans], 1)
    st_q = assert_parity(got, ref_q, 1e-5, f"precision {prec} (rounded weights)")
    _announce(f"  vs oracle on the rounded weights: {st_q}")


# --- paper scale, full size, sampled channels ---------------------------------

@pytest.fixture(scope="module")
def paper_block():
    """The paper-scale block (4.29 GB of int8 voltages), generated once."""
    w = synth.paper()
    return w, w.voltages(workers=16)


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_paper_scale_sampled(gpu, paper_block, prec):
    """The bench's workload and launch: full block, the tile the tile cache
    gives the plan at creation (the one bench.py times), five seeded
    channels against the FP64 oracle."""
    import torch
    w, x = paper_block
    chans = [0, 511, 1023] + list(synth.rng("paper", "check").choice(1024, 2, replace=False))
    with bf.Plan(w.n_ant, w.n_chan, w.n_beams, w.n_samples, w.integration, precision=prec) as plan:
        info = plan.info()
        _announce(f"paper scale {prec} (4.29 GB input), tile {plan.tile()} "
                  f"tuned={info['tile_tuned']}")
        assert info["tile_tuned"] == 1, "the tile cache has no entry for the paper block"
        plan.set_weights(w.pos, w.dirs, w.freqs)
        xd = torch.from_numpy(x).to(gpu)
        p = torch.full((w.n_chan, w.n_beams, w.n_samples // w.integration), float("nan"),
                       dtype=torch.float32, device=gpu)
        plan.run(xd, p)
        torch.cuda.synchronize()
        assert not bool(torch.isnan(p).any()), "some output was never written"
        got = p[chans].cpu().numpy()
        del xd, p
    ref = oracle.beamform(oracle.weights(w.pos, w.dirs, w.freqs[chans]), x[chans], w.integration)
    st = assert_parity(got, ref, TOL[prec], f"paper {prec}")
    _announce(f"  {st}")


# --- ragged and odd shapes ---------------------------------------------------

RAGGED = [  # N, C, B, T, I
    (1, 2, 1, 16, 1), (3, 3, 5, 48, 3), (5, 2, 17, 80, 5), (17, 2, 33, 96, 2),
    (33, 1, 20, 100, 4), (8, 2, 7, 200, 8), (16, 3, 16, 1024, 16), (32, 2, 130, 1040, 16),
    (64, 2, 40, 4096, 64), (40, 1, 9, 3000, 1), (128, 1, 24, 512, 2), (256, 1, 20, 256, 16),
    (24, 2, 50, 1344, 7), (32, 1, 3, 17, 17), (2, 1, 2, 12, 12),
]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("shape", RAGGED, ids=[f"N{s[0]}C{s[1]}B{s[2]}T{s[3]}I{s[4]}" for s in RAGGED])
def test_ragged_shapes(gpu, shape, prec):
    N, C, B, T, I = shape
    _announce(f"ragged {shape} {prec}")
    g = np.random.default_rng(hash(shape) & 0xFFFF)
    pos = synth.disc_positions(N, 200.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.linspace(400e6, 416e6, C)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, dirs, freqs)
        got = run_plan(plan, x, gpu)
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), x, I)
    assert_parity(got, ref, TOL[prec], f"{shape} {prec}")


# --- register-resident pipelined form ------------------------------------------
# Shapes the pipelined unit form serves (2N a multiple of 16, every K chunk in
# registers, I == 1 or a multiple of the row-tile count, T/I a multiple of 4;
# FP32 with one beam tile per pass and 2N <= 64),
# with beam counts that leave a partial last beam range, so pipelined and
# general units share one launch.  Checked against the oracle, and bit for bit
# against a streaming tile, which never takes the pipelined form (both sum each
# window's samples in time order).  N = 24 leaves the last K slice past 2N,
# which the pipelined form reads as zeros.

FAST = [  # N, C, B, T, I
    (8, 2, 130, 512, 4), (16, 2, 128, 1024, 8), (32, 3, 144, 960, 12), (32, 2, 256, 1280, 20),
    (64, 2, 136, 2048, 64), (32, 2, 128, 1024, 1), (24, 1, 200, 768, 1),
]


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("shape", FAST, ids=[f"N{s[0]}C{s[1]}B{s[2]}T{s[3]}I{s[4]}" for s in FAST])
def test_pipelined_form(gpu, shape, prec):
    N, C, B, T, I = shape
    _announce(f"pipelined form {shape} {prec}")
    g = np.random.default_rng(sum(shape) * 7 + len(prec))
    pos = synth.disc_positions(N, 150.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.linspace(401e6, 415e6, C)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    if prec == "fp32":
        resident = (4, 4, 1, 1, 4) if 2 * N <= 64 else (4, 8, 1, 2, 4)
    else:
        resident = (4, 8, 1, 1 if 2 * N <= 64 else 2, 4)
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, dirs, freqs)
        plan.set_tile(*resident)
        got = run_plan(plan, x, gpu)
        plan.set_tile(4, 8, 2, 0, 4)
        streamed = run_plan(plan, x, gpu)
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), x, I)
    assert_parity(got, ref, TOL[prec], f"{shape} {prec}")
    assert np.array_equal(got, streamed), shape


# --- integer-exact weights: bit-exact in every precision ------------------------

@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_integer_exact_bitwise(gpu, prec):
    _announce(f"integer exact {prec}")
    g = np.random.default_rng(8)
    N, C, B, T, I = 32, 3, 40, 512, 16
    units = np.array([1, -1, 1j, -1j])
    W = units[g.integers(0, 4, (C, B, N))]
    x = g.integers(-7, 8, (C, T, N, 2)).astype(np.int8)
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights_raw(W)
        got = run_plan(plan, x, gpu)
    ref = oracle.beamform(W, x, I)
    assert np.array_equal(got.astype(np.float64), ref)


# --- determinism, tile invariance ---------------------------------------------

@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_deterministic_and_tile_invariant(gpu, prec):
    _announce(f"tile invariance {prec}")
    g = np.random.default_rng(9)
    N, C, B, T, I = 32, 2, 128, 4096, 16
    pos = synth.grid_positions(4, 8, 10.0, 20.0)
    dirs = synth.random_dirs(B, g)
    freqs = np.array([401e6, 415e6])
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, dirs, freqs)
        base = run_plan(plan, x, gpu)
        assert np.array_equal(base, run_plan(plan, x, gpu))
        cands = plan.tile_candidates()
        assert len(cands) >= 8
        for i, t in enumerate(cands):
            sgw = [1, 2, 3, 4][i % 4] * (2 if t[0] == 8 else 1)
            plan.set_tile(*t, sgw)
            assert np.array_equal(base, run_plan(plan, x, gpu)), (t, sgw)


# --- integration across blocks -------------------------------------------------

def test_accumulate_flag(gpu):
    _announce("accumulate")
    g = np.random.default_rng(12)
    N, C, B, T, I = 32, 2, 20, 256, 16
    pos = synth.line_positions(N)
    dirs = synth.random_dirs(B, g)
    freqs = np.array([402e6, 410e6])
    x1 = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    x2 = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    import torch
    with bf.Plan(N, C, B, T, I) as a, bf.Plan(N, C, B, T, I, accumulate=True) as b:
        a.set_weights(pos, dirs, freqs)
        b.set_weights(pos, dirs, freqs)
        p1 = run_plan(a, x1, gpu)
        p2 = run_plan(a, x2, gpu)
        acc = torch.from_numpy(p1).to(gpu)
        b.run(torch.from_numpy(x2).to(gpu), acc)
        torch.cuda.synchronize()
        assert np.array_equal(acc.cpu().numpy(), (p1 + p2).astype(np.float32))


# --- error paths ---------------------------------------------------------------

def test_error_paths(gpu):
    import torch
    with bf.Plan(4, 1, 2, 16, 1) as plan:
        x = torch.zeros((1, 16, 4, 2), dtype=torch.int8, device=gpu)
        p = torch.zeros((1, 2, 16), dtype=torch.float32, device=gpu)
        with pytest.raises(bf.BfError) as e:
            plan.run(x, p)
        assert e.value.status == bf.ERR_STATE
        with pytest.raises(bf.BfError) as e:
            plan.set_weights(np.zeros((4, 3)), np.ones((2, 3)), [400e6])
        assert e.value.status == bf.ERR_INVALID_ARG
        with pytest.raises(bf.BfError) as e:
            plan.set_weights(np.zeros((4, 3)), [[0, 0, 1], [0, 0, 1]], [-1.0])
        assert e.value.status == bf.ERR_INVALID_ARG
        plan.set_weights(np.zeros((4, 3)), [[0, 0, 1], [0, 0, 1]], [400e6])
        buf = torch.zeros(1 * 16 * 4 * 2 + 1, dtype=torch.int8, device=gpu)
        with pytest.raises(bf.BfError) as e:
            plan.run_ptr(buf.data_ptr() + 1, p.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert e.value.status == bf.ERR_INVALID_ARG
        with pytest.raises(bf.BfError) as e:
            plan.set_tile(4, 3, 1, 0, 1)
        assert e.value.status == bf.ERR_UNSUPPORTED
        plan.run(x, p)
        torch.cuda.synchronize()
        assert float(p.abs().sum()) == 0.0


# --- large arrays -----------------------------------------------------------
# Up to N = 1248 (FP16/BF16) or 608 (FP32) a work unit keeps its beams'
# weights for all K = 2N in LDS; beyond, the plan reads weight fragments
# from device memory (tile kres = -1), up to the API's N = 4096.  Checked
# against the oracle on both sides of the switch and at N = 4096, and the
# device-memory tile bit for bit against the LDS tiles where both run.

LARGE = [("fp32", 608, 0), ("fp32", 616, -1), ("fp16", 1248, 0), ("fp16", 1256, -1),
         ("bf16", 1256, -1), ("fp32", 4096, -1), ("fp16", 4096, -1), ("bf16", 4096, -1)]


@pytest.mark.parametrize("prec,n_ant,kres", LARGE, ids=[f"{p}-N{n}" for p, n, _ in LARGE])
def test_large_arrays(gpu, prec, n_ant, kres):
    print(f"large array {prec} N={n_ant}", flush=True)
    g = np.random.default_rng(n_ant + len(prec))
    C, B, T, I = 2, 20, 96, 4
    pos = synth.disc_positions(n_ant, 400.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.array([401e6, 414e6])
    x = g.integers(-128, 128, (C, T, n_ant, 2)).astype(np.int8)
    with bf.Plan(n_ant, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, dirs, freqs)
        assert plan.tile()[3] == kres
        got = run_plan(plan, x, gpu)
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), x, I)
    assert_parity(got, ref, TOL[prec], f"N={n_ant} {prec}")


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_device_memory_weights_tile_bitwise(gpu, prec):
    """At N = 256 both the LDS tiles and the device-memory tile run: same bits."""
    g = np.random.default_rng(77)
    N, C, B, T, I = 256, 2, 40, 512, 16
    pos = synth.disc_positions(N, 200.0, g)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, synth.random_dirs(B, g), np.array([402e6, 409e6]))
        base = run_plan(plan, x, gpu)
        plan.set_tile(4, 2, 2, -1, 4)
        assert np.array_equal(run_plan(plan, x, gpu), base)


def test_large_array_4bit_complex_and_batch(gpu):
    g = np.random.default_rng(4096)
    N, C, B, T = 4096, 1, 17, 64
    pos = synth.disc_positions(N, 400.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.array([405e6])
    x4 = g.integers(0, 256, (C, T, N)).astype(np.uint8)
    W = oracle.weights(pos, dirs, freqs)
    import torch
    with bf.Plan(N, C, B, T, 8, precision="fp16", input_bits=4) as plan:
        plan.set_weights(pos, dirs, freqs)
        got = run_plan(plan, x4, gpu)
        batch = bf.Batch([plan])
        with pytest.raises(bf.BfError) as e:  # the batching kernels stage weights in LDS
            batch.run([torch.from_numpy(x4).to(gpu)],
                      [torch.empty((C, B, T // 8), device=gpu)])
        assert e.value.status == bf.ERR_UNSUPPORTED
        batch.destroy()
    assert_parity(got, oracle.beamform(W, oracle.unpack4(x4), 8), TOL["fp16"], "N=4096 4-bit")
    with bf.Plan(N, C, B, T, 1, precision="fp16", output="complex") as plan:
        plan.set_weights(pos, dirs, freqs)
        plan.set_output_scale(1.0 / 64)
        p = torch.empty(plan.p_shape, dtype=torch.float16, device=gpu)
        plan.run(torch.from_numpy(oracle.unpack4(x4)).to(gpu), p)
        torch.cuda.synchronize()
        o = p.cpu().numpy().astype(np.float64)
    got_c = o[..., 0] + 1j * o[..., 1]
    ref_c = oracle.beams(W, oracle.unpack4(x4)) / 64
    rms = np.sqrt(np.mean(np.abs(ref_c) ** 2, axis=-1, keepdims=True))
    assert np.max(np.abs(got_c - ref_c) / (np.abs(ref_c) + rms)) <= 2e-3
