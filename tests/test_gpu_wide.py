"""The eight-wave streamed form (tiles with kres == -2; FP16/BF16, I == 1
or I a multiple of the row-tile count) against the FP64 oracle and bit for
bit against the four-wave streamed tile (4, 2, 2, 0), which accumulates every
output over the same K slices in the same order and sums each window's
samples in time order.

Shapes: the 256-antenna serving shape with a partial last beam range, an
array whose 2N is not a multiple of the 64-wide K chunk (the last chunk's
slices past 2N read as zero), I == 1 with a block length that leaves a
partial last 16-sample tile, small integrations (I = 4, 8), a work unit
with more store groups than waves, and 4-bit input (Sec. 2.1's F-engine
format)."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity, run_plan

pytestmark = pytest.mark.gpu
TOL = {"fp16": 2e-3, "bf16": 1e-2}

WIDE = [  # N, C, B, T, I
    (256, 2, 100, 2048, 64), (200, 2, 64, 1024, 16), (256, 2, 48, 1000, 1),
    (96, 2, 64, 4096, 8), (256, 1, 32, 2048, 4), (64, 3, 130, 8192, 16),
]


def _base_sgw(I, mt=4):
    """Smallest legal store groups per wave: sgw x (row tiles per store
    group) must be a multiple of MT."""
    from math import gcd
    G = 1 if I == 1 else 2 if I == 2 else 4 * ((I + 3) // 4)
    return mt // gcd(mt, G)


def _inputs(shape, seed):
    N, C, B, T, I = shape
    g = np.random.default_rng(seed)
    pos = synth.disc_positions(N, 250.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.linspace(401e6, 415e6, C)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    return pos, dirs, freqs, x


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("shape", WIDE, ids=[f"N{s[0]}C{s[1]}B{s[2]}T{s[3]}I{s[4]}" for s in WIDE])
def test_wide_form(gpu, shape, prec):
    N, C, B, T, I = shape
    print(f"wide form {shape} {prec}", flush=True)
    pos, dirs, freqs, x = _inputs(shape, sum(shape) + len(prec))
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, dirs, freqs)
        wide = [t for t in plan.tile_candidates() if t[3] == -2]
        assert wide, "no eight-wave tile offered for this shape"
        base = _base_sgw(I)
        plan.set_tile(4, 2, 2, 0, base)
        ref_tile = run_plan(plan, x, gpu)
        outs = []
        for t in wide:
            for sgw in (base, 3 * base):
                plan.set_tile(*t, sgw)
                outs.append((t, sgw, run_plan(plan, x, gpu)))
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), x, I)
    for t, sgw, got in outs:
        assert_parity(got, ref, TOL[prec], f"{shape} {prec} {t} sgw {sgw}")
        assert np.array_equal(got, ref_tile), (shape, prec, t, sgw)


def test_wide_form_4bit(gpu):
    N, C, B, T, I = 256, 2, 64, 2048, 64
    print(f"wide form 4-bit {(N, C, B, T, I)}", flush=True)
    g = np.random.default_rng(77)
    pos = synth.disc_positions(N, 250.0, g)
    dirs = synth.random_dirs(B, g)
    freqs = np.linspace(401e6, 415e6, C)
    x4 = synth.pack4(g.integers(-8, 8, (C, T, N, 2)).astype(np.int8))
    with bf.Plan(N, C, B, T, I, precision="fp16", input_bits=4) as plan:
        plan.set_weights(pos, dirs, freqs)
        assert (4, 4, 4, -2) in plan.tile_candidates()
        plan.set_tile(4, 2, 2, 0, 1)
        ref_tile = run_plan(plan, x4, gpu)
        plan.set_tile(4, 4, 4, -2, 1)
        got = run_plan(plan, x4, gpu)
    ref = oracle.beamform(oracle.weights(pos, dirs, freqs), oracle.unpack4(x4), I)
    assert_parity(got, ref, TOL["fp16"], "wide 4-bit")
    assert np.array_equal(got, ref_tile)


def test_wide_not_offered_where_it_cannot_run(gpu):
    """FP32, complex output, accumulation, I % 4 != 0, byte-load rows and a
    window count that is not a multiple of 4 keep the four-wave forms only;
    I == 2 rejects the tile."""
    cases = [dict(shape=(256, 1, 64, 1024, 64), precision="fp32"),
             dict(shape=(256, 1, 64, 1024, 1), precision="fp16", output="complex"),
             dict(shape=(256, 1, 64, 1024, 64), precision="fp16", accumulate=True),
             dict(shape=(256, 1, 64, 1020, 3), precision="fp16"),
             dict(shape=(36, 1, 64, 1024, 16), precision="fp16"),
             dict(shape=(256, 1, 64, 1000, 4), precision="fp16")]
    for c in cases:
        N, C, B, T, I = c.pop("shape")
        with bf.Plan(N, C, B, T, I, **c) as plan:
            assert all(t[3] != -2 for t in plan.tile_candidates()), c
    with bf.Plan(256, 1, 64, 1024, 2, precision="fp16") as plan:
        assert all(t[3] != -2 for t in plan.tile_candidates())
        with pytest.raises(bf.BfError):
            plan.set_tile(4, 4, 4, -2, 1)
