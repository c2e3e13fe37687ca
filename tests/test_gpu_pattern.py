"""Beam-pattern (array-factor) maps on the GPU (Sec. 3.1's simulated beam
pattern; Eq. 1): every beam of a plan evaluated for a unit plane wave from
each direction of a grid, with the plan's own rounded weights.

Reference: |oracle.beams(W_plan, oracle.steering(...))|^2 in FP64 with the
weights read back from the plan.  The map is FP32 (sin/cos of the reduced
phase and the sums): every element within 2e-5 of its beam's peak response,
and the steered direction within 1e-5 of N^2 for the FP32 plan; the line
array's Dirichlet closed form to the same bound."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth

pytestmark = pytest.mark.gpu


def grid_dirs(nx, ny, span_deg):
    tx = np.linspace(-span_deg, span_deg, nx)
    ty = np.linspace(-span_deg, span_deg, ny)
    TY, TX = np.meshgrid(ty, tx, indexing="ij")
    return synth.dir_from_lm_angles(TX.ravel(), TY.ravel())


def check_map(got, ref, what):
    peak = ref.max(axis=-1, keepdims=True)
    err = np.abs(got.astype(np.float64) - ref) / peak
    assert err.max() <= 2e-5, (what, err.max())


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_pattern_matches_oracle(gpu, prec):
    print(f"pattern {prec}", flush=True)
    w = synth.paper()
    chans = [0, 500, 1023]
    freqs = w.freqs[chans]
    dirs = w.dirs[::7]                          # 19 beams
    gd = grid_dirs(37, 29, 40.0)                # 1073 directions (ragged vs 64)
    with bf.Plan(32, 3, len(dirs), 16, 1, precision=prec) as plan:
        plan.set_weights(w.pos, dirs, freqs)
        got = plan.beam_pattern(w.pos, freqs, gd).cpu().numpy()
        wq = plan.get_weights()
    ref = np.abs(oracle.beams(wq, oracle.steering(w.pos, gd, freqs))) ** 2
    check_map(got, ref, prec)
    if prec == "fp32":
        with bf.Plan(32, 3, len(dirs), 16, 1) as plan:
            plan.set_weights(w.pos, dirs, freqs)
            on = plan.beam_pattern(w.pos, freqs, dirs).cpu().numpy()
        np.testing.assert_allclose(np.diagonal(on, axis1=1, axis2=2), 32.0 ** 2, rtol=1e-5)


def test_pattern_many_antennas_masked(gpu):
    """N = 300 (several antenna chunks, a partial last one) with a masked
    sub-array: the map is the sub-array's."""
    g = np.random.default_rng(60)
    N, C, B = 300, 2, 33
    pos = synth.disc_positions(N, 250.0, g)
    dirs = synth.random_dirs(B, g, 20.0)
    freqs = np.array([402e6, 413e6])
    mask = g.random(N) < 0.6
    gd = grid_dirs(23, 23, 30.0)
    with bf.Plan(N, C, B, 16, 1, precision="fp16") as plan:
        plan.set_antenna_mask(mask)
        plan.set_weights(pos, dirs, freqs)
        got = plan.beam_pattern(pos, freqs, gd).cpu().numpy()
        wq = plan.get_weights()
    assert np.all(wq[:, :, ~mask] == 0)
    ref = np.abs(oracle.beams(wq, oracle.steering(pos, gd, freqs))) ** 2
    check_map(got, ref, "N=300 masked")


def test_pattern_line_array_closed_form(gpu):
    N, d, f = 24, 9.0, 407e6
    pos = synth.line_positions(N, d)
    tb = np.array([0.0, 12.5])
    tg = np.linspace(-40.0, 40.0, 161)
    with bf.Plan(N, 1, 2, 16, 1) as plan:
        plan.set_weights(pos, synth.dir_from_xz_angle(tb), [f])
        got = plan.beam_pattern(pos, [f], synth.dir_from_xz_angle(tg)).cpu().numpy()[0]
    lam = 299_792_458.0 / f
    for i, b in enumerate(tb):
        x = np.pi * d / lam * (np.sin(np.deg2rad(tg)) - np.sin(np.deg2rad(b)))
        with np.errstate(invalid="ignore", divide="ignore"):
            ref = np.where(np.abs(np.sin(x)) < 1e-12, N * N, np.sin(N * x) ** 2 / np.sin(x) ** 2)
        assert np.max(np.abs(got[i] - ref)) <= 2e-5 * N * N, i


def test_pattern_errors(gpu):
    import torch
    with bf.Plan(8, 1, 2, 16, 1) as plan:
        pos = synth.line_positions(8)
        with pytest.raises(bf.BfError) as e:
            plan.beam_pattern(pos, [400e6], [[0, 0, 1]])
        assert e.value.status == bf.ERR_STATE
        plan.set_weights(pos, [[0, 0, 1], [0, 0, 1]], [400e6])
        with pytest.raises(bf.BfError) as e:
            plan.beam_pattern(pos, [400e6], [[0, 0, 2]])
        assert e.value.status == bf.ERR_INVALID_ARG
        with pytest.raises(ValueError):
            plan.beam_pattern(pos, [400e6], [[0, 0, 1]], out=torch.empty((1, 2, 2), device=gpu))
