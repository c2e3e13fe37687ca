"""Batching form: several beam sets of uneven N, C, B, T in one persistent
launch per kernel form (in FP16/BF16 the sets with 2N > 128 run the
eight-wave form in a launch of their own); each set's output must equal
(bitwise) the same set run alone, and match the oracle on sampled
channels."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity, run_plan

pytestmark = pytest.mark.gpu


def _sets(prec, scale_T=1):
    g = np.random.default_rng(21)
    shapes = [(16, 6, 16, 1024), (32, 5, 64, 2048), (64, 3, 40, 1536), (128, 2, 100, 1024),
              (256, 2, 20, 512), (48, 4, 7, 3072)]
    out = []
    for i, (N, C, B, T) in enumerate(shapes):
        pos = synth.disc_positions(N, 250.0, g)
        dirs = synth.random_dirs(B, g)
        freqs = np.linspace(400e6, 416e6, C)
        x = g.integers(-128, 128, (C, T * scale_T, N, 2)).astype(np.int8)
        plan = bf.Plan(N, C, B, T * scale_T, 16, precision=prec)
        plan.set_weights(pos, dirs, freqs)
        out.append((plan, x, pos, dirs, freqs))
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_batch_equals_solo_and_oracle(gpu, prec):
    import torch
    print(f"batch {prec}", flush=True)
    sets = _sets(prec)
    plans = [s[0] for s in sets]
    solo = [run_plan(s[0], s[1], gpu) for s in sets]
    xs = [torch.from_numpy(s[1]).to(gpu) for s in sets]
    ps = [torch.full((p.C, p.B, p.windows), float("nan"), device=gpu) for p in plans]
    batch = bf.Batch(plans)
    for rep in range(2):  # the device queue is reset per launch
        batch.run(xs, ps)
        torch.cuda.synchronize()
        for i, (s, p) in enumerate(zip(solo, ps)):
            assert np.array_equal(s, p.cpu().numpy()), (rep, i)
    batch.destroy()
    tol = {"fp32": 1e-5, "fp16": 2e-3, "bf16": 1e-2}[prec]
    for (plan, x, pos, dirs, freqs), got in zip(sets, solo):
        ref = oracle.beamform(oracle.weights(pos, dirs, freqs[:1]), x[:1], 16)
        assert_parity(got[:1], ref, tol, f"batch set N={plan.N}")
    for p in plans:
        p.destroy()
