"""Time-varying weights on the GPU (Sec. 3.2: the next pointing's
coefficients are computed while the current buffer is beamformed; Sec. 3.1:
tracking beams and sub-array antenna masks).

Asynchronous refresh: each block's output must equal, bit for bit, the same
block run by a plan whose weights were set synchronously for that block's
pointing, however the refreshes (side stream) and runs (main stream)
interleave; runs enqueued before a refresh keep the old weights.  Antenna
mask: the masked plan equals the unmasked plan on voltages whose masked
antennas are zeroed, and the oracle with the masked weights."""
import numpy as np
import pytest

import oracle
from paper_1412_4907_amd import bf, synth
from tests.gpu_util import assert_parity, run_plan

pytestmark = pytest.mark.gpu
N, C, B, T, I = 32, 8, 64, 4096, 16


def _setup(seed):
    g = np.random.default_rng(seed)
    pos = synth.grid_positions(4, 8, 10.0, 20.0)
    freqs = np.linspace(401e6, 415e6, C)
    base = synth.random_dirs(B, g, 20.0)
    return g, pos, freqs, base


def _pointing(base, k):
    """Beam set k: the base grid turned about the zenith by 0.4 deg per block
    (a tracking beam set following the sky)."""
    a = np.deg2rad(0.4 * k)
    rot = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    d = base @ rot.T
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_tracking_refresh_overlapped_with_runs(gpu, prec):
    import torch
    print(f"async refresh {prec}", flush=True)
    g, pos, freqs, base = _setup(50)
    K = 8
    xs = [g.integers(-128, 128, (C, T, N, 2)).astype(np.int8) for _ in range(K)]
    # expected: a fresh synchronous plan per block
    ref = []
    with bf.Plan(N, C, B, T, I, precision=prec) as rp:
        for k in range(K):
            rp.set_weights(pos, _pointing(base, k), freqs)
            ref.append(run_plan(rp, xs[k], gpu))
    run_s, side_s = torch.cuda.Stream(), torch.cuda.Stream()
    xd = [torch.from_numpy(x).to(gpu) for x in xs]
    outs = [torch.full((C, B, T // I), float("nan"), device=gpu) for _ in range(K)]
    torch.cuda.synchronize()
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_weights(pos, _pointing(base, 0), freqs, stream=run_s)
        for k in range(K):
            if k > 0:  # next pointing, generated while block k-1 still runs
                plan.set_weights_async(pos, _pointing(base, k), freqs, stream=side_s)
            plan.run(xd[k], outs[k], stream=run_s)
            if k == 3:  # a second block on the same weights, before the next refresh
                extra = torch.empty_like(outs[k])
                plan.run(xd[k], extra, stream=run_s)
        torch.cuda.synchronize()
        for k in range(K):
            assert np.array_equal(outs[k].cpu().numpy(), ref[k]), k
        assert np.array_equal(extra.cpu().numpy(), ref[3])
        # readback returns the weights of the last pointing
        w = plan.get_weights()
    with bf.Plan(N, C, B, T, I, precision=prec) as rp:
        rp.set_weights(pos, _pointing(base, K - 1), freqs)
        assert np.array_equal(w, rp.get_weights())
    W = oracle.weights(pos, _pointing(base, 5), freqs[:2])
    assert_parity(ref[5][:2], oracle.beamform(W, xs[5][:2], I), 1e-5 if prec == "fp32" else 2e-3,
                  "tracking block 5")


def test_refresh_order_and_supersede(gpu):
    import torch
    g, pos, freqs, base = _setup(51)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    refs = []
    with bf.Plan(N, C, B, T, I) as rp:
        for k in range(3):
            rp.set_weights(pos, _pointing(base, k), freqs)
            refs.append(run_plan(rp, x, gpu))
    with bf.Plan(N, C, B, T, I) as plan:
        # weights only through an asynchronous refresh: the first run takes it
        plan.set_weights_async(pos, _pointing(base, 1), freqs)
        assert np.array_equal(run_plan(plan, x, gpu), refs[1])
        # two refreshes before a run: the later one wins
        side = torch.cuda.Stream()
        plan.set_weights_async(pos, _pointing(base, 0), freqs, stream=side)
        plan.set_weights_async(pos, _pointing(base, 2), freqs, stream=side)
        assert np.array_equal(run_plan(plan, x, gpu), refs[2])
        # a synchronous set supersedes a pending refresh
        plan.set_weights_async(pos, _pointing(base, 1), freqs, stream=side)
        side.synchronize()
        plan.set_weights(pos, _pointing(base, 0), freqs)
        assert np.array_equal(run_plan(plan, x, gpu), refs[0])
        # a refreshed plan is not accepted by the table form
        table = bf.Table(N, I, "fp32")
        xd = torch.from_numpy(x).to(gpu)
        p = torch.empty((C, B, T // I), device=gpu)
        with pytest.raises(bf.BfError) as e:
            table.set([plan], [xd], [p])
        assert e.value.status == bf.ERR_UNSUPPORTED
        table.destroy()


def test_refresh_in_batch(gpu):
    import torch
    g, pos, freqs, base = _setup(52)
    x1 = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    x2 = g.integers(-128, 128, (C, T // 2, N, 2)).astype(np.int8)
    with bf.Plan(N, C, B, T, I, precision="fp16") as a, \
            bf.Plan(N, C, B, T // 2, I, precision="fp16") as b, \
            bf.Plan(N, C, B, T, I, precision="fp16") as ra:
        a.set_weights(pos, _pointing(base, 0), freqs)
        b.set_weights(pos, _pointing(base, 3), freqs)
        batch = bf.Batch([a, b])
        xs = [torch.from_numpy(x1).to(gpu), torch.from_numpy(x2).to(gpu)]
        ps = [torch.empty((C, B, T // I), device=gpu), torch.empty((C, B, T // 2 // I), device=gpu)]
        for k in range(1, 4):
            a.set_weights_async(pos, _pointing(base, k), freqs, stream=torch.cuda.Stream())
            batch.run(xs, ps)
            torch.cuda.synchronize()
            ra.set_weights(pos, _pointing(base, k), freqs)
            assert np.array_equal(ps[0].cpu().numpy(), run_plan(ra, x1, gpu)), k
            assert np.array_equal(ps[1].cpu().numpy(), run_plan(b, x2, gpu)), k
        batch.destroy()


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_antenna_mask_sub_array(gpu, prec):
    g, pos, freqs, base = _setup(53)
    x = g.integers(-128, 128, (C, T, N, 2)).astype(np.int8)
    mask = np.zeros(N, dtype=bool)
    mask[[0, 1, 2, 3, 8, 9, 10, 11, 20, 27]] = True   # a ten-element sub-array
    x0 = x.copy()
    x0[:, :, ~mask] = 0
    with bf.Plan(N, C, B, T, I, precision=prec) as plan:
        plan.set_antenna_mask(mask)
        plan.set_weights(pos, base, freqs)
        got = run_plan(plan, x, gpu)
        wq = plan.get_weights()
        assert np.all(wq[:, :, ~mask] == 0) and np.all(np.abs(wq[:, :, mask]) > 0.99)
        plan.set_antenna_mask(None)
        plan.set_weights(pos, base, freqs)
        full_on_zeroed = run_plan(plan, x0, gpu)
    assert np.array_equal(got, full_on_zeroed)
    W = oracle.weights(pos, base, freqs) * mask[None, None, :]
    tol = {"fp32": 1e-5, "fp16": 2e-3, "bf16": 1e-2}[prec]
    assert_parity(got, oracle.beamform(W, x, I), tol, f"sub-array {prec}")
