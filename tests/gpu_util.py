"""Helpers for the GPU parity tests: run a plan on numpy inputs through the
C ABI and compare with the oracle."""
from __future__ import annotations

import numpy as np


def run_plan(plan, x: np.ndarray, dev, stream=None) -> np.ndarray:
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    p = torch.full((plan.C, plan.B, plan.windows), float("nan"), dtype=torch.float32, device=dev)
    plan.run(xd, p, stream)
    torch.cuda.synchronize()
    return p.cpu().numpy()


def beam_errors(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-beam normwise relative error ||P_gpu - P_ref||_2 / ||P_ref||_2 over
    the window axis."""
    got = got.astype(np.float64)
    num = np.linalg.norm(got - ref, axis=-1)
    den = np.linalg.norm(ref, axis=-1)
    return num / np.maximum(den, 1e-300)


def assert_parity(got: np.ndarray, ref: np.ndarray, tol: float, what: str = "") -> dict:
    """Element by element: |dP| <= tol * (|P_ref| + mean_w P_ref[c, b, :]),
    i.e. relative error, with near-null samples measured against their beam's
    mean power; plus the per-beam normwise error <= tol."""
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    g = got.astype(np.float64)
    scale = np.abs(ref) + np.mean(np.abs(ref), axis=-1, keepdims=True)
    elem = np.abs(g - ref) / np.maximum(scale, 1e-300)
    be = beam_errors(got, ref)
    stats = {"beam_max": float(be.max()), "beam_median": float(np.median(be)),
             "elem_max": float(elem.max())}
    assert be.max() <= tol, f"{what}: per-beam error {be.max():.3e} > {tol:g} {stats}"
    assert elem.max() <= tol, f"{what}: element error {elem.max():.3e} > {tol:g} {stats}"
    return stats


def round_bf16(v: np.ndarray) -> np.ndarray:
    """FP64 -> nearest-even BF16 value (as float64), from frexp: 8
    significant bits.  Valid for normal results, which is all |W| <= 1 produce
    here besides exact zeros."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def round_to(w: np.ndarray, prec: str) -> np.ndarray:
    """Round complex FP64 weights per component to the storage precision."""
    f = {"fp32": lambda a: a.astype(np.float32).astype(np.float64),
         "fp16": lambda a: a.astype(np.float16).astype(np.float64),
         "bf16": round_bf16}[prec]
    return f(w.real) + 1j * f(w.imag)
