"""FP64 CPU oracle for the coherent beamformer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library and its Python binding never touch it.

The arithmetic lives in ``bf_oracle.c`` (plain FP64 loops, OpenMP over
(channel, beam)); this module only marshals numpy arrays:

* ``weights(pos, dirs, freqs)``  -> complex128 [C][B][N], the Eq. 1 phase
  model W = exp(-i 2 pi f_c (k_b . r_n) / c0) (Sec. 1).
* ``beamform(w, x, I)``          -> float64 [C][B][T/I]: per channel the
  coefficient matrix times every antenna vector (Sec. 2.1), power |B|^2,
  summed over non-overlapping windows of I samples.  ``x`` is int8
  [C][T][N][2] or complex128 [C][T][N] (unquantised input for the pins).
* ``beams(w, x)``                -> complex128 [C][B][T] before detection.
* ``steering(pos, dirs, freqs)``  -> complex128 [C][G][N]: a unit plane wave
  from each direction as the antennas receive it, exp(+i 2 pi f_c (k_g . r_n)
  / c0) (Sec. 1); |beams(w, steering)|^2 is the beam-pattern map (Sec. 3.1).
* ``unpack4(x4)``                -> int8 [...][2]: 4-bit complex samples (one
  byte each, Sec. 2.1: two 4-bit two's complement components per antenna
  sample) widened to (re, im); the real part is the high nibble.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        _lib = _load(_build.LIB)
    return _lib


def use_library(path: str):
    """Swap in another build of bf_oracle.c (the mutation tests compile
    planted mistakes into temporary copies).  Returns the previous handle;
    ``restore_library(prev)`` puts it back."""
    global _lib
    prev = lib()
    _lib = _load(path)
    return prev


def restore_library(prev) -> None:
    global _lib
    _lib = prev


def _load(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.bfo_weights.argtypes = [i32, i32, i32, P, P, P, P]
    L.bfo_beamform_i8.argtypes = [i32, i32, i32, i64, i32, P, P, P]
    L.bfo_beamform_f64.argtypes = [i32, i32, i32, i64, i32, P, P, P]
    L.bfo_beams_f64.argtypes = [i32, i32, i32, i64, P, P, P]
    L.bfo_max_threads.restype = ctypes.c_int
    L.bfo_set_threads.argtypes = [ctypes.c_int]
    for f in (L.bfo_weights, L.bfo_beamform_i8, L.bfo_beamform_f64, L.bfo_beams_f64):
        f.restype = ctypes.c_int
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().bfo_set_threads(int(n))


def max_threads() -> int:
    return int(lib().bfo_max_threads())


def weights(pos, dirs, freqs) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    dirs = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    freqs = np.ascontiguousarray(freqs, dtype=np.float64).reshape(-1)
    N, B, C = pos.shape[0], dirs.shape[0], freqs.shape[0]
    w = np.empty((C, B, N, 2), dtype=np.float64)
    if lib().bfo_weights(N, C, B, _p(pos), _p(dirs), _p(freqs), _p(w)) != 0:
        raise ValueError("bfo_weights: invalid arguments")
    return w[..., 0] + 1j * w[..., 1]


def _w_ri(w) -> np.ndarray:
    w = np.asarray(w)
    if np.iscomplexobj(w):
        w = np.stack([w.real, w.imag], axis=-1)
    return np.ascontiguousarray(w, dtype=np.float64)


def beamform(w, x, integration: int = 1) -> np.ndarray:
    """Integrated power [C][B][T/I] (float64)."""
    wri = _w_ri(w)
    C, B, N = wri.shape[:3]
    if np.iscomplexobj(x):
        xr = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1), dtype=np.float64)
        fn = lib().bfo_beamform_f64
    elif x.dtype == np.int8:
        xr = np.ascontiguousarray(x)
        fn = lib().bfo_beamform_i8
    else:
        xr = np.ascontiguousarray(x, dtype=np.float64)
        fn = lib().bfo_beamform_f64
    if xr.shape[0] != C or xr.shape[2] != N or xr.shape[3] != 2:
        raise ValueError(f"shape mismatch: w {wri.shape} x {xr.shape}")
    T = xr.shape[1]
    I = int(integration)
    if I < 1 or T % I:
        raise ValueError("T must be a positive multiple of I")
    p = np.empty((C, B, T // I), dtype=np.float64)
    if fn(N, C, B, T, I, _p(wri), _p(xr), _p(p)) != 0:
        raise ValueError("bfo_beamform: invalid arguments")
    return p


def beams(w, x) -> np.ndarray:
    """Complex beams [C][B][T] (complex128), no detection."""
    wri = _w_ri(w)
    C, B, N = wri.shape[:3]
    x = np.asarray(x)
    if np.iscomplexobj(x):
        xr = np.stack([x.real, x.imag], axis=-1)
    else:
        xr = x
    xr = np.ascontiguousarray(xr, dtype=np.float64)
    T = xr.shape[1]
    out = np.empty((C, B, T, 2), dtype=np.float64)
    if lib().bfo_beams_f64(N, C, B, T, _p(wri), _p(xr), _p(out)) != 0:
        raise ValueError("bfo_beams_f64: invalid arguments")
    return out[..., 0] + 1j * out[..., 1]


def unpack4(x4) -> np.ndarray:
    """Decode packed 4-bit complex voltages: uint8 [...] -> int8 [...][2].

    Each byte holds one antenna sample (Sec. 2.1): the real component in
    bits 7..4 and the imaginary component in bits 3..0, each a 4-bit two's
    complement number, so a nibble n >= 8 stands for n - 16 and the values
    span [-8, 7]."""
    b = np.asarray(x4)
    if b.dtype != np.uint8:
        raise ValueError("packed 4-bit voltages must be uint8")
    hi = (b >> 4).astype(np.int16)
    lo = (b & 0x0F).astype(np.int16)
    re = np.where(hi >= 8, hi - 16, hi)
    im = np.where(lo >= 8, lo - 16, lo)
    return np.stack([re, im], axis=-1).astype(np.int8)


C0 = 299_792_458.0  # m/s


def steering(pos, dirs, freqs) -> np.ndarray:
    """Unit plane waves: [C][G][N] complex128, entry (c, g, n) =
    exp(+i 2 pi f_c (k_g . r_n) / c0) -- the phase a wavefront from k_g
    carries at antenna n relative to the origin (Sec. 1, the delay picture
    behind Eq. 1), evaluated directly in FP64."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    freqs = np.asarray(freqs, dtype=np.float64).reshape(-1)
    delay = (dirs @ pos.T) / C0                     # [G][N] seconds
    return np.exp(2j * np.pi * freqs[:, None, None] * delay[None])
