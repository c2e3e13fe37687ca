"""Thin Python binding of the gfx950 beamformer C ABI (``include/bf.h``).

Argument marshalling only: every step of the beamforming path runs in the
HIP kernels of ``libbf.so``.  PyTorch supplies device memory (tensors passed
by ``data_ptr()``) and streams (``torch.cuda.Stream.cuda_stream``).  If the
library has not been built, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbf.so")

FP32, FP16, BF16 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "fp16": FP16, "bf16": BF16}
ACCUMULATE = 1
INPUT_4BIT = 2
OUTPUT_COMPLEX = 4

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_STATE, ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5

# every entry point declared in include/bf.h
EXPORTS = ["bf_strerror", "bf_version", "bf_last_hip_error", "bf_tune_load", "bf_tune_key",
           "bf_plan_apply_tuned", "bf_plan_create",
           "bf_plan_create_ex", "bf_set_weights", "bf_set_weights_async",
           "bf_plan_set_antenna_mask", "bf_beam_pattern", "bf_set_weights_raw", "bf_get_weights",
           "bf_run", "bf_plan_info", "bf_plan_set_tile", "bf_plan_set_output_scale",
           "bf_plan_tile_candidates",
           "bf_plan_destroy", "bf_batch_create", "bf_batch_tile_candidates", "bf_batch_run",
           "bf_batch_destroy", "bf_table_create", "bf_table_set", "bf_table_run",
           "bf_table_destroy", "bf_beam_pattern_noalloc"]

# capacity of the allocation-free beam-pattern entry point's geometry staging,
# in doubles: 3 N + C + 3 G must not exceed it
PATTERN_SCRATCH_DOUBLES = 1 << 20


class BfError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = ""
        if status in (ERR_HIP, ERR_OOM):
            detail = " [" + lib().bf_last_hip_error().decode() + "]"
        super().__init__(f"{where}: {strerror(status)} ({status}){detail}")


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_antennas", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("n_beams", ctypes.c_int32), ("integration", ctypes.c_int32),
                ("n_samples", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("k_padded", ctypes.c_int32), ("beams_padded", ctypes.c_int32),
                ("tile_mt", ctypes.c_int32), ("tile_nbt", ctypes.c_int32),
                ("tile_nbp", ctypes.c_int32), ("tile_kres", ctypes.c_int32),
                ("sg_per_wave", ctypes.c_int32),
                ("work_units", ctypes.c_int64), ("weight_bytes", ctypes.c_int64),
                ("lds_bytes", ctypes.c_int64), ("flops", ctypes.c_double),
                ("tile_tuned", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Load libbf.so (built in-tree by ``paper_1412_4907_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(python -m paper_1412_4907_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.bf_strerror.restype = ctypes.c_char_p
        L.bf_strerror.argtypes = [ctypes.c_int]
        L.bf_version.restype = ctypes.c_char_p
        L.bf_last_hip_error.restype = ctypes.c_char_p
        L.bf_tune_load.argtypes = [ctypes.c_char_p]
        L.bf_tune_key.argtypes = [P, i32, ctypes.c_char_p, i32]
        L.bf_plan_apply_tuned.argtypes = [P, i32]
        L.bf_plan_create.argtypes = [ctypes.POINTER(P), i32, i32, i32, i64, i32]
        L.bf_plan_create_ex.argtypes = [ctypes.POINTER(P), i32, i32, i32, i64, i32, ctypes.c_int, u32]
        L.bf_set_weights.argtypes = [P, P, P, P, P]
        L.bf_set_weights_async.argtypes = [P, P, P, P, P]
        L.bf_plan_set_antenna_mask.argtypes = [P, P]
        L.bf_beam_pattern.argtypes = [P, P, P, P, i32, P, P]
        L.bf_beam_pattern_noalloc.argtypes = [P, P, P, P, i32, P, P]
        L.bf_set_weights_raw.argtypes = [P, P, P]
        L.bf_get_weights.argtypes = [P, P, P]
        L.bf_run.argtypes = [P, P, P, P]
        L.bf_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
        L.bf_plan_set_tile.argtypes = [P, i32, i32, i32, i32, i32]
        L.bf_plan_set_output_scale.argtypes = [P, ctypes.c_float]
        L.bf_plan_tile_candidates.argtypes = [P, P, i32]
        L.bf_batch_tile_candidates.argtypes = [P, P, i32]
        L.bf_plan_destroy.argtypes = [P]
        L.bf_batch_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(P), i32]
        L.bf_batch_run.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), P]
        L.bf_batch_destroy.argtypes = [P]
        L.bf_table_create.argtypes = [ctypes.POINTER(P), i32, i32, i32, ctypes.c_uint32]
        L.bf_table_set.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), i32, P]
        L.bf_table_run.argtypes = [P, P]
        L.bf_table_destroy.argtypes = [P]
        for name in EXPORTS[3:]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        # the autotuner's tile cache, applied by the library at plan creation
        from . import tune
        path = tune.cache_path()
        if os.path.exists(path):
            tune_load(path)
    return _lib


def tune_load(path: str) -> int:
    """Load a tile cache written by the autotuner (``bf_tune_load``); returns
    the number of entries."""
    n = lib().bf_tune_load(os.fsencode(path))
    if n < 0:
        raise BfError(n, f"bf_tune_load({path})")
    return n


def strerror(status: int) -> str:
    return lib().bf_strerror(int(status)).decode()


def version() -> str:
    return lib().bf_version().decode()


def _check(status: int, where: str) -> None:
    if status != OK:
        raise BfError(status, where)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _host_f64(a, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


class Plan:
    """One beam set: N antennas, C channels, B beams, T samples per block,
    integration I.  Owns the device weights (see ``bf_plan_create_ex``).
    ``input_bits``: 8 (int8 [C][T][N][2]) or 4 (uint8 [C][T][N], real part in
    the high nibble, imaginary part in the low nibble).  ``output``: "power"
    (float32 [C][B][T/I]) or "complex" (float16 [C][B][T][2], I == 1)."""

    def __init__(self, n_antennas: int, n_channels: int, n_beams: int, n_samples: int,
                 integration: int = 1, precision: str | int = "fp32",
                 accumulate: bool = False, input_bits: int = 8, output: str = "power"):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if input_bits not in (4, 8):
            raise ValueError("input_bits must be 4 or 8")
        if output not in ("power", "complex"):
            raise ValueError("output must be 'power' or 'complex'")
        flags = (ACCUMULATE if accumulate else 0) | (INPUT_4BIT if input_bits == 4 else 0)
        flags |= OUTPUT_COMPLEX if output == "complex" else 0
        h = ctypes.c_void_p()
        _check(lib().bf_plan_create_ex(ctypes.byref(h), n_antennas, n_channels, n_beams,
                                       n_samples, integration, prec, flags), "bf_plan_create_ex")
        self._h = h
        self.N, self.C, self.B, self.T, self.I = (n_antennas, n_channels, n_beams, n_samples,
                                                  integration)
        self.precision = prec
        self.input_bits = input_bits
        self.output = output

    @property
    def x_shape(self) -> tuple:
        """Shape of one block of voltages for this plan's input format."""
        if self.input_bits == 4:
            return (self.C, self.T, self.N)
        return (self.C, self.T, self.N, 2)

    @property
    def x_dtype(self):
        import torch
        return torch.uint8 if self.input_bits == 4 else torch.int8

    @property
    def p_shape(self) -> tuple:
        """Shape of one block's output for this plan's output form."""
        if self.output == "complex":
            return (self.C, self.B, self.T, 2)
        return (self.C, self.B, self.windows)

    @property
    def p_dtype(self):
        import torch
        return torch.float16 if self.output == "complex" else torch.float32

    def set_output_scale(self, scale: float) -> None:
        """Factor applied to complex beams before their FP16 rounding."""
        _check(lib().bf_plan_set_output_scale(self.handle, float(scale)),
               "bf_plan_set_output_scale")

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    @property
    def windows(self) -> int:
        return self.T // self.I

    def set_weights(self, pos, dirs, freqs, stream=None) -> None:
        pos = _host_f64(pos, (self.N, 3))
        dirs = _host_f64(dirs, (self.B, 3))
        freqs = _host_f64(freqs, (self.C,))
        _check(lib().bf_set_weights(self.handle, pos.ctypes.data, dirs.ctypes.data,
                                    freqs.ctypes.data, _stream_ptr(stream)), "bf_set_weights")

    def set_weights_async(self, pos, dirs, freqs, stream=None) -> None:
        """Generate the next pointing's weights on ``stream`` into the spare
        buffer; the plan's next run waits for them and switches over."""
        pos = _host_f64(pos, (self.N, 3))
        dirs = _host_f64(dirs, (self.B, 3))
        freqs = _host_f64(freqs, (self.C,))
        _check(lib().bf_set_weights_async(self.handle, pos.ctypes.data, dirs.ctypes.data,
                                          freqs.ctypes.data, _stream_ptr(stream)),
               "bf_set_weights_async")

    def beam_pattern(self, pos, freqs, grid_dirs, out=None, stream=None, noalloc=False):
        """Power of every beam for a unit plane wave from each grid direction:
        float32 [C][B][G] device tensor (``bf_beam_pattern``; with ``noalloc``
        ``bf_beam_pattern_noalloc``, which stages the geometry in the
        library's fixed per-device array and returns without waiting)."""
        import torch
        pos = _host_f64(pos, (self.N, 3))
        freqs = _host_f64(freqs, (self.C,))
        gd = np.ascontiguousarray(grid_dirs, dtype=np.float64).reshape(-1, 3)
        G = gd.shape[0]
        if out is None:
            out = torch.empty((self.C, self.B, G), dtype=torch.float32, device="cuda")
        if out.dtype != torch.float32 or tuple(out.shape) != (self.C, self.B, G) or \
                not out.is_cuda or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 device tensor [{self.C}][{self.B}][{G}]")
        name = "bf_beam_pattern_noalloc" if noalloc else "bf_beam_pattern"
        _check(getattr(lib(), name)(self.handle, pos.ctypes.data, freqs.ctypes.data,
                                    gd.ctypes.data, G, out.data_ptr(), _stream_ptr(stream)),
               name)
        return out

    def set_antenna_mask(self, mask=None) -> None:
        """Antennas used by weights generated from now on (None: all)."""
        if mask is None:
            _check(lib().bf_plan_set_antenna_mask(self.handle, None), "bf_plan_set_antenna_mask")
            return
        m = np.ascontiguousarray(np.asarray(mask).astype(bool), dtype=np.uint8)
        if m.shape != (self.N,):
            raise ValueError(f"mask must have {self.N} entries")
        _check(lib().bf_plan_set_antenna_mask(self.handle, m.ctypes.data),
               "bf_plan_set_antenna_mask")

    def set_weights_raw(self, w, stream=None) -> None:
        w = np.asarray(w)
        if np.iscomplexobj(w):
            w = np.stack([w.real, w.imag], axis=-1)
        w = _host_f64(w, (self.C, self.B, self.N, 2))
        _check(lib().bf_set_weights_raw(self.handle, w.ctypes.data, _stream_ptr(stream)),
               "bf_set_weights_raw")

    def get_weights(self, stream=None) -> np.ndarray:
        out = np.empty((self.C, self.B, self.N, 2), dtype=np.float64)
        _check(lib().bf_get_weights(self.handle, out.ctypes.data, _stream_ptr(stream)),
               "bf_get_weights")
        return out[..., 0] + 1j * out[..., 1]

    def check_io(self, x, p) -> None:
        import torch
        if x.dtype != self.x_dtype or tuple(x.shape) != self.x_shape:
            raise ValueError(f"x must be {self.x_dtype} {list(self.x_shape)}, "
                             f"got {x.dtype} {tuple(x.shape)}")
        if p.dtype != self.p_dtype or tuple(p.shape) != self.p_shape:
            raise ValueError(f"p must be {self.p_dtype} {list(self.p_shape)}, "
                             f"got {p.dtype} {tuple(p.shape)}")
        for t in (x, p):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("x and p must be contiguous device tensors")

    def run(self, x, p, stream=None) -> None:
        """Enqueue one block: x (``x_shape``, ``x_dtype``) -> p (``p_shape``, ``p_dtype``)."""
        self.check_io(x, p)
        _check(lib().bf_run(self.handle, x.data_ptr(), p.data_ptr(), _stream_ptr(stream)),
               "bf_run")

    def run_ptr(self, x_ptr: int, p_ptr: int, stream_ptr: int) -> None:
        """Same as ``run`` on raw device pointers (no checks beyond the C ABI's)."""
        _check(lib().bf_run(self.handle, x_ptr, p_ptr, stream_ptr), "bf_run")

    def info(self) -> dict:
        i = PlanInfo()
        _check(lib().bf_plan_info(self.handle, ctypes.byref(i)), "bf_plan_info")
        return i.as_dict()

    def set_tile(self, mt: int, nbt: int, nbp: int, kres: int, sg_per_wave: int) -> None:
        _check(lib().bf_plan_set_tile(self.handle, mt, nbt, nbp, kres, sg_per_wave),
               "bf_plan_set_tile")

    def tile_candidates(self, batch: bool = False) -> list:
        """Compiled (mt, nbt, nbp, kres) variants that can run this plan
        (``batch``: those the persistent batching kernel carries)."""
        fn = lib().bf_batch_tile_candidates if batch else lib().bf_plan_tile_candidates
        n = fn(self.handle, None, 0)
        if n < 0:
            raise BfError(n, "tile candidates")
        arr = (ctypes.c_int32 * (4 * max(n, 1)))()
        fn(self.handle, ctypes.addressof(arr), n)
        return [tuple(arr[4 * i:4 * i + 4]) for i in range(n)]

    def tune_key(self, batch: bool = False) -> str:
        """The tile-cache key of this plan's shape (``bf_tune_key``)."""
        buf = ctypes.create_string_buffer(256)
        n = lib().bf_tune_key(self.handle, 1 if batch else 0, buf, 256)
        if n < 0:
            raise BfError(n, "bf_tune_key")
        return buf.value.decode()

    def apply_tuned(self, batch: bool = False) -> bool:
        """Apply the loaded tile cache's entry for this shape (``batch``: the
        batching kernel's entry); False if there is none."""
        r = lib().bf_plan_apply_tuned(self.handle, 1 if batch else 0)
        if r < 0:
            raise BfError(r, "bf_plan_apply_tuned")
        return r == 1

    def tile(self) -> tuple:
        i = self.info()
        return (i["tile_mt"], i["tile_nbt"], i["tile_nbp"], i["tile_kres"], i["sg_per_wave"])

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().bf_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Several plans in one persistent launch (``bf_batch_create``)."""

    def __init__(self, plans: Sequence[Plan]):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().bf_batch_create(ctypes.byref(h), arr, len(self.plans)), "bf_batch_create")
        self._h = h

    def run(self, xs, ps, stream=None) -> None:
        if len(xs) != len(self.plans) or len(ps) != len(self.plans):
            raise ValueError("one x and one p per plan")
        for pl, x, p in zip(self.plans, xs, ps):
            pl.check_io(x, p)
        xa = (ctypes.c_void_p * len(xs))(*[x.data_ptr() for x in xs])
        pa = (ctypes.c_void_p * len(ps))(*[p.data_ptr() for p in ps])
        _check(lib().bf_batch_run(self._h, xa, pa, _stream_ptr(stream)), "bf_batch_run")

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().bf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Table:
    """Persistent batched launch over a set table kept in device memory
    (``bf_table_create``): ``set`` stores which plans run on which buffers,
    ``run`` enqueues the same two launches every time, so a graph captured
    around one ``run`` serves every later ``set``."""

    def __init__(self, n_antennas: int, integration: int, precision="fp16", input_bits: int = 8):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if input_bits not in (4, 8):
            raise ValueError("input_bits must be 4 or 8")
        h = ctypes.c_void_p()
        _check(lib().bf_table_create(ctypes.byref(h), int(n_antennas), int(integration), prec,
                                     INPUT_4BIT if input_bits == 4 else 0), "bf_table_create")
        self._h = h

    def set(self, plans: Sequence[Plan], xs, ps, stream=None) -> None:
        if len(xs) != len(plans) or len(ps) != len(plans):
            raise ValueError("one x and one p per plan")
        for pl, x, p in zip(plans, xs, ps):
            pl.check_io(x, p)
        n = len(plans)
        ha = (ctypes.c_void_p * max(n, 1))(*[pl.handle.value for pl in plans])
        xa = (ctypes.c_void_p * max(n, 1))(*[x.data_ptr() for x in xs])
        pa = (ctypes.c_void_p * max(n, 1))(*[p.data_ptr() for p in ps])
        _check(lib().bf_table_set(self._h, ha, xa, pa, n, _stream_ptr(stream)), "bf_table_set")

    def run(self, stream=None) -> None:
        _check(lib().bf_table_run(self._h, _stream_ptr(stream)), "bf_table_run")

    def destroy(self) -> None:
        if getattr(self, "_h", None) is not None:
            lib().bf_table_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
