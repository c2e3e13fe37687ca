"""Seeded synthetic inputs for the coherent beamformer.

This module is shared by the GPU path's tests/bench and by the CPU oracle's
tests.  It holds no beamforming arithmetic: it only draws antenna layouts,
beam pointings, channel frequencies and int8 complex voltages, or 4-bit
complex voltages packed one antenna sample per byte (Sec. 2.1: the BEST-2
F-engine emits 4-bit two's complement components), real part in the high
nibble.  A point
source is injected as a plane wave arriving at antenna n with the geometric
phase exp(+i 2 pi f (k_s . r_n) / c0) (Sec. 1, the delay/phase picture that
Eq. 1 builds on); that is the input model, not the beam sum.

Every random draw comes from ``np.random.default_rng(SeedSequence(4907,
spawn_key=...))`` keyed by (config, channel) or (config, purpose), so any
channel can be regenerated alone, in any order, in any process.

Workloads (the five shapes the beamformer is exercised on):

* ``small``     N=32 line (10 m), C=128 over 400-416 MHz, B=4, T=4096, I=1,
                sigma=16 noise + a tone 32 exp(2 pi i 0.01 t) from beam 0.
* ``paper``     N=32 on a 4x8 grid (10 m E-W, 20 m N-S), C=1024 over 16 MHz
                centred on 408 MHz (BEST-2, Sec. 1.1), B=128 on a 16x8 grid
                spanning +-15 deg, T=65536, I=16, sigma=16 noise + 3 noise-like
                point sources of amplitude 16 at seeded beam-grid centres.
* ``precision`` the ``small`` array and voltages with B=512 beams, I=1.
* ``batch``     12 beam sets, N in {16..256} on seeded positions within a
                250 m radius, C in {256,512,1024}, B in {16,64,256,1024},
                T in [8192, 32768] step 1024, I=16.
* ``serve``     N=256 on a 16x16 grid (10 m), blocks of 1024 ch x 8192
                samples at a 15.625 kHz channel rate (16 Msample/s per
                antenna), I=64.
"""
from __future__ import annotations

import zlib
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s (exact SI value)
SEED = 4907
SIGMA = 16.0
SIGMA4 = 2.0  # noise level of 4-bit workloads: 4 sigma reaches the [-8, 7] rails

# workload ids used as the first spawn-key element
CFG_IDS = {"small": 1, "paper": 2, "precision": 3, "batch": 4, "serve": 5}


def _key(x) -> int:
    if isinstance(x, str):
        return zlib.crc32(x.encode()) & 0x7FFFFFFF
    return int(x)


def rng(cfg: int | str, *key) -> np.random.Generator:
    """Generator for (config, key...). Strings are hashed to ints."""
    cid = CFG_IDS[cfg] if isinstance(cfg, str) else int(cfg)
    return np.random.default_rng(
        np.random.SeedSequence(SEED, spawn_key=(cid,) + tuple(_key(k) for k in key)))


# ----------------------------------------------------------------------------
# geometry, pointings, frequencies
# ----------------------------------------------------------------------------

def line_positions(n: int, spacing: float = 10.0) -> np.ndarray:
    """[n][3] ENU metres: antennas on the E-W axis, x = spacing * n."""
    p = np.zeros((n, 3))
    p[:, 0] = spacing * np.arange(n)
    return p


def grid_positions(nx: int, ny: int, dx: float, dy: float) -> np.ndarray:
    """[nx*ny][3]: antenna n = j*nx + i sits at (i*dx, j*dy, 0)."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    p = np.zeros((nx * ny, 3))
    p[:, 0] = (i * dx).ravel()
    p[:, 1] = (j * dy).ravel()
    return p


def disc_positions(n: int, radius: float, g: np.random.Generator) -> np.ndarray:
    """[n][3]: uniform over a disc of the given radius (z = 0)."""
    r = radius * np.sqrt(g.random(n))
    a = 2 * np.pi * g.random(n)
    p = np.zeros((n, 3))
    p[:, 0] = r * np.cos(a)
    p[:, 1] = r * np.sin(a)
    return p


def dir_from_xz_angle(theta_deg) -> np.ndarray:
    """Unit vectors at angle theta from zenith in the x-z plane."""
    t = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    return np.stack([np.sin(t), np.zeros_like(t), np.cos(t)], axis=-1)


def dir_from_lm_angles(tx_deg, ty_deg) -> np.ndarray:
    """Unit vectors with direction cosines l = sin(tx), m = sin(ty)."""
    l = np.sin(np.deg2rad(np.asarray(tx_deg, dtype=np.float64)))
    m = np.sin(np.deg2rad(np.asarray(ty_deg, dtype=np.float64)))
    return np.stack([l, m, np.sqrt(1.0 - l * l - m * m)], axis=-1)


def channel_freqs(n_chan: int, f_lo: float = 400e6, bw: float = 16e6) -> np.ndarray:
    """Channel centres f_c = f_lo + (c + 1/2) * bw / n_chan, Hz."""
    return f_lo + (np.arange(n_chan) + 0.5) * (bw / n_chan)


# ----------------------------------------------------------------------------
# voltages
# ----------------------------------------------------------------------------

@dataclass
class Source:
    """A point source: direction (unit 3-vector) and a per-sample complex
    envelope kind. ``tone`` = amp*exp(2 pi i nu t); ``noise`` = amp*exp(i psi_t),
    psi_t ~ U[0, 2 pi) drawn from the channel's stream."""
    direction: np.ndarray
    amp: float
    kind: str = "tone"
    nu: float = 0.0


def quantise(v: np.ndarray) -> np.ndarray:
    """Round half to even, clip to [-127, 127], cast to int8 (in place on
    floating input)."""
    v = np.rint(v, out=v) if v.dtype.kind == "f" else np.rint(v)
    np.clip(v, -127, 127, out=v)
    return v.astype(np.int8)


def quantise4(v: np.ndarray) -> np.ndarray:
    """Round half to even, clip to the 4-bit two's complement range [-8, 7],
    cast to int8."""
    v = np.rint(v, out=v) if v.dtype.kind == "f" else np.rint(v)
    np.clip(v, -8, 7, out=v)
    return v.astype(np.int8)


def pack4(x: np.ndarray) -> np.ndarray:
    """int8 [...][2] with components in [-8, 7] -> uint8 [...], one byte per
    sample: real part in the high nibble, imaginary part in the low nibble,
    each as 4-bit two's complement."""
    x = np.asarray(x)
    if x.shape[-1] != 2 or x.min(initial=0) < -8 or x.max(initial=0) > 7:
        raise ValueError("pack4 takes [...][2] components in [-8, 7]")
    u = x.astype(np.uint8) & np.uint8(0x0F)
    return (u[..., 0] << np.uint8(4)) | u[..., 1]


def channel_voltages(cfg: int | str, chan: int, n_samples: int, pos: np.ndarray,
                     freq_hz: float, sources: Sequence[Source] = (),
                     sigma: float = SIGMA, t0: int = 0, bits: int = 8) -> np.ndarray:
    """int8 [T][N][2] voltages for one channel (re, im interleaved,
    antenna-fastest), or for ``bits`` = 4 uint8 [T][N] packed samples
    (``pack4``).  Noise is N(0, sigma^2) per component, drawn as float32
    from the (cfg, chan) stream; each source adds amp * envelope(t) *
    exp(+2 pi i f (k_s . r_n) / c0), phases taken in float64 and the product
    formed in complex64.  ``t0`` offsets tone phases only."""
    g = rng(cfg, chan)
    n = pos.shape[0]
    v = g.standard_normal((n_samples, n, 2), dtype=np.float32)
    v *= np.float32(sigma)
    if sources:
        t = np.arange(n_samples, dtype=np.float64) + t0
        for s in sources:
            ph = np.exp(2j * np.pi * freq_hz * (pos @ s.direction) / C0)  # [N]
            if s.kind == "tone":
                env = s.amp * np.exp(2j * np.pi * s.nu * t)
            else:
                env = s.amp * np.exp(1j * g.uniform(0, 2 * np.pi, n_samples))
            src = env.astype(np.complex64)[:, None] * ph.astype(np.complex64)[None, :]
            v[..., 0] += src.real
            v[..., 1] += src.imag
    if bits == 4:
        return pack4(quantise4(v))
    return quantise(v)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    cfg: int
    n_ant: int
    n_chan: int
    n_beams: int
    n_samples: int
    integration: int
    pos: np.ndarray            # [N][3] m
    dirs: np.ndarray           # [B][3] unit
    freqs: np.ndarray          # [C] Hz
    sources: list = field(default_factory=list)
    sigma: float = SIGMA
    input_bits: int = 8        # 8: int8 [C][T][N][2]; 4: packed uint8 [C][T][N]

    @property
    def flops(self) -> float:
        """8 flop per complex multiply-accumulate (Sec. 2.2)."""
        return 8.0 * self.n_chan * self.n_beams * self.n_samples * self.n_ant

    def x_shape(self, n_chan: int, n_samples: int) -> tuple:
        if self.input_bits == 4:
            return (n_chan, n_samples, self.n_ant)
        return (n_chan, n_samples, self.n_ant, 2)

    @property
    def x_dtype(self):
        return np.uint8 if self.input_bits == 4 else np.int8

    def channel(self, c: int, n_samples: Optional[int] = None, t0: int = 0) -> np.ndarray:
        return channel_voltages(self.cfg, c, n_samples or self.n_samples, self.pos,
                                float(self.freqs[c]), self.sources, self.sigma, t0,
                                self.input_bits)

    def voltages(self, channels: Optional[Sequence[int]] = None,
                 n_samples: Optional[int] = None, out: Optional[np.ndarray] = None,
                 workers: int = 1) -> np.ndarray:
        """int8 [len(channels)][T][N][2] (packed uint8 [len(channels)][T][N]
        for a 4-bit workload).  ``workers`` > 1 fills channels in a thread
        pool (numpy releases the GIL in the heavy calls)."""
        chans = list(range(self.n_chan)) if channels is None else list(channels)
        T = n_samples or self.n_samples
        if out is None:
            out = np.empty(self.x_shape(len(chans), T), dtype=self.x_dtype)
        if workers <= 1:
            for i, c in enumerate(chans):
                out[i] = self.channel(c, T)
        else:
            from concurrent.futures import ThreadPoolExecutor

            def fill(ic):
                i, c = ic
                out[i] = self.channel(c, T)
            with ThreadPoolExecutor(workers) as ex:
                list(ex.map(fill, enumerate(chans)))
        return out


def small(n_beams: int = 4, cfg: int | str = "small") -> Workload:
    """N=32 line at 10 m, 128 channels over 400-416 MHz, T=4096, I=1; beams
    at seeded angles in [-30, 30] deg in the x-z plane; a tone of amplitude 32
    at 0.01 cycles/sample arrives from beam 0's direction."""
    N, C, T = 32, 128, 4096
    g = rng(cfg, "point")
    theta = g.uniform(-30.0, 30.0, n_beams)
    dirs = dir_from_xz_angle(theta)
    src = [Source(dirs[0].copy(), 32.0, "tone", 0.01)]
    cid = CFG_IDS[cfg] if isinstance(cfg, str) else cfg
    return Workload("small" if n_beams == 4 else f"small_b{n_beams}", cid, N, C,
                    n_beams, T, 1, line_positions(N), dirs, channel_freqs(C), src)


def precision() -> Workload:
    """The ``small`` array and voltages (same streams) with 512 beams; beam 0
    still points at the tone."""
    w = small(512, cfg="precision")
    base = small()
    w.name = "precision"
    w.cfg = base.cfg            # identical voltages to ``small``
    w.sources = base.sources
    d = w.dirs.copy()
    d[0] = base.dirs[0]
    w.dirs = d
    return w


def paper() -> Workload:
    """BEST-2-like paper-scale block: 4x8 grid, 1024 ch over 16 MHz at
    408 MHz, 128 beams on a 16x8 grid spanning +-15 deg (b = iy*16 + ix),
    65536 samples, I=16, sigma=16 noise plus three noise-like sources of
    amplitude 16 at seeded, distinct beam-grid centres."""
    N, C, B, T = 32, 1024, 128, 65536
    pos = grid_positions(4, 8, 10.0, 20.0)
    tx = np.linspace(-15.0, 15.0, 16)
    ty = np.linspace(-15.0, 15.0, 8)
    TY, TX = np.meshgrid(ty, tx, indexing="ij")
    dirs = dir_from_lm_angles(TX.ravel(), TY.ravel())
    g = rng("paper", "point")
    beams = g.choice(B, size=3, replace=False)
    src = [Source(dirs[b].copy(), 16.0, "noise") for b in beams]
    return Workload("paper", CFG_IDS["paper"], N, C, B, T, 16, pos, dirs,
                    channel_freqs(C, 400e6, 16e6), src)


def four_bit(w: Workload) -> Workload:
    """The same workload with 4-bit packed input (the BEST-2 format): noise and
    sources scaled by SIGMA4 / SIGMA, so the signal-to-noise ratio is kept
    and the draws come from the same streams."""
    import dataclasses
    k = SIGMA4 / w.sigma
    src = [dataclasses.replace(s, amp=s.amp * k) for s in w.sources]
    return dataclasses.replace(w, name=w.name + "_4bit", sources=src, sigma=SIGMA4,
                               input_bits=4)


def random_dirs(n: int, g: np.random.Generator, max_deg: float = 30.0) -> np.ndarray:
    tx = g.uniform(-max_deg, max_deg, n)
    ty = g.uniform(-max_deg, max_deg, n)
    return dir_from_lm_angles(tx, ty)


def batch_sets(n_sets: int = 12) -> list[Workload]:
    """The uneven batch: seeded N, C, B, T per set; noise-only voltages."""
    g = rng("batch", "sets")
    out = []
    for s in range(n_sets):
        N = int(g.choice([16, 32, 64, 128, 256]))
        C = int(g.choice([256, 512, 1024]))
        B = int(g.choice([16, 64, 256, 1024]))
        T = int(g.integers(8, 33)) * 1024
        gs = rng("batch", "geom", s)
        pos = disc_positions(N, 250.0, gs)
        dirs = random_dirs(B, rng("batch", "point", s))
        w = Workload(f"batch{s}", 100 + s, N, C, B, T, 16, pos, dirs,
                     channel_freqs(C, 400e6, 16e6))
        out.append(w)
    return out


SERVE_CHAN_RATE = 16e6 / 1024  # 15.625 kHz per channel


def serve_array() -> np.ndarray:
    return grid_positions(16, 16, 10.0, 10.0)


def serve_block(block: int, n_chan: int = 1024, n_samples: int = 8192) -> Workload:
    """One streaming block of the 256-antenna grid (noise-only voltages).
    Different blocks use different streams (cfg id offset by the block)."""
    pos = serve_array()
    return Workload(f"serve_blk{block}", 1000 + block, 256, n_chan, 0, n_samples, 64,
                    pos, np.zeros((0, 3)), channel_freqs(n_chan, 400e6, 16e6))


def large(n_beams: int = 512) -> Workload:
    """The serving form's block (256-antenna 16x16 grid, 1024 channels x 8192
    samples, I=64, noise-only voltages) as a single plan of ``n_beams``
    seeded directions within 25 deg of zenith."""
    import dataclasses
    dirs = random_dirs(n_beams, rng("serve", "tracking"), 25.0)
    return dataclasses.replace(serve_block(0), name="large", n_beams=n_beams, dirs=dirs)


def serve_block_arrivals(n_blocks: int, period_s: float, pace: float = 1.0) -> np.ndarray:
    """Seeded Poisson arrival times (seconds from the start) of the serving
    form's voltage blocks: exponential gaps with mean ``period_s / pace``
    (a replay ``pace`` times faster than real time)."""
    g = rng("serve", "blocks")
    return np.cumsum(g.exponential(period_s / pace, n_blocks)) - 0.0


def serve_requests(n: int, mean_concurrent_beams: float = 512.0, mean_lifetime: float = 4.0):
    """Seeded beam-set requests for the serving form: Poisson arrivals (in
    block units), beams log-uniform over 64..2048, lifetimes geometric with
    the given mean; the arrival rate makes the mean number of concurrently
    active beams ``mean_concurrent_beams``.  Returns (arrival_block,
    n_beams, lifetime_blocks, dirs) tuples."""
    g = rng("serve", "req")
    mean_b = (2048 - 64) / np.log(2048 / 64)          # mean of log-uniform 64..2048
    rate = mean_concurrent_beams / (mean_lifetime * mean_b)  # requests per block
    reqs = []
    blk = 0.0
    for i in range(n):
        blk += g.exponential(1.0 / rate)
        nb = int(2 ** g.uniform(6, 11))
        life = int(g.geometric(1.0 / mean_lifetime))
        reqs.append((int(blk), nb, life, random_dirs(nb, rng("serve", "reqdirs", i))))
    return reqs
