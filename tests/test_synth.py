"""The seeded input generator: determinism, independence of channel
streams, value ranges and the documented workload shapes."""
import json
import os

import numpy as np

from paper_1412_4907_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def test_channel_streams_are_independent_and_deterministic():
    w = synth.small()
    a = w.voltages(channels=[0, 5, 6], n_samples=256)
    b = w.voltages(channels=[6], n_samples=256)
    assert np.array_equal(a[2], b[0])
    c = w.voltages(channels=[0, 5, 6], n_samples=256, workers=3)
    assert np.array_equal(a, c)
    assert not np.array_equal(a[1], a[2])


def test_value_range_and_rounding():
    w = synth.paper()
    x = w.voltages(channels=[0], n_samples=4096)
    assert x.dtype == np.int8 and x.shape == (1, 4096, 32, 2)
    assert x.min() >= -127 and x.max() <= 127
    # sigma=16 noise plus three amplitude-16 sources: per-component variance
    # 256 + 3 * 128
    assert 600 < x.astype(float).var() < 680
    v = np.array([0.5, 1.5, -0.5, -2.5, 200.0, -300.0])
    assert synth.quantise(v.copy()).tolist() == [0, 2, 0, -2, 127, -127]


def test_workload_shapes():
    s, p, q = synth.small(), synth.paper(), synth.precision()
    assert (s.n_ant, s.n_chan, s.n_beams, s.n_samples, s.integration) == (32, 128, 4, 4096, 1)
    assert (p.n_ant, p.n_chan, p.n_beams, p.n_samples, p.integration) == (32, 1024, 128, 65536, 16)
    assert (q.n_beams, q.integration) == (512, 1)
    assert np.array_equal(q.voltages(channels=[3], n_samples=64),
                          s.voltages(channels=[3], n_samples=64))
    np.testing.assert_allclose(np.linalg.norm(p.dirs, axis=1), 1.0, atol=1e-15)
    assert abs(p.freqs.mean() - 408e6) < 1 and abs(s.freqs[0] - 400.0625e6) < 1
    gold = json.load(open(GOLD))["best2_grid"]
    assert p.pos.shape[0] == gold["elements"]
    sets = synth.batch_sets()
    assert len(sets) == 12
    for b in sets:
        assert b.n_ant in (16, 32, 64, 128, 256) and b.n_chan in (256, 512, 1024)
        assert b.n_beams in (16, 64, 256, 1024) and 8192 <= b.n_samples <= 32768
        assert np.all(np.linalg.norm(b.pos[:, :2], axis=1) <= 250.0)


def test_paper_accounting_numbers():
    g = json.load(open(GOLD))
    f = g["flops_per_beam_channel_sample_per_antenna"]["value"]
    w = synth.paper()
    assert w.flops == f * w.n_chan * w.n_beams * w.n_samples * w.n_ant == 2.199023255552e12
    d = g["best2_data_rate"]
    rate = d["channels"] * d["samples_per_s"] * d["antennas"] * d["bits_per_sample"]
    assert abs(rate / 1e9 - d["gbps"]) < 1e-12
    # the serving block: 8192 samples at 16 MHz / 1024 channels
    assert abs(8192 / synth.SERVE_CHAN_RATE - 0.524288) < 1e-12


def test_four_bit_workload():
    w = synth.four_bit(synth.paper())
    x = w.voltages(channels=[0, 3], n_samples=2048)
    assert x.dtype == np.uint8 and x.shape == (2, 2048, 32)
    assert w.input_bits == 4 and w.sigma == synth.SIGMA4
    # real and imaginary nibbles as 4-bit two's complement, decoded here by
    # sign-extending shifts rather than the oracle's reading
    s = x.view(np.int8)
    re = (s >> 4).astype(float)
    im = ((s << 4).astype(np.int8) >> 4).astype(float)
    assert re.min() >= -8 and re.max() <= 7 and im.min() >= -8 and im.max() <= 7
    # sigma=2 noise plus three noise-like sources of amplitude 2: variance
    # 4 + 3 * 2 = 10 per component, less a little clipping at the rails
    assert 9.0 < re.var() < 10.6 and 9.0 < im.var() < 10.6
    assert np.array_equal(x[1], w.voltages(channels=[3], n_samples=2048)[0])
    v = np.array([0.5, 1.5, -0.5, -8.5, 7.5, -20.0, 20.0])
    assert synth.quantise4(v.copy()).tolist() == [0, 2, 0, -8, 7, -8, 7]
