"""Mutation check of the oracle's pins: each planted slip is compiled into a
temporary copy of bf_oracle.c, and at least one pin in test_oracle_pins must
fail against it.  Mistakes are planted in the oracle, on the CPU."""
import os
import subprocess
import tempfile

import pytest

import oracle
from oracle import build as obuild
from tests import test_oracle_pins as pins

# (name, exact source text, replacement)
MUTANTS = [
    ("phase sign", "w[o + 1] = -sin(phi);", "w[o + 1] = sin(phi);"),
    ("missing 2 pi", "const double two_pi = 2.0 * M_PI;", "const double two_pi = M_PI;"),
    ("missing c0", "freq[c] * kr / BFO_C0;", "freq[c] * kr / (BFO_C0 * 1.0001);"),
    ("wrong component", "dir[3 * b + 1] * pos[3 * n + 1]", "dir[3 * b + 1] * pos[3 * n + 0]"),
    ("conjugated weights (re)", "re += wr * xr - wi * xi;", "re += wr * xr + wi * xi;"),
    ("conjugated weights (im)", "im += wr * xi + wi * xr;", "im += wr * xi - wi * xr;"),
    ("dropped cross term", "re += wr * xr - wi * xi;", "re += wr * xr;"),
    ("window index", "pb[t / I] +=", "pb[t % nwin] +="),
    ("power", "re * re + im * im;", "re * re + im;"),
    ("antenna stride", "double wr = wb[2 * n], wi = wb[2 * n + 1];",
     "double wr = wb[n], wi = wb[n + 1];"),
]

PINS = [
    pins.test_weight_special_values,
    pins.test_weight_modulus_and_frequency_scaling,
    lambda: pins.test_on_beam_plane_wave(1),
    lambda: pins.test_on_beam_plane_wave(4),
    pins.test_on_beam_quantised_bound,
    pins.test_off_source_line_array_dirichlet,
    pins.test_off_source_grid_product_of_dirichlets,
    pins.test_single_live_antenna,
    pins.test_linearity_scaling_and_parallelogram,
    pins.test_brute_force_tiny,
    pins.test_numpy_zgemm,
    pins.test_dft_parseval,
    pins.test_dft_single_bin,
    lambda: pins.test_integration_windows(3),
    lambda: pins.test_integration_windows(16),
]


def _failures():
    n = 0
    for p in PINS:
        try:
            p()
        except Exception:
            n += 1
    return n


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistakes(name, old, new, tmp_path):
    src = open(obuild.SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name!r} not found"
    d = tmp_path
    with open(os.path.join(d, "bf_oracle.h"), "w") as f:
        f.write(open(os.path.join(obuild.HERE, "bf_oracle.h")).read())
    with open(os.path.join(d, "bf_oracle.c"), "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(d, "libmut.so")
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", lib,
                    os.path.join(d, "bf_oracle.c"), "-lm"], check=True)
    prev = oracle.use_library(lib)
    try:
        n = _failures()
    finally:
        oracle.restore_library(prev)
    assert n >= 1, f"no pin caught the planted mistake {name!r}"


def test_unmutated_oracle_passes_every_pin():
    assert _failures() == 0
