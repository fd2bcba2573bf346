"""The CPU C-FFT baseline (eq. fftarry taken literally) against the oracle's
direct sum: the FFT re-association of eqs. fftexp/fftarry is exact, so the
two agree to rounding on every contour and truncation."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import cfft_cpu, cfft_oracle as co
from workloads import CONTOUR_PARABOLIC, TRUNC_TENSOR, Grid, Substrate, gaussian_coefficients, rooftop_lattice

K0 = 2 * math.pi


def test_term_sets():
    assert len(cfft_cpu.terms(3)) == 10                       # eq. fftarry's ten FFT2
    assert len(cfft_cpu.terms(3, TRUNC_TENSOR)) == 16
    assert set(cfft_cpu.terms(2)) <= set(cfft_cpu.terms(2, TRUNC_TENSOR))


@pytest.mark.parametrize("variant", ["ray", "parabolic", "tensor", "zero_padded"])
@pytest.mark.parametrize("order", [0, 2, 3])
def test_matches_direct_sum(variant, order):
    rng = np.random.default_rng(10 + order)
    grid = Grid(32, 16, 7 * K0, 5 * K0, K0, gamma=1 / 40, order=order)
    if variant == "parabolic":
        grid = dataclasses.replace(grid, contour=CONTOUR_PARABOLIC, beta_end=3.5 * K0)
    elif variant == "tensor":
        grid = dataclasses.replace(grid, truncation=TRUNC_TENSOR)
    elif variant == "zero_padded":
        grid = dataclasses.replace(grid, nx=64, ny=32, kx_max=14 * K0, ky_max=10 * K0, zero_pad=1)
    sub = Substrate(4.4, 0.002, 0.06)
    basis = rooftop_lattice(2, 2)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = np.array([(0, 1), (1, 1)])
    ref = co.tabulate(grid, sub, basis, q, pairs)
    got = cfft_cpu.tabulate_cfft(grid, sub, basis, q, pairs)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
