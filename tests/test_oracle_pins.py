"""Further pins of the oracle against references outside itself.

* Brute force at 30 significant digits (mpmath) of the truncated discrete
  sum of eqs. fftexp and taylors on grids of at most 16 samples per axis,
  with the spectral and displacement axes written out from the Appendix:
  pins the oracle's vectorised, blocked direct sum (its indexing, sign
  conventions and Taylor polynomial) at every order P = 0..3.
* The kernel-level helper tabulate_from_factors (tables from given sampled
  factors, used at sizes where the Green's function and spectra would be
  too slow to sample) against tabulate() fed the factors it samples itself,
  on ray, parabolic, zero-padded and tensor-truncated grids: a wrong contour
  weight, contour ratio, band mask or truncation in the helper fails here.
"""
import math

import numpy as np
import pytest

from oracle import cfft_oracle as co
from workloads import (CONTOUR_PARABOLIC, TRUNC_TENSOR, Grid, Substrate, gaussian_coefficients,
                       rooftop_lattice)

mpmath = pytest.importorskip("mpmath")

K0 = 2 * math.pi


def _mp_axis(n, k_max):
    """Appendix grids at 30 digits: k(i) = -k_max + i 2 k_max / n, D(j) = -x_max + j pi / k_max."""
    km = mpmath.mpf(k_max)
    x_max = n * mpmath.pi / (2 * km)
    ks = [-km + i * 2 * km / n for i in range(n)]
    ds = [-x_max + j * mpmath.pi / km for j in range(n)]
    return ks, ds


def _mp_table(integ, nx, ny, kxm, kym, gamma, order):
    """Z(j1, j2) = dkx dky / 4 pi^2 sum_{n1,n2} I exp(-i k.D) sum_{p<=P} (gamma k.D)^p / p!, term by term."""
    kxs, dxs = _mp_axis(nx, kxm)
    kys, dys = _mp_axis(ny, kym)
    g = mpmath.mpf(gamma)
    scale = (2 * mpmath.mpf(kxm) / nx) * (2 * mpmath.mpf(kym) / ny) / (4 * mpmath.pi ** 2)
    vals = [[mpmath.mpc(complex(integ[n2, n1])) for n1 in range(nx)] for n2 in range(ny)]
    out = np.zeros((ny, nx), dtype=np.complex128)
    for j2 in range(ny):
        for j1 in range(nx):
            acc = mpmath.mpc(0)
            for n2 in range(ny):
                for n1 in range(nx):
                    arg = kxs[n1] * dxs[j1] + kys[n2] * dys[j2]
                    t = mpmath.mpf(0)
                    term = mpmath.mpf(1)
                    for p in range(order + 1):
                        if p:
                            term = term * g * arg / p
                        t += term
                    acc += vals[n2][n1] * mpmath.expj(-arg) * t
            out[j2, j1] = complex(scale * acc)
    return out


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 4), (6, 10)])
def test_direct_sum_against_30_digit_brute_force(nx, ny):
    """The oracle's FP64 direct sum equals the 30-digit term-by-term sum to 1e-13 for P = 0..3."""
    mpmath.mp.dps = 30
    rng = np.random.default_rng(31 + nx * ny)
    kxm, kym = 3.1 * K0, 2.3 * K0
    gamma = 1.0 / 9.0          # large enough that every Taylor term carries weight on these grids
    integ = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    kx, ky = co.grid_samples(nx, ny, kxm, kym)
    DX, DY = np.meshgrid(co.displacement_axis(nx, kxm), co.displacement_axis(ny, kym))
    for order in range(4):
        ref = _mp_table(integ, nx, ny, kxm, kym, gamma, order)
        got = co.direct_sum(integ.reshape(1, -1), kx, ky, DX.ravel(), DY.ravel(), gamma, order,
                            2 * kxm / nx, 2 * kym / ny, block=5).reshape(ny, nx)
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (nx, ny, order, err)


def _factor_case(grid, sub, seed):
    rng = np.random.default_rng(seed)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = np.array([(0, 1), (1, 1), (1, 0)])
    _, _, _, g, mt, mh = co.sampled_factors(grid, sub, basis, q)
    ref = co.tabulate(grid, sub, basis, q, pairs)
    got = co.tabulate_from_factors(grid, pairs, g, mt, mh)
    return np.abs(got - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("variant", ["ray", "parabolic", "zero_padded", "tensor"])
def test_tabulate_from_factors_matches_tabulate(variant):
    sub = Substrate(3.0, 0.001, 0.07)
    grid = Grid(16, 32, 6 * K0, 5 * K0, K0)
    if variant == "parabolic":
        grid.contour = CONTOUR_PARABOLIC
        grid.beta_end = 2.0 * K0 * math.sqrt(sub.eps_r)
    elif variant == "zero_padded":
        grid.zero_pad = 1
    elif variant == "tensor":
        grid.truncation = TRUNC_TENSOR
    assert _factor_case(grid, sub, 7) < 1e-14


def test_tabulate_from_factors_detects_a_wrong_weight():
    """The comparison above is sensitive: factors of another contour height give a different table."""
    sub = Substrate(3.0, 0.001, 0.07)
    grid = Grid(16, 32, 6 * K0, 5 * K0, K0)
    rng = np.random.default_rng(7)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = np.array([(0, 1)])
    other = Grid(16, 32, 6 * K0, 5 * K0, K0, gamma=grid.gamma * 1.5)
    _, _, _, g, mt, mh = co.sampled_factors(grid, sub, basis, q)
    ref = co.tabulate(grid, sub, basis, q, pairs)
    got = co.tabulate_from_factors(other, pairs, g, mt, mh)
    assert np.abs(got - ref).max() / np.abs(ref).max() > 1e-6
