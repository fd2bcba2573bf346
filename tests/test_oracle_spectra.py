"""Pins of the oracle's basis-function and MBF spectra.

The closed forms are checked against Gauss-Legendre quadrature of the spatial
definition F(k) = int f(r) exp(-i k.r) dr at complex k, and the MBF
assembly against the analytic-reflection identity M#(k) = conj(M(conj k)).
"""
import math

import numpy as np
import pytest

from oracle import cfft_oracle as co
from workloads import COSINE_X, COSINE_Y, ROOFTOP_X, ROOFTOP_Y, basis_array, rooftop_lattice

K0 = 2 * math.pi


def _quad_ft(kind, cx, cy, a, b, kx, ky, n=200):
    """Spatial Fourier integral of one basis function by tensor Gauss-Legendre."""
    xg, wg = np.polynomial.legendre.leggauss(n)
    if kind in (ROOFTOP_X, ROOFTOP_Y):
        # triangle: integrate the two halves separately (kink at the centre)
        t = np.concatenate([(xg - 1) * a / 2, (xg + 1) * a / 2])
        wt = np.concatenate([wg, wg]) * a / 2
        ft = 1 - np.abs(t) / a
    else:
        t = xg * a / 2
        wt = wg * a / 2
        ft = np.cos(math.pi * t / a)
    u = xg * b / 2
    wu = wg * b / 2
    if kind in (ROOFTOP_X, COSINE_X):
        X, Y = np.meshgrid(t + cx, u + cy, indexing="ij")
        F = np.outer(ft * wt, wu)
    else:
        X, Y = np.meshgrid(u + cx, t + cy, indexing="ij")
        F = np.outer(wu, ft * wt)
    return np.sum(F * np.exp(-1j * (kx * X + ky * Y)))


@pytest.mark.parametrize("kind", [ROOFTOP_X, ROOFTOP_Y, COSINE_X, COSINE_Y])
def test_basis_ft_matches_quadrature(kind):
    rng = np.random.default_rng(21)
    cx, cy, a, b = 0.11, -0.07, 0.06, 0.03
    if kind in (COSINE_X, COSINE_Y):
        a, b = 0.3, 0.02
    for _ in range(8):
        k = rng.uniform(-60, 60, 2) * (1 + 1j / 130)
        want = _quad_ft(kind, cx, cy, a, b, k[0], k[1])
        got = co.basis_ft(kind, cx, cy, a, b, np.array([k[0]]), np.array([k[1]]))[0]
        assert abs(got - want) < 1e-12 * max(1e-3, abs(want))


def test_cosine_ft_at_removable_points():
    """kx L = +-pi is a removable point of the half-cosine transform."""
    L, W = 0.3, 0.02
    for kx in [math.pi / L, -math.pi / L, 0.0]:
        got = co.basis_ft(COSINE_X, 0, 0, L, W, np.array([kx + 0j]), np.array([0j]))[0]
        want = _quad_ft(COSINE_X, 0, 0, L, W, kx, 0.0)
        assert abs(got - want) < 1e-13


def test_reflection_is_conjugate_of_conjugated_argument():
    """M#_n(k_c) = conj(M_n(conj k_c)): the analytic reflection of eq. MBF_mul22's conjugate."""
    rng = np.random.default_rng(22)
    basis = rooftop_lattice(3, 4)
    q = rng.standard_normal((2, basis.shape[0])) + 1j * rng.standard_normal((2, basis.shape[0]))
    kx, ky = rng.uniform(-40, 40, (2, 30))
    kcx, kcy, _ = co.ray_contour(kx, ky, 1 / 130)
    mt, mh = co.mbf_spectra(basis, q, kcx, kcy)
    mt_c, _ = co.mbf_spectra(basis, q, np.conj(kcx), np.conj(kcy))
    assert np.abs(mh - np.conj(mt_c)).max() < 1e-13 * np.abs(mh).max()
    # on the real axis the reflection is the plain conjugate of eq. FTMBF's spectrum
    mt_r, mh_r = co.mbf_spectra(basis, q, kx + 0j, ky + 0j)
    assert np.abs(mh_r - np.conj(mt_r)).max() < 1e-13 * np.abs(mh_r).max()


def test_lattice_geometry():
    """B = 256 lattice: 128 x- and 128 y-rooftops inside the 0.5 x 0.5 patch."""
    b = rooftop_lattice(8, 16)
    assert b.shape[0] == 256
    assert (b["kind"][:128] == ROOFTOP_X).all() and (b["kind"][128:] == ROOFTOP_Y).all()
    xs = b["cx"][:128]
    assert abs(xs.min() + 0.25 - 0.5 / 9) < 1e-15 and abs(xs.max() - 0.25 + 0.5 / 9) < 1e-15
    # every rooftop lies inside the patch: the triangle (half-base a) along its
    # current and the strip (width b) across it
    xr, yr = b[:128], b[128:]
    assert (np.abs(xr["cx"]) + xr["a"] <= 0.25 + 1e-12).all()
    assert (np.abs(xr["cy"]) + xr["b"] / 2 <= 0.25 + 1e-12).all()
    assert (np.abs(yr["cy"]) + yr["a"] <= 0.25 + 1e-12).all()
    assert (np.abs(yr["cx"]) + yr["b"] / 2 <= 0.25 + 1e-12).all()
    # and they tile it: the outermost triangles and strips touch the patch edges
    assert abs(np.abs(xr["cx"]).max() + xr["a"][0] - 0.25) < 1e-12
    assert abs(np.abs(yr["cx"]).max() + yr["b"][0] / 2 - 0.25) < 1e-12
