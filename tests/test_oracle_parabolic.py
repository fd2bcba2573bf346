"""Pins of the oracle's parabolic contour (the deformation the paper names:
Sec. I and the caption of Fig. 1; the path of eq. spectral_contour).

Reading: beta_I = gamma beta (1 - beta/beta_end) below beta_end, real beyond;
each sample moves to k_c = (1 + i g) k with g = beta_I/beta; weight
W = (1 + i d beta_I/d beta)(1 + i g) (eq. FFT).
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import cfft_oracle as co
from oracle import ocont
from workloads import COSINE_X, Grid, Substrate, basis_array, gaussian_coefficients, rooftop_lattice

K0 = 2 * math.pi


def test_weight_is_the_jacobian_determinant():
    """W = det(d k_c / d k) by central differences, inside and beyond beta_end."""
    gamma, be = 1 / 40, 3.0 * K0
    rng = np.random.default_rng(1)
    pts = np.concatenate([rng.uniform(-2, 2, (6, 2)) * K0, rng.uniform(2.3, 3.5, (3, 2)) * K0])
    h = 1e-6
    for kx, ky in pts:
        def kc(a, b):
            x, y, _, _ = co.parabolic_contour(np.array([a]), np.array([b]), gamma, be)
            return np.array([x[0], y[0]])
        J = np.column_stack([(kc(kx + h, ky) - kc(kx - h, ky)) / (2 * h), (kc(kx, ky + h) - kc(kx, ky - h)) / (2 * h)])
        w = co.parabolic_contour(np.array([kx]), np.array([ky]), gamma, be)[2][0]
        assert abs(np.linalg.det(J) - w) < 1e-8 * abs(w)


def test_sample_at_the_end_of_the_deformation_takes_the_mean_slope():
    """At beta = beta_end the slope jumps from -gamma to 0: the weight there is
    (1 + i(-gamma/2)) (1 + 0i), whether beta rounds just below or above."""
    gamma, be = 1 / 50, 4.5 * K0
    for b in (be, be * (1 - 1e-15), be * (1 + 1e-15)):
        _, _, w, g = co.parabolic_contour(np.array([b]), np.array([0.0]), gamma, be)
        assert abs(g[0]) < 1e-14
        assert abs(w[0] - (1 - 0.5j * gamma)) < 1e-14
    w_in = co.parabolic_contour(np.array([be * 0.999]), np.array([0.0]), gamma, be)[2][0]
    w_out = co.parabolic_contour(np.array([be * 1.001]), np.array([0.0]), gamma, be)[2][0]
    assert abs(w_in.imag + gamma) < 1e-3 and w_out == 1.0


def test_path_is_the_parabola():
    """k_c . k_c = beta_c^2 with Im beta_c = gamma beta (1 - beta/beta_end), and
    real beyond beta_end."""
    gamma, be = 1 / 30, 2.5 * K0
    beta = np.linspace(0.01, 3.0, 40) * K0
    ang = np.linspace(0.1, 6.0, 40)
    kx, ky = beta * np.cos(ang), beta * np.sin(ang)
    kcx, kcy, _, _ = co.parabolic_contour(kx, ky, gamma, be)
    bc = np.sqrt(kcx * kcx + kcy * kcy)
    expect = np.where(beta < be, gamma * beta * (1 - beta / be), 0.0)
    assert np.allclose(bc.real, beta, rtol=1e-13, atol=0)
    assert np.allclose(bc.imag, expect, rtol=1e-12, atol=1e-15)


def test_large_beta_end_tends_to_the_ray():
    """beta_end -> infinity leaves g = gamma everywhere: the ray contour."""
    rng = np.random.default_rng(2)
    basis = rooftop_lattice(2, 2)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    sub = Substrate(2.2, 0.0, 0.05)
    ray = Grid(16, 16, 6 * K0, 6 * K0, K0)
    par = dataclasses.replace(ray, contour=1, beta_end=1e9 * K0)
    pairs = np.array([(0, 1), (1, 1)])
    zr = co.tabulate(ray, sub, basis, q, pairs)
    zp = co.tabulate(par, sub, basis, q, pairs)
    assert np.abs(zp - zr).max() < 1e-7 * np.abs(zr).max()
    assert np.abs(zp - zr).max() > 0          # the parabolic branch was taken


def test_high_order_and_remainder_bound_with_varying_ratio():
    """With g varying per sample the Taylor form still converges to the
    untruncated sum, within K sum |I| |x|^(P+1)/(P+1)! e^|x|, x = g k.Delta."""
    rng = np.random.default_rng(3)
    nx = ny = 16
    km = 6 * K0
    integ = rng.standard_normal((1, nx * ny)) + 1j * rng.standard_normal((1, nx * ny))
    kx, ky = co.grid_samples(nx, ny, km, km)
    g = co.parabolic_contour(kx, ky, 1 / 30, 5 * K0)[3]
    assert np.ptp(g) > 0.01
    dk = 2 * km / nx
    zi = co.direct_sum(integ, kx, ky, [0.7, -1.1], [0.2, 0.9], g, -1, dk, dk)
    z40 = co.direct_sum(integ, kx, ky, [0.7, -1.1], [0.2, 0.9], g, 40, dk, dk)
    assert np.abs(z40 - zi).max() < 1e-13 * np.abs(zi).max()
    K = dk * dk / (4 * math.pi ** 2)
    for P in range(4):
        zp = co.direct_sum(integ, kx, ky, [0.7, -1.1], [0.2, 0.9], g, P, dk, dk)
        for j, (dx, dy) in enumerate([(0.7, 0.2), (-1.1, 0.9)]):
            x = np.abs(g * (kx * dx + ky * dy))
            bound = K * np.sum(np.abs(integ[0]) * x ** (P + 1) / math.factorial(P + 1) * np.exp(x))
            assert abs(zp[0, j] - zi[0, j]) <= bound * (1 + 1e-12)


@pytest.mark.slow
@pytest.mark.parametrize("delta", [(0.0, 0.0), (0.7, 0.3)])
def test_parabolic_path_matches_ray_and_real_axis(delta):
    """Continuum reaction along the parabola equals the real-axis and ray
    values (Cauchy; lossy slab so the real-axis integral exists)."""
    basis = basis_array([(COSINE_X, 0.0, 0.0, 0.3, 0.2)])
    q = np.ones((1, 1), complex)
    args = (K0, 2.2, 0.3, 0.05, basis, q)
    real = ocont.reaction_polar(delta[0], delta[1], 0.0, 6 * K0, *args, n_alpha=48, points=[K0])
    para = ocont.reaction_polar(delta[0], delta[1], 1 / 20, 6 * K0, *args, n_alpha=48, beta_end=3 * K0)
    ray = ocont.reaction_polar(delta[0], delta[1], 1 / 100, 6 * K0, *args, n_alpha=48)
    assert abs(para - real) < 1e-9 * abs(real)
    assert abs(para - ray) < 1e-9 * abs(real)
