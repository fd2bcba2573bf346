"""Pins of the oracle's grounded-slab Green's function remainder.

Checked against textbook physics, not against the oracle itself: the
surface-wave dispersion relations of a grounded slab, equality with the
homogeneous medium + image when eps_r = 1, passivity in the visible region,
decay of the remainder at large beta (the purpose of the extraction named in
Sec. III-A), contour independence of the reaction integral (Cauchy), and a
numerical integration of the transmission-line equations through the slab.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

from oracle import cfft_oracle as co
from oracle import ocont
from workloads import COSINE_X, basis_array

K0 = 2 * math.pi


def _tm_roots(eps, h):
    """Roots in (k0, sqrt(eps) k0) of eps*alpha = k1 tan(k1 h) (textbook TM surface waves)."""
    def f(b):
        a = math.sqrt(b * b - K0 * K0)
        k1 = math.sqrt(eps * K0 * K0 - b * b)
        return eps * a * math.cos(k1 * h) - k1 * math.sin(k1 * h)
    return _roots(f, K0 * (1 + 1e-9), K0 * math.sqrt(eps) * (1 - 1e-9))


def _te_roots(eps, h):
    """Roots of alpha = -k1 cot(k1 h) (textbook TE surface waves)."""
    def f(b):
        a = math.sqrt(b * b - K0 * K0)
        k1 = math.sqrt(eps * K0 * K0 - b * b)
        return a * math.sin(k1 * h) + k1 * math.cos(k1 * h)
    return _roots(f, K0 * (1 + 1e-9), K0 * math.sqrt(eps) * (1 - 1e-9))


def _roots(f, lo, hi, n=4000):
    xs = np.linspace(lo, hi, n)
    vs = [f(x) for x in xs]
    out = []
    for i in range(n - 1):
        if vs[i] == 0 or vs[i] * vs[i + 1] < 0:
            out.append(brentq(f, xs[i], xs[i + 1], xtol=1e-14))
    return out


@pytest.mark.parametrize("eps,h,n_tm,n_te", [(2.2, 0.05, 1, 0), (4.4, 0.06, 1, 0), (10.2, 0.12, 1, 1)])
def test_surface_wave_poles_match_dispersion_relations(eps, h, n_tm, n_te):
    """The immittances have poles exactly at the textbook surface-wave roots."""
    tm = _tm_roots(eps, h)
    te = _te_roots(eps, h)
    assert len(tm) == n_tm and len(te) == n_te
    for b in tm:
        zte, ztm = co.slab_immittances(np.array([b + 0j]), K0, eps, h)
        _, ztm_off = co.slab_immittances(np.array([b * 1.01 + 0j]), K0, eps, h)
        assert abs(1 / ztm[0]) < 1e-9 * abs(1 / ztm_off[0])
    for b in te:
        zte, _ = co.slab_immittances(np.array([b + 0j]), K0, eps, h)
        zte_off, _ = co.slab_immittances(np.array([b * 1.01 + 0j]), K0, eps, h)
        assert abs(1 / zte[0]) < 1e-9 * abs(1 / zte_off[0])


def test_tm0_pole_is_excited_along_propagation():
    """The TM0 surface wave couples to a current along its direction of travel.

    For k along x, Gxx carries the TM immittance and Gyy the TE one, so near
    the TM0 pole (below the TE1 cutoff) Gxx peaks and Gyy stays moderate.
    """
    eps, h = 2.2, 0.05
    bp = _tm_roots(eps, h)[0]
    gamma = 1e-4
    gxx, gxy, gyy = co.green_remainder(np.array([bp]), np.array([0.0]), gamma, K0, eps, 0.0, h)
    assert abs(gxx[0]) > 100 * abs(gyy[0])
    assert abs(gxy[0]) < 1e-12 * abs(gxx[0])
    gxx2, _, gyy2 = co.green_remainder(np.array([0.0]), np.array([bp]), gamma, K0, eps, 0.0, h)
    assert abs(gyy2[0] - gxx[0]) < 1e-9 * abs(gxx[0]) and abs(gxx2[0] - gyy[0]) < 1e-9 * abs(gxx[0])


@pytest.mark.parametrize("eps,td,h", [(2.2, 0.0, 0.05), (4.4, 0.002, 0.06), (10.2, 0.0, 0.12)])
def test_free_space_limit_and_homogeneous_match(eps, td, h):
    """eps_r = 1: slab immittance equals the homogeneous medium + image exactly."""
    rng = np.random.default_rng(11)
    beta = rng.uniform(0, 20 * K0, 200) * (1 + 1j / 130)
    zte, ztm = co.slab_immittances(beta, K0, 1.0, h)
    hte, htm = co.homogeneous_image_immittances(beta, K0, 1.0, h)
    assert np.abs(zte - hte).max() < 1e-13 * np.abs(zte).max()
    assert np.abs(ztm - htm).max() < 1e-13 * np.abs(ztm).max()
    kx, ky = rng.uniform(-15, 15, (2, 100)) * K0
    g = co.green_remainder(kx, ky, 1 / 130, K0, 1.0, 0.0, h)
    assert max(np.abs(c).max() for c in g) < 1e-13


@pytest.mark.parametrize("eps,h", [(2.2, 0.05), (4.4, 0.06), (10.2, 0.12)])
def test_remainder_decays_at_large_beta(eps, h):
    """The extraction leaves a remainder that vanishes as beta grows (Sec. III-A).

    A wrong effective permittivity leaves a TM term growing like beta; a wrong
    branch of k_z in air or in the effective medium makes it blow up.
    """
    betas = np.array([50, 200, 800, 3200]) * K0
    mags = []
    for b in betas:
        g = co.green_remainder(np.array([b]), np.array([0.0]), 1 / 130, K0, eps, 0.0, h)
        mags.append(max(abs(c[0]) for c in g))
    assert all(mags[i + 1] < 0.5 * mags[i] for i in range(len(mags) - 1))
    g2 = co.green_remainder(np.array([2.0 * K0]), np.array([0.0]), 1 / 130, K0, eps, 0.0, h)
    assert mags[-1] < 1e-2 * max(abs(c[0]) for c in g2)


def test_passive_in_visible_region():
    """Re Z_TE, Re Z_TM >= 0 for real beta < k0: power flows into the upper half space."""
    beta = np.linspace(0, 0.999, 200) * K0 + 0j
    for eps, h in [(2.2, 0.05), (10.2, 0.12)]:
        zte, ztm = co.slab_immittances(beta, K0, eps, h)
        assert (zte.real >= -1e-15).all() and (ztm.real >= -1e-15).all()
        assert zte.real.max() > 0 and ztm.real.max() > 0


def test_limit_at_beta_zero_is_isotropic():
    """G(k -> 0) tends to -dZ_TE(0) * identity from every direction."""
    g0 = co.green_remainder(np.array([0.0]), np.array([0.0]), 1 / 130, K0, 4.4, 0.002, 0.06)
    for ang in np.linspace(0, 2 * math.pi, 7):
        r = 1e-7
        g = co.green_remainder(np.array([r * math.cos(ang)]), np.array([r * math.sin(ang)]), 1 / 130, K0, 4.4, 0.002, 0.06)
        assert abs(g[0][0] - g0[0][0]) < 1e-9 and abs(g[2][0] - g0[2][0]) < 1e-9 and abs(g[1][0]) < 1e-9
    assert g0[1][0] == 0 and g0[0][0] == g0[2][0]


def test_even_and_symmetric():
    """G(-k) = G(k); swapping kx and ky swaps Gxx and Gyy."""
    rng = np.random.default_rng(12)
    kx, ky = rng.uniform(-12, 12, (2, 50)) * K0
    a = co.green_remainder(kx, ky, 1 / 130, K0, 4.4, 0.002, 0.06)
    b = co.green_remainder(-kx, -ky, 1 / 130, K0, 4.4, 0.002, 0.06)
    c = co.green_remainder(ky, kx, 1 / 130, K0, 4.4, 0.002, 0.06)
    for u, v in zip(a, b):
        assert np.abs(u - v).max() < 1e-15 * np.abs(u).max() + 1e-300
    assert np.abs(a[0] - c[2]).max() < 1e-14 and np.abs(a[1] - c[1]).max() < 1e-14


def test_transmission_line_ode_through_slab():
    """Shorted slab line: integrate dV/dz, dI/dz numerically and rebuild Z_TE, Z_TM.

    Telegrapher's equations with exp(+i w t): dV/dz = -i kz Zc I,
    dI/dz = -i kz V / Zc, V(0) = 0 at the ground plane; the stub seen from
    z = h has Z_down = -V(h)/I(h) (current entering the stub flows in -z).
    The sheet sees Z_down in parallel with matched air.
    """
    eps, h = 4.4 * (1 - 0.002j), 0.06
    for beta in [0.3 * K0, 1.05 * K0 * (1 + 1j / 130), 3.0 * K0 * (1 + 1j / 130), (8 + 0.5j) * K0]:
        kz1 = np.sqrt(eps * K0 ** 2 - beta ** 2)
        kz0 = co.sqrt_radiating(np.array([K0 ** 2 - beta ** 2]))[0]
        out = []
        for zc_sub, zc_air in [(K0 / kz1, K0 / kz0), (kz1 / (K0 * eps), kz0 / K0)]:
            def rhs(z, y):
                v = y[0] + 1j * y[1]
                i = y[2] + 1j * y[3]
                dv = -1j * kz1 * zc_sub * i
                di = -1j * kz1 * v / zc_sub
                return [dv.real, dv.imag, di.real, di.imag]
            sol = solve_ivp(rhs, (0, h), [0, 0, 1, 0], rtol=1e-12, atol=1e-14, method="DOP853")
            v = sol.y[0, -1] + 1j * sol.y[1, -1]
            i = sol.y[2, -1] + 1j * sol.y[3, -1]
            z_down = -v / i
            out.append(1 / (1 / z_down + 1 / zc_air))
        zte, ztm = co.slab_immittances(np.array([beta]), K0, eps, h)
        assert abs(out[0] - zte[0]) < 1e-8 * abs(zte[0])
        assert abs(out[1] - ztm[0]) < 1e-8 * abs(ztm[0])


@pytest.mark.slow
@pytest.mark.parametrize("delta", [(0.0, 0.0), (0.7, 0.3), (-1.2, 0.9)])
def test_contour_independence(delta):
    """The reaction integral is the same along the real axis and two ray contours.

    With a lossy slab (tan delta = 0.3) the surface-wave poles leave the real
    axis, so the real-axis integral is defined; Cauchy's theorem then requires
    every path with the same end points to agree, which pins the branches of
    the vertical wavenumbers and the absence of spurious singularities.
    """
    basis = basis_array([(COSINE_X, 0.0, 0.0, 0.3, 0.2)])
    q = np.ones((1, 1), complex)
    vals = []
    for gamma in [0.0, 1 / 100, 1 / 200]:
        vals.append(ocont.reaction_polar(delta[0], delta[1], gamma, 6 * K0, K0, 2.2, 0.3, 0.05, basis, q,
                                         n_alpha=48, points=[K0] if gamma == 0 else None))
    assert abs(vals[1] - vals[0]) < 1e-9 * abs(vals[0])
    assert abs(vals[2] - vals[0]) < 1e-9 * abs(vals[0])
