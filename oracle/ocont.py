"""Continuum reaction integral by polar quadrature along a deformed contour.

TEST INFRASTRUCTURE ONLY (accuracy reference and contour-independence pin).

eq. polarcord writes the reaction in polar spectral coordinates; eq.
spectral_contour deforms the radial path into the complex beta plane and
integrates along it with the Jacobian of the path.  Here the radial path is
the ray beta_c = (1 + i gamma) t, t in [0, B], closed back to the real axis by
the vertical segment from B(1 + i gamma) to B, or the parabolic path that
returns to the real axis at beta_end, so that every path shares the same
end point and (by Cauchy's theorem, the integrand being analytic between the
paths) the same value.  gamma = 0 is the real axis itself.  The angle is
integrated with the trapezoidal rule (periodic integrand), the radial path
adaptively (scipy quad_vec), all in FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad_vec

from . import cfft_oracle as co


def _kernel(beta_c, dbeta, alphas, dx, dy, k0, eps_r, tan_delta, h, basis, q, m, n, green_one):
    c = np.cos(alphas)
    s = np.sin(alphas)
    kcx = beta_c * c
    kcy = beta_c * s
    if green_one:
        gxx = np.ones_like(kcx)
        gxy = np.zeros_like(kcx)
        gyy = np.ones_like(kcx)
    else:
        gxx, gxy, gyy = co.green_polar(beta_c * np.ones_like(c), c, s, k0, eps_r, tan_delta, h)
    mt, mh = co.mbf_spectra(basis, q, kcx, kcy)
    hm = co.integrand(mt[m], mh[n], gxx, gxy, gyy, 1.0)
    # beta_c d beta_c d alpha, exp(-i k_c . Delta)
    return hm * np.exp(-1j * (kcx * dx + kcy * dy)) * beta_c * dbeta


def reaction_polar(dx, dy, gamma, beta_max, k0, eps_r, tan_delta, h, basis, q, m=0, n=0,
                   n_alpha=64, green_one=False, epsabs=1e-13, epsrel=1e-11, points=None, beta_end=None):
    """Z_mn(Delta) = 1/(4 pi^2) int d alpha int_path beta_c d beta_c H(k_c) e^{-i k_c.Delta}.

    beta_end given: the parabolic path beta_c = t + i gamma t (1 - t/beta_end)
    for t in [0, beta_end], then the real axis up to beta_max (no closing
    segment is needed, the path already ends on the real axis)."""
    alphas = 2.0 * math.pi * np.arange(n_alpha) / n_alpha
    if beta_end is not None:
        def para(t):
            bc = t + 1j * gamma * t * (1.0 - t / beta_end)
            dbc = 1.0 + 1j * gamma * (1.0 - 2.0 * t / beta_end)
            return _kernel(bc, dbc, alphas, dx, dy, k0, eps_r, tan_delta, h, basis, q, m, n, green_one)
        total, _ = quad_vec(para, 0.0, beta_end, epsabs=epsabs, epsrel=epsrel)
        if beta_max > beta_end:
            def real(t):
                return _kernel(t + 0j, 1.0, alphas, dx, dy, k0, eps_r, tan_delta, h, basis, q, m, n, green_one)
            rest, _ = quad_vec(real, beta_end, beta_max, epsabs=epsabs, epsrel=epsrel)
            total = total + rest
        return np.sum(total) * (2.0 * math.pi / n_alpha) / (4.0 * math.pi ** 2)
    s = 1.0 + 1j * gamma

    def ray(t):
        return _kernel(s * t, s, alphas, dx, dy, k0, eps_r, tan_delta, h, basis, q, m, n, green_one)

    total, _ = quad_vec(ray, 0.0, beta_max, epsabs=epsabs, epsrel=epsrel, points=points)
    if gamma != 0.0:
        def seg(u):
            # from B(1 + i gamma) down to B: beta_c = B + i gamma B (1 - u), d beta_c = -i gamma B du
            return _kernel(beta_max + 1j * gamma * beta_max * (1.0 - u), -1j * gamma * beta_max,
                           alphas, dx, dy, k0, eps_r, tan_delta, h, basis, q, m, n, green_one)
        tail, _ = quad_vec(seg, 0.0, 1.0, epsabs=epsabs, epsrel=epsrel)
        total = total + tail
    return np.sum(total) * (2.0 * math.pi / n_alpha) / (4.0 * math.pi ** 2)
