"""CPU C-FFT baseline: eq. fftarry taken literally, one FFT2 per Taylor term.

TEST INFRASTRUCTURE ONLY (a like-for-like CPU implementation of the paper's
algorithm, timed beside the GPU path; its result is checked against the
oracle's direct sum in the tests).

Per pair, with the integrand I on the sample grid (eq. FFT), the modified
integrand I_f = (-1)^(n1+n2) I of the Appendix, and the per-sample contour
ratio g:

    Z(j1, j2) = K' sum_{(a,b)} Dx(j1)^a Dy(j2)^b / (a! b!)
                      FFT2[ (g kx)^a (g ky)^b I_f ](j1, j2)

over the total-degree terms a + b <= P (eq. fftarry; the tensor-product
variant uses a <= P and b <= P), K' = dkx dky / (4 pi^2) sigma (-1)^(j1+j2)
with sigma = exp(-i pi (nx+ny)/2) (Appendix change of variables).  The FFT2
is scipy's, on all the given worker threads.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

from . import cfft_oracle as co


def terms(order: int, truncation: int = 0):
    """(a, b) exponent pairs of the Taylor terms kept."""
    if truncation == 1:
        return [(a, b) for a in range(order + 1) for b in range(order + 1)]
    return [(a, b) for s in range(order + 1) for a in range(s + 1) for b in [s - a]]


def tabulate_cfft(grid, substrate, basis, q, pairs, workers=1, factors=None):
    """Tables [npairs][ny][nx] by one FFT2 per Taylor term (eq. fftarry)."""
    nx, ny = grid.nx, grid.ny
    kx, ky, w, g, mt, mh = factors if factors is not None else co.sampled_factors(grid, substrate, basis, q)
    gam = co.grid_contour(kx, ky, grid)[3]
    gam = np.broadcast_to(np.asarray(gam, dtype=np.float64), kx.shape).reshape(ny, nx)
    gkx = gam * kx.reshape(ny, nx)
    gky = gam * ky.reshape(ny, nx)
    n1 = np.arange(nx)
    n2 = np.arange(ny)
    alt = np.where((n2[:, None] + n1[None, :]) % 2 == 0, 1.0, -1.0)          # (-1)^(n1+n2), also (-1)^(j1+j2)
    dx = co.displacement_axis(nx, grid.kx_max)[None, :]
    dy = co.displacement_axis(ny, grid.ky_max)[:, None]
    sigma = (-1.0) ** (((nx + ny) // 2) % 2)
    kscale = (2.0 * grid.kx_max / nx) * (2.0 * grid.ky_max / ny) / (4.0 * math.pi ** 2) * sigma
    keep = terms(grid.order, getattr(grid, "truncation", 0))
    integ = co.pair_integrands(pairs, w, g, mt, mh)
    mask = co.band_mask(grid)
    if mask is not None:
        integ = integ * mask
    out = np.empty((len(pairs), ny, nx), dtype=np.complex128)
    for p in range(len(pairs)):
        i_f = integ[p].reshape(ny, nx) * alt
        z = np.zeros((ny, nx), dtype=np.complex128)
        for a, b in keep:
            f = scipy.fft.fft2(gkx ** a * gky ** b * i_f, workers=workers)
            z += (dx ** a * dy ** b / (math.factorial(a) * math.factorial(b))) * f
        out[p] = kscale * alt * z
    return out
