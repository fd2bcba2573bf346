"""Pin of the oracle's loss gradient against central finite differences.

The oracle differentiates the lookup loss with a Cauchy-integral rule for
eps_r and h and with the exact sesquilinear form for q; both are checked here
against central differences (step 1e-6) of the oracle's own forward loss.
"""
import math

import numpy as np

from oracle import cfft_oracle as co
from workloads import Grid, Substrate, rooftop_lattice

K0 = 2 * math.pi


def _problem():
    rng = np.random.default_rng(31)
    grid = Grid(16, 16, 6 * K0, 6 * K0, K0)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(1, 2)
    q = rng.standard_normal((2, basis.shape[0])) + 1j * rng.standard_normal((2, basis.shape[0]))
    pairs = np.array([(0, 0), (0, 1), (1, 0), (1, 1)], dtype=np.int32)
    dxa = co.displacement_axis(16, grid.kx_max)
    pts = rng.uniform(dxa[0], dxa[-2], (5, 2))
    zt = co.lookup_direct(grid, Substrate(2.3, 0.0, 0.05), basis,
                          q + 0.1 * (rng.standard_normal(q.shape) + 1j * rng.standard_normal(q.shape)), pairs, pts)
    return grid, sub, basis, q, pairs, pts, zt


def test_gradient_matches_central_differences():
    grid, sub, basis, q, pairs, pts, zt = _problem()
    loss, d_eps, d_h, gq = co.loss_gradient(grid, sub, basis, q, pairs, pts, zt)
    step = 1e-6

    def L(eps=sub.eps_r, h=sub.h, qq=q):
        return co.loss_value(co.lookup_direct(grid, Substrate(eps, 0.0, h), basis, qq, pairs, pts), zt)
    fd_eps = (L(eps=sub.eps_r + step) - L(eps=sub.eps_r - step)) / (2 * step)
    fd_h = (L(h=sub.h + step) - L(h=sub.h - step)) / (2 * step)
    assert abs(d_eps - fd_eps) < 1e-6 * abs(fd_eps)
    assert abs(d_h - fd_h) < 1e-6 * abs(fd_h)
    for (m, j) in [(0, 0), (1, 3), (0, 2)]:
        dq = np.zeros_like(q)
        dq[m, j] = step
        fd_re = (L(qq=q + dq) - L(qq=q - dq)) / (2 * step)
        fd_im = (L(qq=q + 1j * dq) - L(qq=q - 1j * dq)) / (2 * step)
        assert abs(gq[m, j] - (fd_re + 1j * fd_im)) < 1e-6 * np.abs(gq).max()


def test_second_order_lookup_on_a_refined_grid():
    """Second-order lookups in a x2 zero-padded table (the paper's table use,
    Sec. III-B.3): the node-by-node lookup equals quadratic_lookup of the
    whole table, and the loss gradient (band samples only) matches central
    differences of the oracle's own loss."""
    import dataclasses
    rng = np.random.default_rng(37)
    base = Grid(16, 16, 6 * K0, 6 * K0, K0)
    grid = dataclasses.replace(base, nx=32, ny=32, kx_max=12 * K0, ky_max=12 * K0, zero_pad=1)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(1, 2)
    q = rng.standard_normal((2, basis.shape[0])) + 1j * rng.standard_normal((2, basis.shape[0]))
    pairs = np.array([(0, 1), (1, 1)], dtype=np.int32)
    dxa = co.displacement_axis(32, grid.kx_max)
    pts = rng.uniform(dxa[0], dxa[-1], (5, 2))
    table = co.tabulate(grid, sub, basis, q, pairs)
    direct = co.lookup_direct(grid, sub, basis, q, pairs, pts, order=2)
    assert np.abs(direct - co.quadratic_lookup(grid, table, pts)).max() < 1e-12 * np.abs(direct).max()
    zt = co.lookup_direct(grid, Substrate(2.3, 0.0, 0.05), basis, q * 1.1, pairs, pts, order=2)
    loss, d_eps, d_h, gq = co.loss_gradient(grid, sub, basis, q, pairs, pts, zt, order=2)
    step = 1e-6

    def L(eps=sub.eps_r, h=sub.h, qq=q):
        return co.loss_value(co.lookup_direct(grid, Substrate(eps, 0.0, h), basis, qq, pairs, pts, order=2), zt)
    assert abs(loss - L()) <= 1e-14 * loss
    fd_eps = (L(eps=sub.eps_r + step) - L(eps=sub.eps_r - step)) / (2 * step)
    fd_h = (L(h=sub.h + step) - L(h=sub.h - step)) / (2 * step)
    assert abs(d_eps - fd_eps) < 1e-6 * abs(fd_eps)
    assert abs(d_h - fd_h) < 1e-6 * abs(fd_h)
    for m, j in [(0, 0), (1, 3)]:
        d = np.zeros_like(q)
        d[m, j] = step
        fr = (L(qq=q + d) - L(qq=q - d)) / (2 * step)
        fi = (L(qq=q + 1j * d) - L(qq=q - 1j * d)) / (2 * step)
        assert abs(gq[m, j] - (fr + 1j * fi)) < 1e-6 * np.abs(gq).max()
