"""Pins of the oracle's reduced-matrix fill (Sec. II eq. MBF: an MA x MA
matrix of MBF interaction blocks; Sec. III-B.1 and Sec. III-B.3, last
paragraph: the blocks are read from the table by low-order interpolation at
the relative displacement of the two elements).

Reading: Delta = r_test - r_basis (the sign convention of the table), row
i*M + m for MBF m of testing element i, column j*M + n for MBF n of basis
element j; self blocks are left to the caller.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import cfft_oracle as co
from workloads import Grid, Substrate, gaussian_coefficients, rooftop_lattice

K0 = 2 * math.pi


@pytest.mark.parametrize("order", [1, 2])
def test_node_aligned_layout_reads_the_table(order):
    """Elements on a lattice of the table's displacement step: every entry is
    the table value at the node found by integer index arithmetic."""
    rng = np.random.default_rng(1)
    grid = Grid(32, 16, 7 * K0, 5 * K0, K0)
    pairs = [(0, 1), (1, 1), (2, 0)]
    table = rng.standard_normal((3, 16, 32)) + 1j * rng.standard_normal((3, 16, 32))
    d_x, d_y = math.pi / grid.kx_max, math.pi / grid.ky_max
    cells = np.array([(0, 0), (3, -2), (-5, 1), (2, 3), (-1, -3)])
    pos = cells * np.array([d_x, d_y])
    f = co.fill_reduced(grid, table, pairs, 3, pos, order=order)
    assert f.shape == (15, 15)
    for i in range(5):
        for j in range(5):
            blk = f[3 * i:3 * i + 3, 3 * j:3 * j + 3]
            if i == j:
                assert np.all(np.isnan(blk))
                continue
            j1 = 16 + cells[i, 0] - cells[j, 0]
            j2 = 8 + cells[i, 1] - cells[j, 1]
            for p, (m, n) in enumerate(pairs):
                assert abs(blk[m, n] - table[p, j2, j1]) <= 1e-13 * abs(table[p, j2, j1])
            listed = np.zeros((3, 3), dtype=bool)
            for m, n in pairs:
                listed[m, n] = True
            assert np.all(np.isnan(blk[~listed]))


def test_displacements_outside_the_table_are_nan():
    grid = Grid(16, 16, 6 * K0, 6 * K0, K0)
    table = np.ones((1, 16, 16), dtype=np.complex128)
    x_max = 16 * math.pi / (2 * grid.kx_max)
    pos = np.array([(0.0, 0.0), (0.3 * x_max, 0.0), (1.5 * x_max, 0.0)])
    f = co.fill_reduced(grid, table, [(0, 0)], 1, pos)
    assert abs(f[0, 1] - 1) < 1e-14 and abs(f[1, 0] - 1) < 1e-14
    assert np.isnan(f[2, 0]) and np.isnan(f[0, 2]) and np.isnan(f[1, 2])


@pytest.mark.parametrize("order", [1, 2])
def test_fill_of_a_refined_table_within_the_interpolation_bound(order):
    """Off-node layout on a x2 zero-padded table: each entry differs from the
    direct sum of the samples at the exact displacement by at most the
    interpolation remainder.  With f(D) = K sum_n I_n e^{-ik.D} T_P(gamma k.D)
    and |T_P^(r)(z)| <= e^{|z|}, |d^r f/dDx^r| <= K sum |I| |kx|^r
    (1 + gamma)^r e^{gamma |k.D|}.  Three-node Lagrange error per axis with
    |t| <= 1/2: h^3 max|f'''| / 16; the tensor form adds the x-weights'
    absolute sum (<= 5/4) on the y error.  Two-node (bilinear) error:
    h^2 max|f''| / 8 per axis."""
    rng = np.random.default_rng(5)
    base = Grid(16, 16, 6 * K0, 6 * K0, K0, order=3)
    pad = dataclasses.replace(base, nx=32, ny=32, kx_max=12 * K0, ky_max=12 * K0, zero_pad=1)
    sub = Substrate(4.4, 0.002, 0.06)
    basis = rooftop_lattice(2, 2)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = np.array([(0, 0), (0, 1), (1, 0), (1, 1)])
    table = co.tabulate(pad, sub, basis, q, pairs)
    pos = rng.uniform(-0.3, 0.3, (5, 2))
    f = co.fill_reduced(pad, table, pairs, 2, pos, order=order)
    kx, ky, w, g, mt, mh = co.sampled_factors(pad, sub, basis, q)
    integ = co.pair_integrands(pairs, w, g, mt, mh) * co.band_mask(pad)
    ii, jj = np.nonzero(~np.eye(5, dtype=bool))
    d = pos[ii] - pos[jj]
    dk = 2 * pad.kx_max / pad.nx
    exact = co.direct_sum(integ, kx, ky, d[:, 0], d[:, 1], pad.gamma, pad.order, dk, dk)
    h = math.pi / pad.kx_max
    K = dk * dk / (4 * math.pi ** 2)
    gam = pad.gamma
    reach = np.exp(gam * (np.abs(kx)[None, :] * (np.abs(d[:, 0])[:, None] + 1.5 * h)
                          + np.abs(ky)[None, :] * (np.abs(d[:, 1])[:, None] + 1.5 * h)))
    r = order + 1
    for p, (m, n) in enumerate(pairs):
        mx = K * np.sum(np.abs(integ[p])[None, :] * (np.abs(kx) * (1 + gam))[None, :] ** r * reach, axis=1)
        my = K * np.sum(np.abs(integ[p])[None, :] * (np.abs(ky) * (1 + gam))[None, :] ** r * reach, axis=1)
        bound = (mx + 1.25 * my) * h ** 3 / 16 if order == 2 else (mx + my) * h ** 2 / 8
        err = np.abs(f[ii * 2 + m, jj * 2 + n] - exact[p])
        assert np.all(err <= bound)
        assert np.all(bound < 0.05 * np.abs(exact[p]).max())     # the bound is informative
