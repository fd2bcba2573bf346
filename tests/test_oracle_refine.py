"""Pins of the x2 zero-padded (Whittaker-Shannon refined) table of Sec.
III-B.3: the padded grid carries the original samples on its central half,
so its table is the original truncated sum evaluated at half the
displacement step."""
import dataclasses
import math

import numpy as np

from oracle import cfft_cpu, cfft_oracle as co
from workloads import Grid, Substrate, gaussian_coefficients, rooftop_lattice

K0 = 2 * math.pi


def _case():
    rng = np.random.default_rng(6)
    base = Grid(16, 8, 6 * K0, 4 * K0, K0, gamma=1 / 40, order=3)
    pad = dataclasses.replace(base, nx=32, ny=16, kx_max=12 * K0, ky_max=8 * K0, zero_pad=1)
    basis = rooftop_lattice(2, 2)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    return base, pad, Substrate(4.4, 0.002, 0.06), basis, q, np.array([(0, 1), (1, 1)])


def test_padded_grid_holds_the_original_samples():
    base, pad, *_ = _case()
    kb, _ = co.grid_samples(base.nx, base.ny, base.kx_max, base.ky_max)
    kp, _ = co.grid_samples(pad.nx, pad.ny, pad.kx_max, pad.ky_max)
    mask = co.band_mask(pad)
    assert mask.sum() == base.nx * base.ny
    assert np.allclose(np.sort(np.unique(kp[mask])), np.sort(np.unique(kb)), rtol=0, atol=1e-12)
    assert np.allclose(co.displacement_axis(pad.nx, pad.kx_max)[::2], co.displacement_axis(base.nx, base.kx_max))


def test_even_nodes_reproduce_the_table_and_odd_nodes_are_midpoint_sums():
    base, pad, sub, basis, q, pairs = _case()
    zb = co.tabulate(base, sub, basis, q, pairs)
    zp = co.tabulate(pad, sub, basis, q, pairs)
    assert np.abs(zp[:, ::2, ::2] - zb).max() <= 1e-13 * np.abs(zb).max()
    # every refined node: the original samples summed at that displacement
    kx, ky, w, g, mt, mh = co.sampled_factors(base, sub, basis, q)
    integ = co.pair_integrands(pairs, w, g, mt, mh)
    DX, DY = np.meshgrid(co.displacement_axis(pad.nx, pad.kx_max), co.displacement_axis(pad.ny, pad.ky_max))
    dkx, dky = 2 * base.kx_max / base.nx, 2 * base.ky_max / base.ny
    ref = co.direct_sum(integ, kx, ky, DX.ravel(), DY.ravel(), base.gamma, base.order, dkx, dky)
    assert np.abs(zp.reshape(2, -1) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_cpu_cfft_on_the_padded_grid():
    _, pad, sub, basis, q, pairs = _case()
    ref = co.tabulate(pad, sub, basis, q, pairs)
    got = cfft_cpu.tabulate_cfft(pad, sub, basis, q, pairs)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
