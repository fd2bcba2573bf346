"""Pins of the oracle's grid, contour, Taylor truncation and direct sum.

Each test checks the oracle against something other than itself: a library
FFT, a closed-form correlation, the coefficients printed in eq. fftarry, an
exact invariant, or brute-force arithmetic.
"""
import math
import os

import numpy as np
import pytest

from oracle import cfft_oracle as co
from workloads import COSINE_X, ROOFTOP_X, ROOFTOP_Y, Grid, Substrate, basis_array, rooftop_lattice

HERE = os.path.dirname(os.path.abspath(__file__))
K0 = 2 * math.pi


def _rng(seed=0):
    return np.random.default_rng(1000 + seed)


@pytest.mark.parametrize("nx,ny", [(16, 16), (6, 8), (8, 12), (10, 10)])
def test_p0_equals_library_fft2(nx, ny):
    """At P = 0 the sum is a centred 2-D DFT (Appendix change of variables).

    Z(j1,j2) = K' sigma (-1)^(j1+j2) FFT2[(-1)^(n1+n2) I](j1,j2) with
    K' = dkx dky / 4 pi^2 and the global phase sigma = exp(-i pi (nx+ny)/2)
    that the printed K' leaves out (it is 1 when (nx+ny)/2 is even).
    """
    rng = _rng(1)
    kxm, kym = 3.7 * K0, 2.9 * K0
    integ = rng.standard_normal((ny, nx)) + 1j * rng.standard_normal((ny, nx))
    kx, ky = co.grid_samples(nx, ny, kxm, kym)
    dxa = co.displacement_axis(nx, kxm)
    dya = co.displacement_axis(ny, kym)
    DX, DY = np.meshgrid(dxa, dya)
    dkx, dky = 2 * kxm / nx, 2 * kym / ny
    z = co.direct_sum(integ.reshape(1, -1), kx, ky, DX.ravel(), DY.ravel(), 0.3, 0, dkx, dky)
    z = z.reshape(ny, nx)
    n2, n1 = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    sign = (-1.0) ** (n1 + n2)
    sigma = np.exp(-1j * math.pi * (nx + ny) / 2)
    ref = dkx * dky / (4 * math.pi ** 2) * sigma * sign * np.fft.fft2(sign * integ)
    assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()


def test_grid_spacings_from_appendix():
    """dk * dDelta = 2 pi / N and Delta = 0 sits at index N/2 (Appendix)."""
    for n, km in [(64, 8 * K0), (512, 10.488 * K0), (6, 1.0)]:
        k = co.spectral_axis(n, km)
        d = co.displacement_axis(n, km)
        assert abs((k[1] - k[0]) * (d[1] - d[0]) - 2 * math.pi / n) < 1e-12
        assert abs(k[0] + km) < 1e-12 and abs(d[n // 2]) < 1e-12 and abs(k[n // 2]) < 1e-12


def test_taylor_coefficients_match_eq_fftarry():
    """T_3(gamma(kx dx + ky dy)) expands to the ten FFT2 terms printed in eq. fftarry."""
    rows = [tuple(float(v) for v in line.split()) for line in open(os.path.join(HERE, "golden", "fftarry_coefficients.txt"))
            if line.strip() and not line.startswith("#")]
    rng = _rng(2)
    g = 0.37
    for _ in range(20):
        kx, ky, dx, dy = rng.uniform(-3, 3, 4)
        poly = co.taylor_poly(np.array([g * (kx * dx + ky * dy)]), 3)[0]
        printed = sum(c * dx ** a * dy ** b * (g * kx) ** a * (g * ky) ** b for a, b, c in rows)
        assert abs(poly - printed) < 1e-12 * max(1.0, abs(printed))
    assert len(rows) == 10                     # N_t = (P+1)(P+2)/2 at P = 3


def test_taylor_converges_to_exponential():
    """High-order truncation equals the untruncated E_I (eq. taylors)."""
    rng = _rng(3)
    nx = ny = 16
    kxm = kym = 4 * K0
    integ = rng.standard_normal((2, nx * ny)) + 1j * rng.standard_normal((2, nx * ny))
    kx, ky = co.grid_samples(nx, ny, kxm, kym)
    dx = rng.uniform(-1, 1, 7)
    dy = rng.uniform(-1, 1, 7)
    dk = 2 * kxm / nx
    z40 = co.direct_sum(integ, kx, ky, dx, dy, 1 / 130, 40, dk, dk)
    zex = co.direct_sum(integ, kx, ky, dx, dy, 1 / 130, -1, dk, dk)
    assert np.abs(z40 - zex).max() <= 1e-13 * np.abs(zex).max()


def test_taylor_remainder_bound():
    """|Z^(P) - Z^(inf)| <= dk^2/4pi^2 sum |I| |x|^(P+1)/(P+1)! e^|x|, x = gamma k.Delta."""
    rng = _rng(4)
    nx = ny = 16
    km = 6 * K0
    gamma = 1 / 60
    integ = rng.standard_normal((1, nx * ny)) + 1j * rng.standard_normal((1, nx * ny))
    kx, ky = co.grid_samples(nx, ny, km, km)
    dk = 2 * km / nx
    for dx, dy in [(0.3, -0.2), (0.9, 0.7), (-0.6, 0.0)]:
        for p in range(4):
            zp = co.direct_sum(integ, kx, ky, [dx], [dy], gamma, p, dk, dk)[0, 0]
            zi = co.direct_sum(integ, kx, ky, [dx], [dy], gamma, -1, dk, dk)[0, 0]
            x = np.abs(gamma * (kx * dx + ky * dy))
            bound = dk * dk / (4 * math.pi ** 2) * np.sum(np.abs(integ[0]) * x ** (p + 1) / math.factorial(p + 1) * np.exp(x))
            assert abs(zp - zi) <= bound * (1 + 1e-12)


def test_delta_zero_independent_of_order():
    """At Delta = 0, E_I = 1, so every truncation order gives the same entry."""
    grid = Grid(16, 16, 6 * K0, 6 * K0, K0)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(2, 2)
    q = np.array([[1 + 2j, -0.5j, 0.3, 1.0, 0.2 - 0.1j, 0.0, 1j, 0.7]], dtype=complex)
    idx = np.array([8 * 16 + 8])                       # j = N/2 in both axes
    vals = [co.tabulate(grid, sub, basis, q, np.array([[0, 0]]), out_idx=idx, order=p)[0, 0] for p in range(4)]
    for v in vals[1:]:
        assert abs(v - vals[0]) <= 1e-14 * abs(vals[0])


def test_contour_weight_is_jacobian():
    """W = (1 + i gamma)^2 = det(d k_c / d k) (eq. FFT weight), by central differences."""
    gamma = 0.13
    kx0, ky0, h = 1.7, -0.4, 1e-6

    def kc(kx, ky):
        a, b, _ = co.ray_contour(np.array(kx), np.array(ky), gamma)
        return complex(a), complex(b)
    j11 = (kc(kx0 + h, ky0)[0] - kc(kx0 - h, ky0)[0]) / (2 * h)
    j12 = (kc(kx0, ky0 + h)[0] - kc(kx0, ky0 - h)[0]) / (2 * h)
    j21 = (kc(kx0 + h, ky0)[1] - kc(kx0 - h, ky0)[1]) / (2 * h)
    j22 = (kc(kx0, ky0 + h)[1] - kc(kx0, ky0 - h)[1]) / (2 * h)
    det = j11 * j22 - j12 * j21
    w = co.ray_contour(np.array(kx0), np.array(ky0), gamma)[2]
    assert abs(det - w) < 1e-8
    # eq. complexbeta: kcx^2 + kcy^2 = beta_c^2 with beta_c = (1 + i gamma) beta
    a, b = kc(kx0, ky0)
    assert abs(a * a + b * b - ((1 + 1j * gamma) * math.hypot(kx0, ky0)) ** 2) < 1e-12


def _corr_cosine(dx, dy, length, width):
    d = np.abs(dx)
    c = np.where(d <= length, 0.5 * (length - d) * np.cos(np.pi * d / length)
                 + length / (2 * np.pi) * np.sin(np.pi * d / length), 0.0)
    return c * np.maximum(width - np.abs(dy), 0.0)


@pytest.mark.parametrize("gamma", [0.0, 0.05])
def test_unit_green_gives_current_correlation(gamma):
    """With G = identity the reaction is the spatial correlation of the two currents.

    The integrand M_m . M#_n is entire, so deforming the contour does not
    change the integral when the weight W of eq. FFT is right; the rectangle
    rule converges to int f_m(r) f_n(r + Delta) dr, here for two half-cosine
    patches, the basis one shifted by c = (0.1, 0.05) so that the sign of
    Delta and the reflection F(-k_c) on the basis side are both exercised.
    Without W the deformed result is off by ~10 % (checked below).
    """
    L = Wd = 0.3
    c = (0.1, 0.05)
    basis = basis_array([(COSINE_X, 0.0, 0.0, L, Wd), (COSINE_X, c[0], c[1], L, Wd)])
    q = np.eye(2, dtype=complex)
    n, km = 256, 32 * K0
    kx, ky = co.grid_samples(n, n, km, km)
    kcx, kcy, w = co.ray_contour(kx, ky, gamma)
    mt, mh = co.mbf_spectra(basis, q, kcx, kcy)
    one, zero = np.ones_like(kcx), np.zeros_like(kcx)
    integ = co.integrand(mt[0], mh[1], one, zero, one, w)[None]
    pts = np.array([[0.0, 0.0], [0.1, 0.05], [0.2, -0.1], [-0.15, 0.2], [0.45, 0.1], [0.3, 0.3]])
    dk = 2 * km / n
    z = co.direct_sum(integ, kx, ky, pts[:, 0], pts[:, 1], gamma, -1, dk, dk)[0]
    ref = _corr_cosine(pts[:, 0] - c[0], pts[:, 1] - c[1], L, Wd)
    err = np.abs(z - ref).max() / np.abs(ref).max()
    assert err < 0.015
    if gamma > 0:
        z_now = co.direct_sum(integ / w, kx, ky, pts[:, 0], pts[:, 1], gamma, -1, dk, dk)[0]
        assert np.abs(z_now - ref).max() / np.abs(ref).max() > 0.05
    # the mirrored sign of Delta is far off
    ref_bad = _corr_cosine(pts[:, 0] + c[0], pts[:, 1] + c[1], L, Wd)
    assert np.abs(z - ref_bad).max() / np.abs(ref).max() > 0.1


def test_reciprocity_on_symmetric_grid():
    """Z'_nm(-Delta; Q) = Z'_mn(Delta; conj Q) on a grid symmetric about k = 0.

    Follows from eq. MBF (Z' = Q^H Z Q), the evenness of G and the symmetry
    G_xy = G_yx.  An odd number of samples centred on 0 makes the rectangle
    rule symmetric, so the identity holds to rounding.
    """
    rng = _rng(5)
    n = 15
    km = 5 * K0
    k1 = (np.arange(n) - n // 2) * (2 * km / n)
    KX, KY = np.meshgrid(k1, k1)
    kx, ky = KX.ravel(), KY.ravel()
    gamma = 1 / 100
    basis = rooftop_lattice(2, 3)
    q = rng.standard_normal((2, basis.shape[0])) + 1j * rng.standard_normal((2, basis.shape[0]))
    kcx, kcy, w = co.ray_contour(kx, ky, gamma)
    g = co.green_remainder(kx, ky, gamma, K0, 4.4, 0.002, 0.06)
    dk = 2 * km / n
    pts = rng.uniform(-0.8, 0.8, (6, 2))

    def z(qq, m, nn, sgn):
        mt, mh = co.mbf_spectra(basis, qq, kcx, kcy)
        integ = co.integrand(mt[m], mh[nn], *g, w)[None]
        return co.direct_sum(integ, kx, ky, sgn * pts[:, 0], sgn * pts[:, 1], gamma, 3, dk, dk)[0]
    lhs = z(q, 1, 0, -1.0)
    rhs = z(np.conj(q), 0, 1, 1.0)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()
    # for real coefficients it reduces to Z_nm(-Delta) = Z_mn(Delta)
    qr = q.real.copy()
    assert np.abs(z(qr, 1, 0, -1.0) - z(qr, 0, 1, 1.0)).max() <= 1e-12 * np.abs(z(qr, 0, 1, 1.0)).max()


def test_sesquilinearity_q_h_z_q():
    """eq. MBF: Z'_mn = sum_ij conj(q_mi) q_nj Z_ij with Z_ij the elementary reactions."""
    rng = _rng(6)
    grid = Grid(16, 16, 6 * K0, 6 * K0, K0)
    sub = Substrate(4.4, 0.002, 0.06)
    basis = rooftop_lattice(2, 2)                       # B = 8
    b = basis.shape[0]
    q = rng.standard_normal((3, b)) + 1j * rng.standard_normal((3, b))
    pairs = np.array([(m, n) for m in range(3) for n in range(3)], dtype=np.int32)
    idx = rng.choice(256, 12, replace=False)
    zq = co.tabulate(grid, sub, basis, q, pairs, out_idx=idx)
    ze = co.tabulate(grid, sub, basis, np.eye(b, dtype=complex),
                     np.array([(i, j) for i in range(b) for j in range(b)]), out_idx=idx).reshape(b, b, -1)
    for p, (m, n) in enumerate(pairs):
        ref = np.einsum("i,j,ijq->q", np.conj(q[m]), q[n], ze)
        assert np.abs(zq[p] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_free_space_limit_zero_table():
    """eps_r = 1: the slab is air, the extracted remainder vanishes, so Z = 0."""
    grid = Grid(16, 16, 6 * K0, 6 * K0, K0)
    basis = rooftop_lattice(2, 2)
    q = np.ones((1, basis.shape[0]), dtype=complex)
    z = co.tabulate(grid, Substrate(1.0, 0.0, 0.05), basis, q, np.array([[0, 0]]))
    zs = co.tabulate(grid, Substrate(2.2, 0.0, 0.05), basis, q, np.array([[0, 0]]))
    assert np.abs(z).max() <= 1e-13 * np.abs(zs).max()


def test_bilinear_lookup_reproduces_nodes_and_planes():
    """Bilinear lookup is exact at table nodes and for functions affine in (dx, dy)."""
    grid = Grid(16, 12, 3 * K0, 2 * K0, K0)
    dxa = co.displacement_axis(16, grid.kx_max)
    dya = co.displacement_axis(12, grid.ky_max)
    DX, DY = np.meshgrid(dxa, dya)
    table = ((2 + 1j) * DX - (0.5 - 3j) * DY + 0.25)[None]
    rng = _rng(7)
    pts = np.stack([rng.uniform(dxa[0], dxa[-1] - 1e-9, 50), rng.uniform(dya[0], dya[-1] - 1e-9, 50)], axis=1)
    got = co.bilinear_lookup(grid, table, pts)[0]
    want = (2 + 1j) * pts[:, 0] - (0.5 - 3j) * pts[:, 1] + 0.25
    assert np.abs(got - want).max() < 1e-12
    nodes = np.stack([DX.ravel()[:30], DY.ravel()[:30]], axis=1)
    # nodes on the last row/column are outside the cell range; take interior ones
    inner = (nodes[:, 0] < dxa[-1]) & (nodes[:, 1] < dya[-1])
    got = co.bilinear_lookup(grid, table, nodes[inner])[0]
    assert np.abs(got - table[0].ravel()[:30][inner]).max() < 1e-12
    with pytest.raises(ValueError):
        co.bilinear_lookup(grid, table, np.array([[dxa[-1] + 0.01, 0.0]]))


def test_quadratic_lookup_is_exact_for_quadratics_and_at_nodes():
    """Second-order interpolation (Sec. III-B.3): exact on any table that is
    a product of quadratics in the two indices, equal to the node value at a
    node, and never reading outside the table at the edges."""
    grid = Grid(16, 8, 5 * K0, 3 * K0, K0)
    j1 = np.arange(16)
    j2 = np.arange(8)
    px = lambda u: 0.3 - 1.1j * u + (0.25 + 0.1j) * u * u
    py = lambda u: 1.0 + 0.4 * u - 0.05j * u * u
    table = (py(j2)[:, None] * px(j1)[None, :])[None]
    dxa = co.displacement_axis(16, grid.kx_max)
    dya = co.displacement_axis(8, grid.ky_max)
    rng = np.random.default_rng(8)
    ux = np.concatenate([rng.uniform(0, 15, 40), [0.0, 15.0, 0.2, 14.9]])
    uy = np.concatenate([rng.uniform(0, 7, 40), [0.0, 7.0, 6.95, 0.01]])
    pts = np.stack([dxa[0] + ux * (dxa[1] - dxa[0]), dya[0] + uy * (dya[1] - dya[0])], axis=1)
    got = co.quadratic_lookup(grid, table, pts)[0]
    assert np.abs(got - py(uy) * px(ux)).max() < 1e-12 * np.abs(got).max()
    node = np.array([[dxa[5], dya[3]]])
    assert abs(co.quadratic_lookup(grid, table, node)[0, 0] - table[0, 3, 5]) < 1e-14 * abs(table[0, 3, 5])
    with pytest.raises(ValueError):
        co.quadratic_lookup(grid, table, np.array([[dxa[-1] + 1e-9, 0.0]]))
