"""Pins of the oracle's tensor-product truncation mode (a <= P and b <= P).

On the ray contour E_I = exp(gamma kx Dx) exp(gamma ky Dy) exactly (Sec.
III-B.2, eq. taylors with a constant gamma); the tensor mode replaces each
factor by its own Taylor polynomial.  Not in the paper: these checks pin the
mode to its definition by routes that do not reuse the oracle's kernel.
"""
import math

import numpy as np

from oracle import cfft_oracle as co

K0 = 2 * math.pi


def _problem(seed, nx=8, ny=8, km=5 * K0):
    rng = np.random.default_rng(seed)
    integ = rng.standard_normal((2, nx * ny)) + 1j * rng.standard_normal((2, nx * ny))
    kx, ky = co.grid_samples(nx, ny, km, km)
    dk = 2 * km / nx
    dx = rng.uniform(-1.5, 1.5, 5)
    dy = rng.uniform(-1.5, 1.5, 5)
    return integ, kx, ky, dx, dy, dk


def test_order_zero_equals_total_degree():
    integ, kx, ky, dx, dy, dk = _problem(1)
    zt = co.direct_sum(integ, kx, ky, dx, dy, 1 / 130, 0, dk, dk, truncation=1)
    zd = co.direct_sum(integ, kx, ky, dx, dy, 1 / 130, 0, dk, dk, truncation=0)
    assert np.array_equal(zt, zd)


def test_high_order_equals_untruncated():
    integ, kx, ky, dx, dy, dk = _problem(2)
    gamma = 1 / 40
    zt = co.direct_sum(integ, kx, ky, dx, dy, gamma, 40, dk, dk, truncation=1)
    zi = co.direct_sum(integ, kx, ky, dx, dy, gamma, -1, dk, dk)
    assert np.abs(zt - zi).max() <= 1e-13 * np.abs(zi).max()


def test_difference_is_the_extra_terms():
    """Z_tensor - Z_total = sum over a, b <= P with a + b > P of the single-term
    sums K sum_n I e^{-ik.D} (g kx Dx)^a (g ky Dy)^b / (a! b!), enumerated
    explicitly per sample and output."""
    integ, kx, ky, dx, dy, dk = _problem(3)
    gamma, P = 1 / 20, 3
    zt = co.direct_sum(integ, kx, ky, dx, dy, gamma, P, dk, dk, truncation=1)
    zd = co.direct_sum(integ, kx, ky, dx, dy, gamma, P, dk, dk, truncation=0)
    K = dk * dk / (4 * math.pi ** 2)
    extra = np.zeros_like(zt)
    for q in range(dx.size):
        for n in range(kx.size):
            u = gamma * kx[n] * dx[q]
            v = gamma * ky[n] * dy[q]
            ph = complex(math.cos(kx[n] * dx[q] + ky[n] * dy[q]), -math.sin(kx[n] * dx[q] + ky[n] * dy[q]))
            s = 0.0
            for a in range(P + 1):
                for b in range(P + 1):
                    if a + b > P:
                        s += u ** a * v ** b / (math.factorial(a) * math.factorial(b))
            extra[:, q] += K * integ[:, n] * ph * s
    assert np.abs((zt - zd) - extra).max() <= 1e-13 * np.abs(zt).max()


def test_separable_integrand_factorises():
    """For I(kx, ky) = f(kx) g(ky) the tensor table is K times the product of
    two one-dimensional truncated sums (a property the total-degree form
    lacks); this also fixes which factor goes with which axis."""
    rng = np.random.default_rng(4)
    nx, ny = 16, 8
    kxm, kym = 6 * K0, 4 * K0
    f = rng.standard_normal(nx) + 1j * rng.standard_normal(nx)
    g = rng.standard_normal(ny) + 1j * rng.standard_normal(ny)
    integ = np.outer(g, f).ravel()[None, :]           # [ny][nx], x fastest
    kx, ky = co.grid_samples(nx, ny, kxm, kym)
    dkx, dky = 2 * kxm / nx, 2 * kym / ny
    kx1 = -kxm + dkx * np.arange(nx)
    ky1 = -kym + dky * np.arange(ny)
    gamma, P = 1 / 15, 2
    dx = np.array([-0.7, 0.1, 0.9])
    dy = np.array([0.4, -1.1, 0.05])
    zt = co.direct_sum(integ, kx, ky, dx, dy, gamma, P, dkx, dky, truncation=1)[0]
    zd = co.direct_sum(integ, kx, ky, dx, dy, gamma, P, dkx, dky, truncation=0)[0]
    K = dkx * dky / (4 * math.pi ** 2)
    for q in range(dx.size):
        sx = sum(f[i] * np.exp(-1j * kx1[i] * dx[q]) * sum((gamma * kx1[i] * dx[q]) ** a / math.factorial(a)
                                                            for a in range(P + 1)) for i in range(nx))
        sy = sum(g[i] * np.exp(-1j * ky1[i] * dy[q]) * sum((gamma * ky1[i] * dy[q]) ** b / math.factorial(b)
                                                            for b in range(P + 1)) for i in range(ny))
        ref = K * sx * sy
        assert abs(zt[q] - ref) <= 1e-13 * abs(ref)
        assert abs(zd[q] - ref) > 1e-8 * abs(ref)       # the total-degree form does not factorise


def test_remainder_bound_and_no_worse_than_total_degree_bound():
    """|Z_tensor - Z_inf| <= K sum |I| (e^{|u|+|v|} - T_P(|u|) T_P(|v|)) with
    u = gamma kx Dx, v = gamma ky Dy; the bound never exceeds the total-degree
    one, K sum |I| (e^{|u|+|v|} - T_P(|u|+|v|)), since the tensor form misses
    a subset of the total-degree form's (non-negative) terms."""
    integ, kx, ky, dx, dy, dk = _problem(5, km=6 * K0)
    gamma = 1 / 25
    K = dk * dk / (4 * math.pi ** 2)
    for P in range(4):
        zt = co.direct_sum(integ, kx, ky, dx, dy, gamma, P, dk, dk, truncation=1)
        zi = co.direct_sum(integ, kx, ky, dx, dy, gamma, -1, dk, dk)
        for q in range(dx.size):
            u = np.abs(gamma * kx * dx[q])
            v = np.abs(gamma * ky * dy[q])
            tp_u = sum(u ** a / math.factorial(a) for a in range(P + 1))
            tp_v = sum(v ** b / math.factorial(b) for b in range(P + 1))
            miss_tensor = np.exp(u + v) - tp_u * tp_v
            miss_total = np.exp(u + v) - sum((u + v) ** s / math.factorial(s) for s in range(P + 1))
            assert np.all(miss_tensor <= miss_total * (1 + 1e-12) + 1e-300)
            bound = K * np.abs(integ) @ miss_tensor
            assert np.all(np.abs(zt[:, q] - zi[:, q]) <= bound * (1 + 1e-12))
