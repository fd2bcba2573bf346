"""Seeded synthetic inputs for the contour-FFT tabulation.

This module only *describes* inputs: grid sizes, substrate parameters,
basis-function geometry, MBF coefficients and query displacements.  It holds
none of the method's arithmetic (no Green's function, no spectra, no
transforms), so both the CPU oracle and the GPU path can import it without
sharing any computation.

Units: lengths in free-space wavelengths at the reference frequency f0
(lambda0 = 1), so k0 = 2*pi*f/f0.  The paper works with a 24.125 GHz patch
whose mesh and MBF coefficients are not published; the workloads below stand
in for it with the sizes, contrasts and coefficient statistics of the
benchmark configurations (paper Sec. III-A geometry; Sec. IV-F sizing rule
k_max ~ 5 k_d).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

BASE_SEED = 14047357

# Basis-function kinds (shared vocabulary with include/cfft.h).
ROOFTOP_X = 0   # x-directed rooftop: triangle of half-base a along x, pulse of width b along y
ROOFTOP_Y = 1   # y-directed rooftop: transpose of ROOFTOP_X
COSINE_X = 2    # x-directed half-cosine cos(pi x/a) on |x|<=a/2, uniform on |y|<=b/2
COSINE_Y = 3    # y-directed transpose of COSINE_X

CONTOUR_RAY = 0
CONTOUR_PARABOLIC = 1
FP64 = 0
MIXED = 1
TRUNC_TOTAL = 0    # terms a + b <= P of the Taylor series of E_I (eq. fftarry)
TRUNC_TENSOR = 1   # terms a <= P and b <= P (product of per-axis polynomials)

BASIS_DTYPE = np.dtype([("kind", np.int32), ("pad", np.int32), ("cx", np.float64),
                        ("cy", np.float64), ("a", np.float64), ("b", np.float64)])


def basis_array(records) -> np.ndarray:
    """Pack (kind, cx, cy, a, b) tuples into the C-ABI record layout."""
    out = np.zeros(len(records), dtype=BASIS_DTYPE)
    for i, (kind, cx, cy, a, b) in enumerate(records):
        out[i] = (kind, 0, cx, cy, a, b)
    return out


def rooftop_lattice(n_along: int, n_across: int, size: float = 0.5) -> np.ndarray:
    """Rooftop mesh of a size x size patch centred on the origin.

    Per orientation there are n_along rooftops along the current direction
    (shared edges of n_along+1 cells, half-base a = size/(n_along+1)) times
    n_across strips of width b = size/n_across.  The y-directed set is the
    transpose of the x-directed one.  Total B = 2*n_along*n_across.
    """
    a = size / (n_along + 1)
    b = size / n_across
    half = size / 2
    recs = []
    for p in range(n_along):
        for r in range(n_across):
            recs.append((ROOFTOP_X, -half + (p + 1) * a, -half + (r + 0.5) * b, a, b))
    for p in range(n_along):
        for r in range(n_across):
            recs.append((ROOFTOP_Y, -half + (r + 0.5) * b, -half + (p + 1) * a, a, b))
    return basis_array(recs)


def gaussian_coefficients(rng: np.random.Generator, m: int, b: int) -> np.ndarray:
    """MBF coefficients q ~ N(0,1) + i N(0,1), shape [M][B], complex128."""
    re = rng.standard_normal((m, b))
    im = rng.standard_normal((m, b))
    return (re + 1j * im).astype(np.complex128)


def query_displacements(rng: np.random.Generator, count: int, half_span: float,
                        min_radius: float = 0.5) -> np.ndarray:
    """Query displacements uniform in |dx|,|dy| < half_span with |d| >= min_radius.

    Rejection sampling; returns float64 [count][2] (dx, dy).
    """
    out = np.empty((0, 2))
    while out.shape[0] < count:
        cand = rng.uniform(-half_span, half_span, size=(2 * count, 2))
        keep = np.hypot(cand[:, 0], cand[:, 1]) >= min_radius
        out = np.concatenate([out, cand[keep]], axis=0)
    return np.ascontiguousarray(out[:count])


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    kx_max: float
    ky_max: float
    k0: float
    gamma: float = 1.0 / 130.0
    order: int = 3
    contour: int = CONTOUR_RAY
    beta_end: float = 0.0
    precision: int = FP64
    truncation: int = TRUNC_TOTAL
    zero_pad: int = 0                  # 1: x2 zero-padded grid (integrand on the central half only)


@dataclasses.dataclass
class Substrate:
    eps_r: float
    tan_delta: float
    h: float


@dataclasses.dataclass
class Workload:
    name: str
    description: str
    grids: List[Grid]
    substrates: List[Substrate]          # one per grid (frequency sweep changes only k0)
    basis: np.ndarray                    # BASIS_DTYPE records
    q: np.ndarray                        # complex128 [M][B]
    pairs: np.ndarray                    # int32 [npairs][2] (m, n)
    queries: Optional[np.ndarray] = None  # float64 [Q][2]
    target_eps_r: Optional[float] = None
    target_q: Optional[np.ndarray] = None
    layout: Optional[np.ndarray] = None   # float64 [A][2] element positions of an array

    @property
    def M(self) -> int:
        return self.q.shape[0]

    @property
    def B(self) -> int:
        return self.q.shape[1]

    def entries(self) -> int:
        return sum(g.nx * g.ny for g in self.grids) * len(self.pairs)


def all_pairs(m: int) -> np.ndarray:
    return np.array([(i, j) for i in range(m) for j in range(m)], dtype=np.int32)


def k0_of(f_over_f0: float) -> float:
    return 2.0 * math.pi * f_over_f0


def c1_single_cosine(precision: int = FP64) -> Workload:
    """One x-directed half-cosine MBF (0.3 x 0.02), eps_r 2.2, h 0.05, 64^2 over +-8 k0."""
    k0 = k0_of(1.0)
    basis = basis_array([(COSINE_X, 0.0, 0.0, 0.3, 0.02)])
    q = np.ones((1, 1), dtype=np.complex128)
    g = Grid(64, 64, 8 * k0, 8 * k0, k0, precision=precision)
    return Workload("c1_cosine_patch_64", "1 MBF, half-cosine patch, 64^2 grid", [g],
                    [Substrate(2.2, 0.0, 0.05)], basis, q, all_pairs(1))


def c2_rooftop_512(precision: int = FP64, n: int = 512) -> Workload:
    """M=4 MBFs of B=256 rooftops on 0.5 x 0.5, eps_r 4.4 tan 0.002 h 0.06, 512^2, 16 pairs."""
    rng = np.random.default_rng(BASE_SEED + 1)
    k0 = k0_of(1.0)
    eps = 4.4
    km = 5.0 * math.sqrt(eps) * k0
    basis = rooftop_lattice(8, 16)
    q = gaussian_coefficients(rng, 4, basis.shape[0])
    g = Grid(n, n, km, km, k0, precision=precision)
    return Workload(f"c2_rooftop_m4_b256_{n}", "4 MBFs x 256 rooftops, FR4-like slab", [g],
                    [Substrate(eps, 0.002, 0.06)], basis, q, all_pairs(4))


def c3_frequency_sweep(precision: int = MIXED) -> Workload:
    """16 pairs x 8 frequencies 0.9..1.1 f0, eps_r 3.0, h 0.08 (at f0), grids 256/512/1024."""
    rng = np.random.default_rng(BASE_SEED + 2)
    eps = 3.0
    basis = rooftop_lattice(8, 16)
    q = gaussian_coefficients(rng, 4, basis.shape[0])
    grids, subs = [], []
    sizes = [256, 512, 1024]
    for i in range(8):
        f = 0.9 + 0.2 * i / 7.0
        k0 = k0_of(f)
        km = 5.0 * math.sqrt(eps) * k0
        n = sizes[i % 3]
        grids.append(Grid(n, n, km, km, k0, precision=precision))
        subs.append(Substrate(eps, 0.0, 0.08))
    return Workload("c3_sweep_8freq_uneven", "16 pairs x 8 frequencies, uneven grids",
                    grids, subs, basis, q, all_pairs(4))


def c4_large(precision: int = MIXED, n: int = 4096) -> Workload:
    """M=6 MBFs of B=1024 rooftops, eps_r 10.2 h 0.12, 4096^2 over 200 x 200, 1e5 lookups."""
    rng = np.random.default_rng(BASE_SEED + 3)
    k0 = k0_of(1.0)
    span = 200.0 * n / 4096.0
    km = math.pi * n / span           # d_delta = pi/k_max = span/n
    basis = rooftop_lattice(16, 32)
    q = gaussian_coefficients(rng, 6, basis.shape[0])
    half = 0.5 * span - 0.1 * span / 200.0
    queries = query_displacements(rng, 100000, half, 0.5)
    g = Grid(n, n, km, km, k0, precision=precision)
    return Workload(f"c4_rooftop_m6_b1024_{n}", "6 MBFs x 1024 rooftops, high-contrast slab",
                    [g], [Substrate(10.2, 0.0, 0.12)], basis, q, all_pairs(6), queries)


def c5_gradient(n: int = 1024, nq: int = 4096) -> Workload:
    """M=4, B=256, eps_r 2.2 h 0.05, 1024^2 over +-8 k0, 4096 lookups, target at eps 2.3."""
    rng = np.random.default_rng(BASE_SEED + 4)
    k0 = k0_of(1.0)
    km = 8.0 * k0
    basis = rooftop_lattice(8, 16)
    q = gaussian_coefficients(rng, 4, basis.shape[0])
    span = n * math.pi / km
    queries = query_displacements(rng, nq, 0.5 * span - 0.1, 0.5)
    target_q = q + 0.1 * gaussian_coefficients(rng, 4, basis.shape[0])
    g = Grid(n, n, km, km, k0, precision=FP64)
    return Workload(f"c5_gradient_{n}", "loss over 4096 lookups, gradient wrt eps_r, h, q",
                    [g], [Substrate(2.2, 0.0, 0.05)], basis, q, all_pairs(4), queries,
                    target_eps_r=2.3, target_q=target_q)


def regular_layout(nx: int, ny: int, spacing: float) -> np.ndarray:
    """Element positions of an nx x ny regular array centred on the origin."""
    ix, iy = np.meshgrid(np.arange(nx) - 0.5 * (nx - 1), np.arange(ny) - 0.5 * (ny - 1))
    return (spacing * np.stack([ix.ravel(), iy.ravel()], 1)).astype(np.float64)


def paper_array_2048(n: int = 2048, elements: int = 25) -> Workload:
    """The paper's table setup with synthetic MBFs: a 2048^2 FFT including the
    x2 zero padding (1024^2 samples over +-5 k_d, eps_r 2.2, h 0.381 mm at
    24.125 GHz = 0.0307 lambda0), M = 9 MBFs (81 pairs) of B = 256 rooftops,
    FP64; the layout is the 25 x 25 regular array at 0.58 lambda0."""
    rng = np.random.default_rng(BASE_SEED + 5)
    k0 = k0_of(1.0)
    eps = 2.2
    km = 5.0 * math.sqrt(eps) * k0                # spectral half-span of the original samples
    basis = rooftop_lattice(8, 16)
    q = gaussian_coefficients(rng, 9, basis.shape[0])
    g = Grid(n, n, 2.0 * km, 2.0 * km, k0, precision=FP64, zero_pad=1)
    return Workload(f"paper_array_m9_{n}_zero_padded", "81 pairs on a x2 zero-padded grid, 25 x 25 array fill",
                    [g], [Substrate(eps, 0.0, 0.381 / (299.792458 / 24.125))], basis, q, all_pairs(9),
                    layout=regular_layout(elements, elements, 0.58))


def random_smooth_field(rng: np.random.Generator, shape, scale: float = 1.0) -> np.ndarray:
    """Seeded complex128 noise for kernel-level tests (no physical meaning)."""
    return (scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex128)
