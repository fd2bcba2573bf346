"""Plain FP64 oracle of the C-FFT tabulation (test infrastructure only).

Every function states the passage of the paper it follows and what pins it.
Conventions (the paper leaves them implicit; the readings are listed in the
design notes):
  * time dependence exp(+i w t); lossy permittivity eps' (1 - i tan_delta)
  * spatial Fourier transform F(k) = int f(r) exp(-i k.r) dr
  * displacement Delta = r_test - r_basis
  * free-space impedance eta0 = 1, lengths in lambda0, k0 = 2 pi f/f0
  * ray contour: k_c = (1 + i gamma) k for every real sample k; parabolic
    contour: k_c = (1 + i g(beta)) k with g(beta) = gamma (1 - beta/beta_end)
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOFTOP_X, ROOFTOP_Y, COSINE_X, COSINE_Y = 0, 1, 2, 3


# --------------------------------------------------------------------------
# Grids (Appendix: change of variables used for the FFT)
# --------------------------------------------------------------------------
def spectral_axis(n: int, k_max: float) -> np.ndarray:
    """Real spectral samples k(i) = -k_max + i * (pi / x_max), i = 0..n-1.

    Appendix: with x_max = n pi / (2 k_max) the spectral step pi/x_max equals
    2 k_max / n, so the samples cover [-k_max, k_max) (rectangle rule of
    eq. fftexp).  Pinned by the P=0 FFT special case (test_oracle_core).
    """
    x_max = n * math.pi / (2.0 * k_max)
    return -k_max + np.arange(n, dtype=np.float64) * (math.pi / x_max)


def displacement_axis(n: int, k_max: float) -> np.ndarray:
    """Output displacements Delta(j) = -x_max + j * pi / k_max (Appendix)."""
    x_max = n * math.pi / (2.0 * k_max)
    return -x_max + np.arange(n, dtype=np.float64) * (math.pi / k_max)


# --------------------------------------------------------------------------
# Contour (Sec. III-B.2, eqs. complexbeta .. ratioNew and eq. FFT)
# --------------------------------------------------------------------------
def ray_contour(kx: np.ndarray, ky: np.ndarray, gamma: float):
    """Analytic extension of the real sample (kx, ky) onto the deformed contour.

    eq. ratioNew sets k_xI/k_xR = k_yI/k_yR = beta_I/beta_R = gamma, i.e.
    k_c = (1 + i gamma) k.  The weight that multiplies the MBF kernel in
    eq. FFT is (1 + i d beta_I/d beta_R)(1 + i gamma); on a ray beta_I =
    gamma beta_R so d beta_I/d beta_R = gamma and W = (1 + i gamma)^2, which is
    also det(d k_c / d k) (pinned by a finite-difference Jacobian test).
    Returns (kcx, kcy, W).
    """
    s = 1.0 + 1j * gamma
    return s * kx, s * ky, s * s


def parabolic_contour(kx: np.ndarray, ky: np.ndarray, gamma: float, beta_end: float):
    """Parabolic deformation of the radial path (Sec. I and the caption of
    Fig. 1: a parabolic contour whose height is set by gamma; Sec. II, eq.
    spectral_contour: the path is beta_c = beta_R + i beta_I(beta_R)).

    Reading: beta_I = gamma beta (1 - beta/beta_end) for beta < beta_end and
    0 beyond (the path rejoins the real axis at beta_end, past every
    surface-wave pole).  Each real sample k then moves to k_c = (1 + i g) k
    with the local ratio g = beta_I/beta = gamma (1 - beta/beta_end) (eq.
    ratioNew holds sample by sample), and the weight of eq. FFT is
    W = (1 + i d beta_I/d beta)(1 + i g), which equals det(d k_c / d k).
    The slope d beta_I/d beta jumps from -gamma to 0 at beta_end; a sample
    lying there (within a relative 1e-9, so that rounding of beta cannot
    decide) takes the mean of the two one-sided slopes, -gamma/2.  g itself
    is continuous (0 at beta_end).
    Returns (kcx, kcy, W, g) with g per sample.
    """
    kx = np.asarray(kx, dtype=np.float64)
    ky = np.asarray(ky, dtype=np.float64)
    beta = np.hypot(kx, ky)
    inside = beta < beta_end
    at_end = np.abs(beta - beta_end) <= 1e-9 * beta_end
    g = np.where(inside, gamma * (1.0 - beta / beta_end), 0.0)
    dbi = np.where(at_end, -0.5 * gamma, np.where(inside, gamma * (1.0 - 2.0 * beta / beta_end), 0.0))
    s = 1.0 + 1j * g
    return s * kx, s * ky, (1.0 + 1j * dbi) * s, g


def grid_contour(kx, ky, grid):
    """(kcx, kcy, W, g) of a grid's contour; g is gamma (ray) or per sample."""
    if getattr(grid, "contour", 0) == 1:
        return parabolic_contour(kx, ky, grid.gamma, grid.beta_end)
    kcx, kcy, w = ray_contour(kx, ky, grid.gamma)
    return kcx, kcy, w, grid.gamma


def sqrt_radiating(z):
    """Square root whose branch cut lies on the positive imaginary axis.

    Radiation condition for exp(+i w t): a vertical wavenumber k_z must make
    exp(-i k_z z) decay or propagate upward, i.e. Im k_z <= 0 with k_z > 0 for
    a propagating wave.  For every passive medium and every point of the
    deformed contour the argument lies in the closed lower half plane, where
    this root has exactly that property; putting the cut on the positive
    imaginary axis (rather than the negative real axis) keeps the root
    analytic in the substrate parameters, which the Cauchy-rule gradient
    needs.  Pinned by the large-beta decay, passivity and contour-independence
    tests.
    """
    z = np.asarray(z, dtype=np.complex128)
    return np.exp(-0.25j * math.pi) * np.sqrt(1j * z)


# --------------------------------------------------------------------------
# Grounded-slab Green's function minus homogeneous medium + image
# (Sec. II and Sec. III-A: layered-medium dyadic from which an effective
# homogeneous medium and its image through the ground are extracted)
# --------------------------------------------------------------------------
def slab_immittances(beta_c, k0, eps_r, h):
    """Input impedances Z_TE, Z_TM seen by a current sheet on a grounded slab.

    Transmission-line model of the stratified medium: the sheet sits at the
    air/dielectric interface, looking up into matched air and down into a slab
    line of length h shorted by the ground plane.  The two admittances add.
    Characteristic admittances (eta0 = 1):
        TE: Y = k_z / k0          TM: Y = k0 eps / k_z
    Shorted line of length h seen from its open end: Y_in = -i Y cot(k_z h),
    written with exp(-2 i k_z h) so that large |Im k_z h| cannot overflow.
    Pinned by: eps_r = 1 equality with the homogeneous part, textbook
    surface-wave dispersion roots, and a numerical ODE integration of the
    transmission-line equations through the slab (test_oracle_green).
    """
    beta2 = np.asarray(beta_c, dtype=np.complex128) ** 2
    kz0 = sqrt_radiating(k0 * k0 - beta2)
    # kz1 appears only in even functions; the Im <= 0 root keeps
    # e = exp(-2 i kz1 h) bounded so that nothing overflows at large beta.
    kz1 = sqrt_radiating(eps_r * k0 * k0 - beta2)
    e = np.exp(-2j * kz1 * h)
    one_minus_e = -np.expm1(-2j * kz1 * h)
    # -i cot(kz1 h) = (1 + e) / (1 - e)
    m_icot = (1.0 + e) / one_minus_e
    y_te = kz0 / k0 + (kz1 / k0) * m_icot
    y_tm = k0 / kz0 + (k0 * eps_r / kz1) * m_icot
    return 1.0 / y_te, 1.0 / y_tm


def homogeneous_image_immittances(beta_c, k0, eps_r, h):
    """Effective homogeneous medium eps_e = (eps_r + 1)/2 plus its ground image.

    A sheet in an unbounded medium sees Z_c/2 (half each way); the image
    current through the ground plane at distance 2h is reversed and adds
    -Z_c/2 exp(-2 i k_e h).  TE: Z_c = k0/k_e; TM: Z_c = k_e/(k0 eps_e).
    The paper names this extraction but gives no formula; this is the reading
    that makes the remainder vanish for eps_r = 1 and decay at large beta.
    """
    eps_e = 0.5 * (eps_r + 1.0)
    beta2 = np.asarray(beta_c, dtype=np.complex128) ** 2
    ke = sqrt_radiating(eps_e * k0 * k0 - beta2)
    img = 1.0 - np.exp(-2j * ke * h)
    return 0.5 * k0 / ke * img, 0.5 * ke / (k0 * eps_e) * img


def green_remainder(kx, ky, gamma, k0, eps_r, tan_delta, h):
    """Dyadic G_s = G_slab - G_homogeneous+image at k_c = (1 + i gamma) k.

    Spectral dyadic of a horizontal current sheet: TM immittance along the
    in-plane propagation direction (c, s) = (kx, ky)/|k|, TE across it, with
    the minus sign of E = -Z J:
        Gxx = -(c^2 dZ_TM + s^2 dZ_TE)
        Gyy = -(s^2 dZ_TM + c^2 dZ_TE)
        Gxy = Gyx = -c s (dZ_TM - dZ_TE)
    At k = 0 the angular factors are 0/0; the limit is -dZ_TE(0) * identity
    (dZ_TM(0) = dZ_TE(0)).  Returns (Gxx, Gxy, Gyy), complex128, same shape as kx.
    """
    kx = np.asarray(kx, dtype=np.float64)
    ky = np.asarray(ky, dtype=np.float64)
    beta = np.hypot(kx, ky)
    zero = beta == 0
    safe = np.where(zero, 1.0, beta)
    c = np.where(zero, 1.0, kx / safe)
    s = np.where(zero, 0.0, ky / safe)
    g = green_polar((1.0 + 1j * gamma) * beta, c, s, k0, eps_r, tan_delta, h)
    # limit at k = 0: dZ_TM(0) = dZ_TE(0), so the dyadic is isotropic
    gxx, gxy, gyy = g
    iso = green_polar(np.zeros(1, dtype=np.complex128), 1.0, 0.0, k0, eps_r, tan_delta, h)[0][0]
    return (np.where(zero, iso, gxx), np.where(zero, 0.0, gxy), np.where(zero, iso, gyy))


def green_polar(beta_c, c, s, k0, eps_r, tan_delta, h):
    """Dyadic remainder at k_c = beta_c (c, s) for complex beta_c and real direction (c, s)."""
    eps = eps_r * (1.0 - 1j * tan_delta)
    zte, ztm = slab_immittances(beta_c, k0, eps, h)
    hte, htm = homogeneous_image_immittances(beta_c, k0, eps, h)
    dte = zte - hte
    dtm = ztm - htm
    gxx = -(c * c * dtm + s * s * dte)
    gyy = -(s * s * dtm + c * c * dte)
    gxy = -(c * s) * (dtm - dte)
    return gxx, gxy, gyy


# --------------------------------------------------------------------------
# Basis-function and MBF spectra (Sec. III-A, eq. FTMBF)
# --------------------------------------------------------------------------
def sinc(z):
    """sin(z)/z for complex z, with the removable point handled by its series."""
    z = np.asarray(z, dtype=np.complex128)
    small = np.abs(z) < 1e-4
    zs = np.where(small, 1.0, z)
    z2 = z * z
    return np.where(small, 1.0 - z2 / 6.0 + z2 * z2 / 120.0, np.sin(zs) / zs)


def basis_ft(kind, cx, cy, a, b, kcx, kcy):
    """Closed-form Fourier transform of one basis function at complex (kcx, kcy).

    Rooftop (paper Sec. III-A: analytic transforms of rooftops), unit peak:
      x-directed  f = tri((x-cx)/a) rect((y-cy)/b):
         F = a sinc^2(kx a/2) * b sinc(ky b/2) * exp(-i(kx cx + ky cy))
    Half-cosine x-directed  f = cos(pi (x-cx)/a) on |x-cx|<=a/2, |y-cy|<=b/2:
         F = (a/2)[sinc((kx a - pi)/2) + sinc((kx a + pi)/2)] * b sinc(ky b/2) * phase
    y-directed kinds are the transposes.  Returns the scalar component along
    the basis direction.  Pinned by Gauss-Legendre quadrature of the spatial
    integral at complex k (test_oracle_spectra).
    """
    phase = np.exp(-1j * (kcx * cx + kcy * cy))
    if kind in (ROOFTOP_Y, COSINE_Y):
        along, across = kcy, kcx
    else:
        along, across = kcx, kcy
    if kind in (ROOFTOP_X, ROOFTOP_Y):
        f_along = a * sinc(along * a / 2) ** 2
    else:
        f_along = 0.5 * a * (sinc((along * a - math.pi) / 2) + sinc((along * a + math.pi) / 2))
    f_across = b * sinc(across * b / 2)
    return f_along * f_across * phase


def mbf_spectra(basis, q, kcx, kcy):
    """Testing and reflected basis spectra of every MBF at k_c.

    eq. FTMBF: M_m(k) = sum_j conj(q_mj) F_j(k) (testing side).  The basis side
    enters eq. MBF_mul22 conjugated; on the complex contour the conjugate is
    read as the analytic reflection M#_n(k_c) = conj(M_n(conj k_c))
    = sum_j q_nj F_j(-k_c), which equals the plain conjugate on the real axis.
    Returns (mt, mh) each complex128 [M][2][...] with component 0 = x, 1 = y.
    Pinned by sesquilinearity Z' = Q^H Z Q (eq. MBF) and reciprocity tests.
    """
    q = np.asarray(q, dtype=np.complex128)
    m_count = q.shape[0]
    shape = np.shape(kcx)
    mt = np.zeros((m_count, 2) + shape, dtype=np.complex128)
    mh = np.zeros((m_count, 2) + shape, dtype=np.complex128)
    for j, rec in enumerate(basis):
        kind, cx, cy, a, b = int(rec["kind"]), float(rec["cx"]), float(rec["cy"]), float(rec["a"]), float(rec["b"])
        comp = 1 if kind in (ROOFTOP_Y, COSINE_Y) else 0
        fp = basis_ft(kind, cx, cy, a, b, kcx, kcy)
        fm = basis_ft(kind, cx, cy, a, b, -kcx, -kcy)
        for m in range(m_count):
            mt[m, comp] += np.conj(q[m, j]) * fp
            mh[m, comp] += q[m, j] * fm
    return mt, mh


# --------------------------------------------------------------------------
# Integrand (eqs. MBF_mul, MBF_mul22 and eq. FFT)
# --------------------------------------------------------------------------
def integrand(mt_m, mh_n, gxx, gxy, gyy, weight):
    """I_mn(k) = W * sum_{a,b in {x,y}} M_m^a(k_c) G_ab(k_c) M#_n^b(k_c).

    eq. MBF_mul22 (dyadic sandwich) times the contour weight of eq. FFT.
    mt_m, mh_n are [2][...] (x, y components).
    """
    s = (mt_m[0] * (gxx * mh_n[0] + gxy * mh_n[1])
         + mt_m[1] * (gxy * mh_n[0] + gyy * mh_n[1]))
    return weight * s


def taylor_poly(z, order):
    """T_P(z) = sum_{p=0}^{P} z^p / p!  (eq. taylors truncated at order P)."""
    out = np.zeros_like(z, dtype=np.complex128)
    term = np.ones_like(z, dtype=np.complex128)
    for p in range(order + 1):
        if p > 0:
            term = term * z / p
        out = out + term
    return out


# --------------------------------------------------------------------------
# The table: direct sum per output displacement (eqs. FFT, taylors, fftexp)
# --------------------------------------------------------------------------
def direct_sum(integrands, kx, ky, dx, dy, gamma, order, dkx, dky, block=32, workers=1, truncation=0):
    """Z^(P)_p(Delta_q) for every integrand p and output displacement q.

    Rectangle-rule discretisation of eq. FFT with E_I replaced by its Taylor
    polynomial of order P (eqs. taylors, fftexp):
        Z(Delta) = dkx dky / (4 pi^2) * sum_n I(k_n) exp(-i k_n.Delta)
                                          * T_P(gamma k_n.Delta)
    order < 0 means the untruncated exponential (E_I itself).  gamma is one
    value (ray contour) or one value per sample (parabolic contour, where the
    ratio beta_I/beta_R varies along the path).  truncation = 1
    selects the tensor-product variant (not in the paper): on the ray contour
    E_I = exp(gamma kx Dx) exp(gamma ky Dy) exactly, and each factor is
    replaced by its own Taylor polynomial, T_P(gamma kx Dx) T_P(gamma ky Dy).
    The sum over samples is a matrix product with the [samples x outputs]
    kernel matrix, built one block of outputs at a time.

    integrands: [npairs][ns] complex; kx, ky: [ns] real sample coordinates;
    dx, dy: [nq] output displacements.  Returns [npairs][nq] complex128.
    """
    integrands = np.asarray(integrands, dtype=np.complex128)
    kx = np.asarray(kx, dtype=np.float64).ravel()
    ky = np.asarray(ky, dtype=np.float64).ravel()
    dx = np.asarray(dx, dtype=np.float64).ravel()
    dy = np.asarray(dy, dtype=np.float64).ravel()
    nq = dx.size
    gam = np.asarray(gamma, dtype=np.float64)
    gam = gam.ravel() if gam.ndim else gam       # per-sample contour ratio (parabolic) or one value (ray)
    scale = dkx * dky / (4.0 * math.pi ** 2)
    out = np.zeros((integrands.shape[0], nq), dtype=np.complex128)

    ns = kx.size
    # the sum over samples is accumulated in slices of at most ~4M terms per
    # output block so that huge grids fit in host memory
    sstep = max(1, min(ns, (1 << 22) // max(1, block)))

    def one_block(q0):
        q1 = min(nq, q0 + block)
        acc = np.zeros((integrands.shape[0], q1 - q0), dtype=np.complex128)
        for s0 in range(0, ns, sstep):
            s1 = min(ns, s0 + sstep)
            argx = np.outer(kx[s0:s1], dx[q0:q1])
            argy = np.outer(ky[s0:s1], dy[q0:q1])
            arg = argx + argy                                                       # k.Delta
            g = gam[s0:s1, None] if gam.ndim else gam
            kern = np.exp(-1j * arg)
            if order < 0:
                kern *= np.exp(g * arg)
            elif truncation == 1:
                kern *= taylor_poly(g * argx, order) * taylor_poly(g * argy, order)
            else:
                kern *= taylor_poly(g * arg, order)
            acc += integrands[:, s0:s1] @ kern
        out[:, q0:q1] = scale * acc

    starts = list(range(0, nq, block))
    if workers > 1:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one_block, starts))
    else:
        for q0 in starts:
            one_block(q0)
    return out


def grid_samples(nx, ny, kx_max, ky_max):
    """Flattened sample coordinates (row-major, x fastest) of the spectral grid."""
    kx1 = spectral_axis(nx, kx_max)
    ky1 = spectral_axis(ny, ky_max)
    KX, KY = np.meshgrid(kx1, ky1)        # [ny][nx]
    return KX.ravel(), KY.ravel()


def sampled_factors(grid, substrate, basis, q, workers=1):
    """G_s and the MBF spectra on every sample of one grid (flattened, x fastest).

    workers > 1 evaluates contiguous slices of the samples in parallel threads
    (the same per-sample arithmetic; the slices are concatenated in order).
    """
    kx, ky = grid_samples(grid.nx, grid.ny, grid.kx_max, grid.ky_max)
    kcx, kcy, w, gam = grid_contour(kx, ky, grid)

    def part(sl):
        g_ = green_remainder(kx[sl], ky[sl], gam[sl] if np.ndim(gam) else gam, grid.k0, substrate.eps_r,
                             substrate.tan_delta, substrate.h)
        return g_, mbf_spectra(basis, q, kcx[sl], kcy[sl])

    n = kx.size
    if workers <= 1 or n < 4096:
        g, (mt, mh) = part(slice(0, n))
        return kx, ky, w, g, mt, mh
    step = -(-n // workers)
    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(part, [slice(i, min(n, i + step)) for i in range(0, n, step)]))
    g = tuple(np.concatenate([p_[0][c] for p_ in parts]) for c in range(3))
    mt = np.concatenate([p_[1][0] for p_ in parts], axis=-1)
    mh = np.concatenate([p_[1][1] for p_ in parts], axis=-1)
    return kx, ky, w, g, mt, mh


def pair_integrands(pairs, w, g, mt, mh):
    """Integrands [npairs][ns] for the listed (m, n) pairs."""
    gxx, gxy, gyy = g
    return np.stack([integrand(mt[m], mh[n], gxx, gxy, gyy, w) for m, n in pairs])


def band_mask(grid):
    """Samples that carry the integrand on a x2 zero-padded grid.

    Sec. III-B.3, last paragraph: the tables are refined by Whittaker-Shannon
    interpolation with zero padding to twice the FFT size.  Reading: a grid
    with zero_pad set is the padded grid itself (2N samples over twice the
    spectral span, same spacing); the original samples are its central half
    on each axis, n in [N'/4, 3N'/4), and every other sample is zero.  The
    table then has half the displacement step over the same span.  Returns a
    flat boolean array (x fastest) or None when the grid is not padded.
    """
    if not getattr(grid, "zero_pad", 0):
        return None
    n1 = np.arange(grid.nx)
    n2 = np.arange(grid.ny)
    in1 = (n1 >= grid.nx // 4) & (n1 < 3 * grid.nx // 4)
    in2 = (n2 >= grid.ny // 4) & (n2 < 3 * grid.ny // 4)
    return (in2[:, None] & in1[None, :]).ravel()


def tabulate(grid, substrate, basis, q, pairs, out_idx=None, order=None, workers=1, block=32):
    """Table Z'_mn on the displacement grid (or on a subset of it).

    out_idx: None for the full [npairs][ny][nx] table, else an int array of
    flattened output indices j2*nx + j1 (returns [npairs][len(out_idx)]).
    block: outputs per task of the direct sum (workers share the tasks).
    """
    order = grid.order if order is None else order
    kx, ky, w, g, mt, mh = sampled_factors(grid, substrate, basis, q, workers=workers)
    integ = pair_integrands(pairs, w, g, mt, mh)
    mask = band_mask(grid)
    if mask is not None:
        integ = integ * mask
    dxa = displacement_axis(grid.nx, grid.kx_max)
    dya = displacement_axis(grid.ny, grid.ky_max)
    DX, DY = np.meshgrid(dxa, dya)
    dx, dy = DX.ravel(), DY.ravel()
    if out_idx is not None:
        dx, dy = dx[out_idx], dy[out_idx]
    dkx = 2.0 * grid.kx_max / grid.nx
    dky = 2.0 * grid.ky_max / grid.ny
    gam = grid_contour(kx, ky, grid)[3]
    z = direct_sum(integ, kx, ky, dx, dy, gam, order, dkx, dky, block=block, workers=workers,
                   truncation=getattr(grid, "truncation", 0))
    if out_idx is None:
        z = z.reshape(len(pairs), grid.ny, grid.nx)
    return z


def tabulate_from_factors(grid, pairs, g, mt, mh, out_idx=None, order=None, workers=1, block=32):
    """Same as tabulate() but from given sampled factors (kernel-level tests).

    g: (gxx, gxy, gyy) each [ny*nx]; mt, mh: [M][2][ny*nx].  The contour
    weight W = (1 + i gamma)^2 is applied here as in eq. FFT.
    """
    order = grid.order if order is None else order
    kx, ky = grid_samples(grid.nx, grid.ny, grid.kx_max, grid.ky_max)
    _, _, w, gam = grid_contour(kx, ky, grid)
    integ = pair_integrands(pairs, w, g, mt, mh)
    mask = band_mask(grid)
    if mask is not None:
        integ = integ * mask
    dxa = displacement_axis(grid.nx, grid.kx_max)
    dya = displacement_axis(grid.ny, grid.ky_max)
    DX, DY = np.meshgrid(dxa, dya)
    dx, dy = DX.ravel(), DY.ravel()
    if out_idx is not None:
        dx, dy = dx[out_idx], dy[out_idx]
    dkx = 2.0 * grid.kx_max / grid.nx
    dky = 2.0 * grid.ky_max / grid.ny
    z = direct_sum(integ, kx, ky, dx, dy, gam, order, dkx, dky, block=block, workers=workers,
                   truncation=getattr(grid, "truncation", 0))
    if out_idx is None:
        z = z.reshape(len(pairs), grid.ny, grid.nx)
    return z


# --------------------------------------------------------------------------
# Table use: bilinear lookup (Sec. III-B.3 last paragraph; the paper refines
# by zero padding and interpolates at second order, here first order)
# --------------------------------------------------------------------------
def bilinear_corners(grid, pts):
    """Corner indices and weights of bilinear interpolation in the table.

    Returns (j1, j2, tx, ty) with Z(pt) = sum over the four corners
    (1-tx)(1-ty) Z[j2][j1] + tx(1-ty) Z[j2][j1+1] + (1-tx)ty Z[j2+1][j1]
    + tx ty Z[j2+1][j1+1].  Points must lie inside the table's cell range.
    """
    pts = np.asarray(pts, dtype=np.float64)
    x_max = grid.nx * math.pi / (2.0 * grid.kx_max)
    y_max = grid.ny * math.pi / (2.0 * grid.ky_max)
    ux = (pts[:, 0] + x_max) / (math.pi / grid.kx_max)
    uy = (pts[:, 1] + y_max) / (math.pi / grid.ky_max)
    j1 = np.floor(ux).astype(np.int64)
    j2 = np.floor(uy).astype(np.int64)
    if np.any(j1 < 0) or np.any(j1 > grid.nx - 2) or np.any(j2 < 0) or np.any(j2 > grid.ny - 2):
        raise ValueError("query outside the table")
    return j1, j2, ux - j1, uy - j2


def bilinear_lookup(grid, table, pts):
    """Bilinear interpolation of table [npairs][ny][nx] at pts [Q][2] -> [npairs][Q]."""
    j1, j2, tx, ty = bilinear_corners(grid, pts)
    t = np.asarray(table)
    return ((1 - tx) * (1 - ty) * t[:, j2, j1] + tx * (1 - ty) * t[:, j2, j1 + 1]
            + (1 - tx) * ty * t[:, j2 + 1, j1] + tx * ty * t[:, j2 + 1, j1 + 1])


def quadratic_nodes(grid, pts):
    """Stencil centre and offsets of second-order (3 x 3 Lagrange) interpolation.

    Sec. III-B.3, last paragraph: the refined table is searched with a
    second-order interpolation.  Reading: per axis the three nodes around the
    nearest one, c - 1, c, c + 1, with c = round(u) kept in [1, n-2] (u the
    fractional table index), and the quadratic Lagrange weights in
    t = u - c: t (t - 1)/2, 1 - t^2, t (t + 1)/2.  Points must satisfy
    0 <= u <= n - 1 on both axes.  Returns (c1, c2, tx, ty).
    """
    pts = np.asarray(pts, dtype=np.float64)
    x_max = grid.nx * math.pi / (2.0 * grid.kx_max)
    y_max = grid.ny * math.pi / (2.0 * grid.ky_max)
    ux = (pts[:, 0] + x_max) / (math.pi / grid.kx_max)
    uy = (pts[:, 1] + y_max) / (math.pi / grid.ky_max)
    if np.any(ux < 0) or np.any(ux > grid.nx - 1) or np.any(uy < 0) or np.any(uy > grid.ny - 1):
        raise ValueError("query outside the table")
    c1 = np.clip(np.floor(ux + 0.5).astype(np.int64), 1, grid.nx - 2)
    c2 = np.clip(np.floor(uy + 0.5).astype(np.int64), 1, grid.ny - 2)
    return c1, c2, ux - c1, uy - c2


def lagrange3(t):
    """Quadratic Lagrange weights of the nodes -1, 0, +1 at offset t."""
    return np.stack([0.5 * t * (t - 1.0), (1.0 - t) * (1.0 + t), 0.5 * t * (t + 1.0)])


def quadratic_lookup(grid, table, pts):
    """Second-order interpolation of table [npairs][ny][nx] at pts [Q][2] -> [npairs][Q]."""
    c1, c2, tx, ty = quadratic_nodes(grid, pts)
    wx, wy = lagrange3(tx), lagrange3(ty)
    t = np.asarray(table)
    out = np.zeros((t.shape[0], len(c1)), dtype=np.complex128)
    for b in range(3):
        for a in range(3):
            out += wy[b] * wx[a] * t[:, c2 + b - 1, c1 + a - 1]
    return out


def fill_reduced(grid, table, pairs, nmbf, positions, order=2):
    """Substrate part of the reduced MoM matrix of an array of identical elements.

    The reduced matrix is MA x MA (Sec. II, eq. MBF): block (i, j) holds the
    interactions of the MBFs of testing element i with those of basis
    element j.  Sec. III-B.1 and Sec. III-B.3 (last paragraph) fill it from
    the table: entry (m, n) of block (i, j) is Z'_mn read at the relative
    displacement r_i - r_j by low-order interpolation (order 2:
    quadratic_lookup, order 1: bilinear_lookup).  Row i*M + m, column
    j*M + n.  Self blocks (i = j; the paper computes them by the traditional
    MBF method, Sec. IV-F), (m, n) not listed in pairs and displacements
    outside the table stay NaN.
    """
    pos = np.asarray(positions, dtype=np.float64)
    a_count = pos.shape[0]
    out = np.full((a_count * nmbf, a_count * nmbf), complex(np.nan, np.nan))
    ii, jj = np.nonzero(~np.eye(a_count, dtype=bool))
    delta = pos[ii] - pos[jj]
    x_max = grid.nx * math.pi / (2.0 * grid.kx_max)
    y_max = grid.ny * math.pi / (2.0 * grid.ky_max)
    ux = (delta[:, 0] + x_max) / (math.pi / grid.kx_max)
    uy = (delta[:, 1] + y_max) / (math.pi / grid.ky_max)
    inside = (ux >= 0) & (ux <= grid.nx - 1) & (uy >= 0) & (uy <= grid.ny - 1)
    if order == 1:
        inside &= (ux < grid.nx - 1) & (uy < grid.ny - 1)
    ii, jj, delta = ii[inside], jj[inside], delta[inside]
    vals = (quadratic_lookup if order == 2 else bilinear_lookup)(grid, table, delta)
    for p, (m, n) in enumerate(pairs):
        out[ii * nmbf + m, jj * nmbf + n] = vals[p]
    return out


def interpolation_corners(grid, pts, order=1):
    """(j1, j2, weight) of every table node an interpolated value uses: the
    four bilinear corners (order 1) or the 3 x 3 second-order stencil of
    quadratic_nodes with the products of lagrange3 weights (order 2)."""
    if order == 2:
        c1, c2, tx, ty = quadratic_nodes(grid, pts)
        wx, wy = lagrange3(tx), lagrange3(ty)
        return [(c1 + a - 1, c2 + b - 1, wx[a] * wy[b]) for b in range(3) for a in range(3)]
    j1, j2, tx, ty = bilinear_corners(grid, pts)
    return [(j1, j2, (1 - tx) * (1 - ty)), (j1 + 1, j2, tx * (1 - ty)),
            (j1, j2 + 1, (1 - tx) * ty), (j1 + 1, j2 + 1, tx * ty)]


def lookup_direct(grid, substrate, basis, q, pairs, pts, workers=1, order=1):
    """Lookup (bilinear or second order) with the nodes it uses evaluated by direct sum only."""
    corners = interpolation_corners(grid, pts, order)
    idx = np.concatenate([c[1] * grid.nx + c[0] for c in corners])
    z = tabulate(grid, substrate, basis, q, pairs, out_idx=idx, workers=workers)
    nq = len(pts)
    out = np.zeros((len(pairs), nq), dtype=np.complex128)
    for i, (_, _, wgt) in enumerate(corners):
        out += wgt * z[:, i * nq:(i + 1) * nq]
    return out


# --------------------------------------------------------------------------
# Loss and its gradient (differentiation of the tabulation)
# --------------------------------------------------------------------------
def loss_value(z_pts, z_target):
    """L = sum over points and pairs of |Z - Z_target|^2."""
    r = np.asarray(z_pts) - np.asarray(z_target)
    return float(np.sum(r.real ** 2 + r.imag ** 2))


def _with_substrate(substrate, eps_r=None, h=None):
    import copy
    s = copy.copy(substrate)
    if eps_r is not None:
        s.eps_r = eps_r
    if h is not None:
        s.h = h
    return s


def cauchy_derivative(f, z0, radius=None, count=32):
    """f'(z0) of a holomorphic f by the trapezoidal Cauchy integral (Lyness-Moler).

    f'(z0) ~ 1/(K r) sum_k f(z0 + r e^{2 pi i k/K}) e^{-2 pi i k/K}; the error
    decays like (r/rho)^K for f analytic in a disc of radius rho > r.  The
    table is analytic in eps_r and h only up to the substrate values at which
    a surface-wave pole reaches a contour sample, which for a thin slab lies
    within ~20 % of h; the default radius is therefore 0.2 % of |z0|.
    """
    if radius is None:
        radius = 2e-3 * max(abs(z0), 1e-3)
    acc = None
    for k in range(count):
        e = np.exp(2j * math.pi * k / count)
        v = np.asarray(f(z0 + radius * e)) * np.conj(e)
        acc = v if acc is None else acc + v
    return acc / (count * radius)


def loss_gradient(grid, substrate, basis, q, pairs, pts, z_target, workers=1, order=1):
    """(L, dL/d eps_r, dL/d h, dL/dq) of the lookup loss, in FP64.

    The lookup is bilinear (order 1) or second order (order 2, the
    interpolation of Sec. III-B.3 in the refined table); on a zero-padded
    grid only the band samples carry the integrand (band_mask).

    eps_r and h enter the table holomorphically, so dZ/dtheta comes from the
    Cauchy rule applied to the oracle's own forward map with complex theta;
    then dL/dtheta = 2 Re sum conj(Z - Z_t) dZ/dtheta.  q enters
    sesquilinearly (eq. MBF: Z' = Q^H Z Q), so its gradient is exact: with
    A_jn the table of (testing = basis j, basis = MBF n) and B_mj that of
    (testing = MBF m, basis = basis j),
        dL/dq_kj (as d/dRe + i d/dIm) = 2 [sum_n A_jn conj(R_kn) + sum_m R_mk conj(B_mj)]
    where R = Z - Z_target.  Returns the gradient of q in the same
    d/dRe + i d/dIm convention.
    """
    pairs = np.asarray(pairs)
    z = lookup_direct(grid, substrate, basis, q, pairs, pts, workers=workers, order=order)
    r = z - z_target
    loss = loss_value(z, z_target)

    def z_of_eps(e):
        return lookup_direct(grid, _with_substrate(substrate, eps_r=e), basis, q, pairs, pts, workers=workers,
                             order=order)

    def z_of_h(hh):
        return lookup_direct(grid, _with_substrate(substrate, h=hh), basis, q, pairs, pts, workers=workers,
                             order=order)

    dz_de = cauchy_derivative(z_of_eps, substrate.eps_r)
    dz_dh = cauchy_derivative(z_of_h, substrate.h)
    d_eps = 2.0 * float(np.sum((np.conj(r) * dz_de).real))
    d_h = 2.0 * float(np.sum((np.conj(r) * dz_dh).real))

    # exact q gradient from single-basis tables
    m_count, b_count = q.shape
    corners = interpolation_corners(grid, pts, order)
    idx = np.concatenate([c[1] * grid.nx + c[0] for c in corners])
    kx, ky, w, g, mt, mh = sampled_factors(grid, substrate, basis, q)
    eye = np.eye(b_count, dtype=np.complex128)
    # unit-coefficient spectra of each basis: testing side uses conj(1) = 1
    kcx, kcy, _, gam = grid_contour(kx, ky, grid)
    ut, uh = mbf_spectra(basis, eye, kcx, kcy)
    dxa = displacement_axis(grid.nx, grid.kx_max)
    dya = displacement_axis(grid.ny, grid.ky_max)
    DX, DY = np.meshgrid(dxa, dya)
    dx, dy = DX.ravel()[idx], DY.ravel()[idx]
    dkx = 2.0 * grid.kx_max / grid.nx
    dky = 2.0 * grid.ky_max / grid.ny
    gxx, gxy, gyy = g
    nq = len(pts)

    def lookup_of(integ):
        zz = direct_sum(integ, kx, ky, dx, dy, gam, grid.order, dkx, dky, workers=workers,
                        truncation=getattr(grid, "truncation", 0))
        out = np.zeros((integ.shape[0], nq), dtype=np.complex128)
        for i, (_, _, wgt) in enumerate(corners):
            out += wgt * zz[:, i * nq:(i + 1) * nq]
        return out

    mask = band_mask(grid)
    mask = 1.0 if mask is None else mask
    # A[j, n]: testing basis j (unit), basis MBF n
    a_int = np.stack([integrand(ut[j], mh[n], gxx, gxy, gyy, w) for j in range(b_count) for n in range(m_count)]) * mask
    A = lookup_of(a_int).reshape(b_count, m_count, nq)
    # B[m, j]: testing MBF m, basis j (unit)
    b_int = np.stack([integrand(mt[m], uh[j], gxx, gxy, gyy, w) for m in range(m_count) for j in range(b_count)]) * mask
    Bm = lookup_of(b_int).reshape(m_count, b_count, nq)
    # residual per (m, n)
    R = np.zeros((m_count, m_count, nq), dtype=np.complex128)
    for p, (m, n) in enumerate(pairs):
        R[m, n] += r[p]
    present = np.zeros((m_count, m_count), dtype=bool)
    for m, n in pairs:
        present[m, n] = True
    gq = np.zeros((m_count, b_count), dtype=np.complex128)
    for k in range(m_count):
        for n in range(m_count):
            if present[k, n]:
                gq[k] += np.sum(A[:, n, :] * np.conj(R[k, n])[None, :], axis=1)
        for m in range(m_count):
            if present[m, k]:
                gq[k] += np.sum(R[m, k][None, :] * np.conj(Bm[m]), axis=1)
    gq *= 2.0
    return loss, d_eps, d_h, gq
