/*
 * cfft.h -- C ABI of the MI355X contour-FFT (C-FFT) tabulation library.
 *
 * The library tabulates the substrate-related reaction terms Z'_mn between
 * Macro Basis Functions (MBFs) of identical printed antennas on a grounded
 * dielectric slab, for every relative displacement on a regular grid, as in
 * Jha & Craeye, "Contour-FFT based Spectral Domain MBF Analysis of Large
 * Printed Antenna Arrays":
 *
 *   Z'_mn(Dx,Dy) = 1/(4 pi^2) sum_{n1,n2} I_mn(k) exp(-i k.D) T_P(g k.D) dkx dky
 *   I_mn(k)      = W * M_m(k_c) . G_s(k_c) . M#_n(k_c),   k_c = (1 + i g) k
 *
 * with g = beta_I/beta_R the contour ratio of eq. ratioNew and W = (1 + i
 * d beta_I/d beta_R)(1 + i g) the weight of eq. FFT.  Ray contour: g = gamma
 * everywhere, W = (1 + i gamma)^2.  Parabolic contour (the deformation the
 * paper names, Sec. I and Fig. 1): beta_I = gamma beta (1 - beta/beta_end)
 * below beta_end and 0 beyond, so g = gamma (1 - beta/beta_end) varies per
 * sample, the per-axis factorisation of the Taylor terms is lost, and the row
 * pass runs all (P+1)(P+2)/2 terms of eq. fftarry.
 *
 * (Sec. III-A eqs. spectral, MBF_mul, MBF_mul22, FTMBF; Sec. III-B.2 eqs.
 * complexbeta..ratioNew and FFT; Sec. III-B.3 eqs. taylors, fftexp, fftarry;
 * Appendix change of variables.)  T_P is the Taylor polynomial of order P of
 * the contour's real exponential E_I, truncated at total degree P.
 *
 * Conventions.  Time dependence exp(+i w t); lengths in free-space
 * wavelengths at f0 (lambda0 = 1), k0 = 2 pi f/f0; eta0 = 1; lossy
 * permittivity eps_r (1 - i tan_delta); F(k) = int f(r) exp(-i k.r) dr;
 * D = r_test - r_basis.  Complex numbers are interleaved (re, im).  Arrays
 * are row-major with x fastest.
 *
 * Grids (Appendix).  Spectral samples kx(n1) = -kx_max + n1 * 2 kx_max/nx,
 * n1 = 0..nx-1 (likewise y); output displacements Dx(j1) = -x_max + j1 pi/kx_max
 * with x_max = nx pi/(2 kx_max), so D = 0 sits at j1 = nx/2.
 *
 * Memory ownership.  The caller owns every bulk device buffer (inputs and
 * outputs).  A plan owns its twiddle tables, geometry tables and the
 * workspace for the intermediate arrays between the row and column passes,
 * and frees them in c_fft_plan_destroy.  Host arrays passed to a call are
 * read during the call and not retained.
 *
 * Execution.  Entry points taking a `stream` (a hipStream_t, NULL = the
 * default stream) enqueue their kernels on it and return without waiting,
 * except where stated.  One plan must not be used from two streams at once,
 * with one exception: slab_green_eval touches no plan workspace, so it may
 * run on a second stream beside the other entry points of the same plan
 * when the plan was made without CFFT_FLAG_CHECK_FINITE.  A plan is not
 * thread-safe: issue its calls from one host thread at a time.
 *
 * Environment (read at each call).  CFFT_WORKSPACE_MB caps the pass
 * workspace of a plan (MiB, default 65536; the pairs then go in smaller
 * chunks).  CFFT_PAIR_CHUNK (pairs per launch), CFFT_LANES (1 or 2) and
 * CFFT_COL_TILE (0 default, 1 half width, 2 the other points per thread on
 * columns of 1024 points and more) force one schedule of cfft_tabulate and
 * switch CFFT_FLAG_AUTOTUNE off; values outside these ranges are ignored.
 * CFFT_TEST_FAIL_ALLOC (non-empty, not "0") makes every device allocation
 * of the library fail with CFFT_ERR_ALLOC, to test that path.
 *
 * Errors.  Every call returns a status.  Arguments are validated on the host
 * before anything is launched; on error nothing is enqueued and
 * cfft_last_error() returns a message (thread-local).  No exception or abort
 * crosses the ABI.  There is no CPU fallback: without a usable gfx950 device
 * the calls fail with CFFT_ERR_HIP.
 */
#ifndef CFFT_H
#define CFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cfft_plan_s* cfft_plan_t;

typedef enum {
  CFFT_OK = 0,
  CFFT_ERR_INVALID_ARG = 1,   /* bad size, null pointer, out-of-range index, non-finite scalar */
  CFFT_ERR_UNSUPPORTED = 2,   /* valid request outside what the library implements */
  CFFT_ERR_ALLOC = 3,         /* device allocation failed */
  CFFT_ERR_HIP = 4,           /* HIP runtime error (no device, launch failure) */
  CFFT_ERR_NONFINITE = 5      /* a kernel produced NaN/Inf (only with CFFT_FLAG_CHECK_FINITE) */
} cfft_status_t;

enum { CFFT_CONTOUR_RAY = 0, CFFT_CONTOUR_PARABOLIC = 1 };
/* Truncation of the Taylor series of E_I (eq. taylors):
 *   TOTAL : terms (gamma kx Dx)^a (gamma ky Dy)^b / (a! b!) with a + b <= P,
 *           the N_t = (P+1)(P+2)/2 terms of eq. fftarry;
 *   TENSOR: every term with a <= P and b <= P.  On the ray contour E_I is
 *           exactly exp(gamma kx Dx) exp(gamma ky Dy), and this truncation is
 *           the product of the two per-axis Taylor polynomials: a superset of
 *           TOTAL's terms, and one intermediate array per pair between the
 *           row and column passes instead of P+1.  Not in the paper. */
enum { CFFT_TRUNC_TOTAL = 0, CFFT_TRUNC_TENSOR = 1 };
enum { CFFT_FP64 = 0, CFFT_MIXED = 1 };
enum { CFFT_ROOFTOP_X = 0, CFFT_ROOFTOP_Y = 1, CFFT_COSINE_X = 2, CFFT_COSINE_Y = 3 };
/* CHECK_FINITE: scan every output for NaN/Inf and report CFFT_ERR_NONFINITE
 *   (makes the call synchronous).
 * AUTOTUNE: the first cfft_tabulate per (grid, npairs) times the candidate
 *   schedules (synchronously): pairs per launch, one or two plan-owned lanes
 *   taking alternate chunks, and the column tile (the default, half its
 *   width, or for columns of 1024 points and more the other number of points
 *   per thread, 8 or 16, with its widest tile); the plan keeps the fastest.  That first call runs the passes several times on the
 *   caller's buffers (z ends with the same table).
 * ZERO_PAD2: every grid of the plan is the x2 zero-padded extension of the
 *   grid the caller samples (Sec. III-B.3, last paragraph: Whittaker-Shannon
 *   refinement with zero padding to twice the FFT size).  Only the central
 *   half of the samples on each axis, n in [N/4, 3N/4), carries the
 *   integrand; the table then has half the displacement step over the same
 *   span, and its even nodes are the unrefined table.  The grid descriptor
 *   describes the padded grid (2N samples over twice the spectral span).
 *   slab_green_eval and mbf_spectra still write every sample; the passes
 *   read only the band and skip the rows that are zero; cfft_backward
 *   returns no gradient from the samples outside the band. */
enum { CFFT_FLAG_CHECK_FINITE = 1, CFFT_FLAG_AUTOTUNE = 2, CFFT_FLAG_ZERO_PAD2 = 4 };

/* One spectral grid.  64 bytes, natural alignment. */
typedef struct {
  int32_t nx, ny;        /* samples = outputs per axis: powers of two, 16 <= n <= 4096 */
  double kx_max, ky_max; /* spectral half-spans (rad per lambda0), > 0 */
  double k0;             /* free-space wavenumber 2 pi f/f0, > 0 */
  double gamma;          /* contour height ratio beta_I/beta_R (eq. ratioNew), > 0 */
  int32_t contour;       /* CFFT_CONTOUR_RAY or CFFT_CONTOUR_PARABOLIC */
  int32_t order;         /* Taylor order P >= 0 of eq. taylors, 0 <= P <= 7 */
  double beta_end;       /* PARABOLIC: where the path rejoins the real axis (> every
                            surface-wave pole), finite > 0; unused for RAY */
  int32_t precision;     /* CFFT_FP64 (complex128 everywhere) or CFFT_MIXED */
  int32_t truncation;    /* CFFT_TRUNC_TOTAL (0, the paper's) or CFFT_TRUNC_TENSOR */
} cfft_grid_desc_t;

/* One elementary basis function (40 bytes).  Sec. III-A: rooftops with an
 * analytic Fourier transform.
 *   CFFT_ROOFTOP_X: x-directed, triangle of half-base a along x, pulse of width b along y
 *   CFFT_ROOFTOP_Y: y-directed transpose
 *   CFFT_COSINE_X : x-directed cos(pi (x-cx)/a) on |x-cx| <= a/2, pulse of width b along y
 *   CFFT_COSINE_Y : y-directed transpose
 * (cx, cy) is the centre relative to the antenna's local origin. */
typedef struct {
  int32_t kind;
  int32_t pad;           /* must be 0 */
  double cx, cy, a, b;   /* a > 0, b > 0 */
} cfft_basis_t;

/* Create a plan for `ngrids` grids (a frequency sweep may use one grid per
 * frequency) and up to `max_mbf` MBFs per antenna (1..16).  Allocates the
 * twiddle tables on the current device (synchronous).  `flags` is a bitwise
 * OR of CFFT_FLAG_*.  On success *out receives the plan. */
cfft_status_t c_fft_plan(const cfft_grid_desc_t* grids, int32_t ngrids, int32_t max_mbf,
                         int32_t flags, cfft_plan_t* out);

/* Free a plan and everything it owns (synchronises the device first).
 * NULL is accepted and ignored. */
cfft_status_t c_fft_plan_destroy(cfft_plan_t plan);

/* Grounded-slab spectral dyadic Green's function minus the effective
 * homogeneous medium (eps_e = (eps_r + 1)/2) and its image through the ground
 * plane (Sec. II, Sec. III-A), sampled at k_c = (1 + i gamma) k on every
 * sample of grid `grid`, in FP64.
 *   g : device, complex128 [3][ny][nx]: Gxx, Gxy (= Gyx), Gyy.
 * eps_r >= 1 finite, tan_delta >= 0, h > 0 (in lambda0). */
cfft_status_t slab_green_eval(cfft_plan_t plan, int32_t grid, double eps_r, double tan_delta,
                              double h, void* g, void* stream);

/* Spectra of the MBFs on the contour (eq. FTMBF), evaluated in FP64 and
 * stored in the grid's precision: complex128 for CFFT_FP64, complex64
 * (rounded) for CFFT_MIXED.
 *   basis : host, nbasis records (read during the call; the geometry is
 *           uploaded to plan-owned device memory, blocking, and cached)
 *   q     : device, complex128 [nmbf][nbasis], row m = coefficients of MBF m
 *   spec  : device, complex128 or complex64 [nmbf][4][ny][nx]:
 *           [0] Mx_m(k_c) = sum_j conj(q_mj) Fx_j(k_c)    (testing side)
 *           [1] My_m(k_c)
 *           [2] Mx#_m(k_c) = sum_j q_mj Fx_j(-k_c)        (basis side: analytic
 *           [3] My#_m(k_c)                                  reflection of conj M)
 * 1 <= nmbf <= max_mbf, 1 <= nbasis <= 65536. */
cfft_status_t mbf_spectra(cfft_plan_t plan, int32_t grid, const cfft_basis_t* basis,
                          int32_t nbasis, const void* q, int32_t nmbf, void* spec, void* stream);

/* The C-FFT table (eqs. FFT, fftexp, fftarry and the Appendix) for the
 * listed MBF pairs: integrand assembly, contour weight, P+1 row FFTs per row
 * (ray contour; (P+1)(P+2)/2 on the parabolic contour) with partial
 * recombination, P+1 column FFTs per column with the per-output
 * recombination and the Appendix scaling.
 *   spec  : device, output of mbf_spectra for nmbf MBFs (the grid's precision)
 *   g     : device, output of slab_green_eval
 *   pairs : host, int32 [npairs][2] = (m, n), 0 <= m, n < nmbf (testing m, basis n)
 *   z     : device [npairs][ny][nx], complex128 (FP64) or complex64 (MIXED);
 *           z[p][j2][j1] = Z'_mn(Dx(j1), Dy(j2))
 * 1 <= npairs <= 4096.  The plan's workspace grows on first use (allocation
 * is synchronous; later calls of the same or smaller size do not allocate). */
cfft_status_t cfft_tabulate(cfft_plan_t plan, int32_t grid, const void* spec, int32_t nmbf,
                            const void* g, const int32_t* pairs, int32_t npairs, void* z,
                            void* stream);

/* Allocation-free cfft_tabulate, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, result and errors as cfft_tabulate, but
 * the intermediates between the row and column passes live in a fixed
 * device array of CFFT_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device it runs on (resolved by c_fft_plan) instead of the plan's
 * workspace, and no schedule is autotuned (one lane, pairs in chunks that
 * fit the array; CFFT_FLAG_AUTOTUNE is ignored here).  The call allocates
 * no device memory.
 *   Limit: the intermediates of one pair, (P+1) nx ny complex values in the
 *   grid's storage precision (one value per sample with the tensor
 *   truncation), must fit the array: up to 2048^2 FP64 or 4096 x 2048 mixed
 *   at P = 3.  Larger grids return CFFT_ERR_UNSUPPORTED before any launch.
 *   Concurrency: every call on a device shares that device's array, so calls
 *   that overlap in time on one device (other streams, other plans, other
 *   host threads) race; serialise them. */
#define CFFT_NOALLOC_SCRATCH_BYTES (256u << 20)
cfft_status_t cfft_tabulate_noalloc(cfft_plan_t plan, int32_t grid, const void* spec, int32_t nmbf,
                                    const void* g, const int32_t* pairs, int32_t npairs, void* z,
                                    void* stream);

/* Bilinear interpolation in the table (first-order stand-in for the
 * interpolation of Sec. III-B.3, last paragraph).
 *   z   : device table as written by cfft_tabulate (precision of the grid)
 *   pts : device, float64 [npts][2] = (Dx, Dy)
 *   out : device, complex128 [npairs][npts]
 * A point outside [Dx(0), Dx(nx-1)) x [Dy(0), Dy(ny-1)) yields NaN. */
cfft_status_t cfft_lookup(cfft_plan_t plan, int32_t grid, const void* z, int32_t npairs,
                          const double* pts, int32_t npts, void* out, void* stream);

/* Second-order interpolation in the table (Sec. III-B.3, last paragraph:
 * the refined tables are searched with a second-order method).  Per axis the
 * three nodes c-1, c, c+1 around the nearest node c (kept inside the
 * table), with quadratic Lagrange weights.  Same arguments and output as
 * cfft_lookup; a point outside [Dx(0), Dx(nx-1)] x [Dy(0), Dy(ny-1)] yields
 * NaN. */
cfft_status_t cfft_lookup_quadratic(cfft_plan_t plan, int32_t grid, const void* z, int32_t npairs,
                                    const double* pts, int32_t npts, void* out, void* stream);

/* Reduced-matrix fill for an array of identical elements (Sec. II eq. MBF:
 * the reduced matrix is MA x MA; Sec. III-B.1 and the last paragraph of
 * Sec. III-B.3: its blocks are read from the table by low-order
 * interpolation).  For every ordered pair of distinct elements (i, j) and
 * every listed MBF pair k = (m, n):
 *   out[(i*nmbf + m) * (nelem*nmbf) + j*nmbf + n] = Z'_mn(r_i - r_j)
 * interpolated in table k of z (order 1: as cfft_lookup, 2: as
 * cfft_lookup_quadratic; NaN outside the table).
 *   z     : device table as written by cfft_tabulate for these pairs
 *   pairs : host int32 [npairs][2], 0 <= m, n < nmbf, each (m, n) at most once
 *   pos   : device float64 [nelem][2], element reference points (x, y) [lambda0]
 *   out   : device complex128 [nelem*nmbf][nelem*nmbf], row-major, caller-owned
 * Self blocks (i == j) and entries of unlisted (m, n) are not written: the
 * caller fills them (the paper computes self terms by the traditional MBF
 * method).  Limits: 1 <= nmbf <= 16, nelem*nmbf <= 65535, order 1 or 2;
 * violations return CFFT_ERR_INVALID_ARG before any launch. */
cfft_status_t cfft_fill(cfft_plan_t plan, int32_t grid, const void* z, const int32_t* pairs,
                        int32_t npairs, int32_t nmbf, const double* pos, int32_t nelem,
                        int32_t order, void* out, void* stream);

/* Adjoint of cfft_fill: every entry the fill writes scatters its cotangent,
 * times its interpolation weights, into the table of its pair:
 *   dz[k][j2][j1] += sum over written entries of weight(j1, j2) dout[row][col]
 *   dout : device complex128 [nelem*nmbf][nelem*nmbf], dL/dRe + i dL/dIm
 *   dz   : device complex128 [npairs][ny][nx], zeroed by the caller before
 *          the first accumulation (FP64 grids only)
 * Other arguments and limits as cfft_fill; entries that the fill does not
 * write (self blocks, unlisted pairs, displacements outside the table)
 * contribute nothing. */
cfft_status_t cfft_fill_backward(cfft_plan_t plan, int32_t grid, const void* dout, const int32_t* pairs,
                                 int32_t npairs, int32_t nmbf, const double* pos, int32_t nelem,
                                 int32_t order, void* dz, void* stream);

/* Adjoint of cfft_lookup: dz[p][j2][j1] += sum over points of the bilinear
 * weight times dout[p][q] (complex128, FP64 grids only).  dz must be zeroed
 * by the caller before the first accumulation. */
cfft_status_t cfft_lookup_backward(cfft_plan_t plan, int32_t grid, const void* dout,
                                   int32_t npairs, const double* pts, int32_t npts, void* dz,
                                   void* stream);

/* Adjoint of cfft_lookup_quadratic: dz[p][j2][j1] += sum over points of the
 * 3 x 3 Lagrange weight of node (j1, j2) times dout[p][q]; points outside
 * the table contribute nothing.  Same arguments, layout and conditions as
 * cfft_lookup_backward. */
cfft_status_t cfft_lookup_quadratic_backward(cfft_plan_t plan, int32_t grid, const void* dout,
                                             int32_t npairs, const double* pts, int32_t npts, void* dz,
                                             void* stream);

/* Gradient of a real loss L through the whole table (FP64 grids on the ray
 * contour, zero-padded or not; other grids return CFFT_ERR_UNSUPPORTED).
 *   dz       : device complex128 [npairs][ny][nx], dL/dRe z + i dL/dIm z
 *   eps_r, tan_delta, h, basis, nbasis, q, nmbf, pairs, npairs : the forward inputs
 *   g, spec  : device, the forward's sampled Green's function and spectra
 *              (the checkpoint of the sampled integrand; required)
 *   grad_sub : device float64 [2] <- (dL/d eps_r, dL/d h), overwritten
 *   grad_q   : device complex128 [nmbf][nbasis] <- dL/dRe q + i dL/dIm q, overwritten
 * eps_r is differentiated as the real part eps' of eps' (1 - i tan_delta). */
cfft_status_t cfft_backward(cfft_plan_t plan, int32_t grid, const void* dz, double eps_r,
                            double tan_delta, double h, const cfft_basis_t* basis, int32_t nbasis,
                            const void* q, int32_t nmbf, const int32_t* pairs, int32_t npairs,
                            const void* g, const void* spec, double* grad_sub, void* grad_q,
                            void* stream);

/* Kernel timing (instrumentation).  While enabled, every kernel a plan
 * launches is bracketed by HIP events on the caller's stream, per kernel
 * class; cfft_profile_read waits for the recorded events and returns the
 * summed duration (ms) and launch count of one class since the last read
 * (the class's events are released).  Classes:
 *   0 slab_green_eval  1 mbf_spectra tables+spectra  2 row pass  3 column pass
 *   4 lookup  5 adjoint column pass  6 adjoint row pass  7 integrand adjoint
 *   8 Green's function adjoint + reductions  9 spectra adjoint
 * enable = 0 disables recording (pending events are kept until read). */
cfft_status_t cfft_profile(cfft_plan_t plan, int32_t enable);
cfft_status_t cfft_profile_read(cfft_plan_t plan, int32_t kernel_class, double* total_ms, int64_t* launches);

/* Message of the last failed call on this thread ("" if none). */
const char* cfft_last_error(void);

/* Library version string. */
const char* cfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CFFT_H */
