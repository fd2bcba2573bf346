"""MI355X (gfx950) contour-FFT tabulation of substrate-related MBF reaction terms.

Python face of libcfft.so (include/cfft.h).  PyTorch provides device memory
and streams; every step of the method runs in the library's HIP kernels.
Importing the package fails loudly when the library is not built.

    from paper_1404_7357_amd import Tabulator
    tab = Tabulator(grid, basis, max_mbf=4)
    g = tab.green(eps_r, tan_delta, h)          # [3][ny][nx] complex128
    spec = tab.spectra(q)                       # [M][4][ny][nx] complex128 (complex64 for mixed grids)
    z = tab.tabulate(spec, g, pairs)            # [npairs][ny][nx]
    vals = tab.lookup(z, pts)                   # [npairs][Q] complex128
"""
from __future__ import annotations

import math

import torch

from . import _lib
from ._lib import (CONTOUR_RAY, FLAG_AUTOTUNE, FLAG_CHECK_FINITE, FLAG_ZERO_PAD2, FP64, MIXED,  # noqa: F401
                   TRUNC_TENSOR, TRUNC_TOTAL, CfftError, Plan, cfft_backward, cfft_fill, cfft_fill_backward, cfft_lookup,
                   cfft_lookup_backward, cfft_lookup_quadratic, cfft_lookup_quadratic_backward, cfft_tabulate,
                   mbf_spectra, slab_green_eval)

_lib.load()

__all__ = ["Tabulator", "Plan", "CfftError", "TableFunction", "LookupFunction", "FillFunction", "FP64", "MIXED",
           "slab_green_eval", "mbf_spectra", "cfft_tabulate", "cfft_lookup", "cfft_lookup_quadratic",
           "cfft_fill", "cfft_fill_backward", "cfft_lookup_backward", "cfft_lookup_quadratic_backward", "cfft_backward",
           "displacement_axis"]


def displacement_axis(n: int, k_max: float):
    """Output displacements of the table along one axis (host helper, float64)."""
    x_max = n * math.pi / (2.0 * k_max)
    return [-x_max + j * math.pi / k_max for j in range(n)]


def _check_buffer(t, shape, dtype, name):
    """Shape, dtype, memory layout and device of a caller-provided buffer (the C
    ABI sees only a pointer): any mismatch raises ValueError before a launch."""
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        raise ValueError(f"{name} must be a {dtype} cuda tensor of shape {tuple(shape)}, got {t.dtype} "
                         f"{tuple(t.shape)} on {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (the library reads it as a dense row-major array)")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a cuda tensor, got one on {t.device}")


class Tabulator:
    """One plan bound to one or more grids and one basis set."""

    def __init__(self, grids, basis, max_mbf: int, flags: int = 0, device: str = "cuda"):
        self.grids = list(grids) if isinstance(grids, (list, tuple)) else [grids]
        self.plan = Plan(self.grids, max_mbf, flags)
        self.basis = _lib.basis_array(basis)
        self.nbasis = len(self.basis)
        self.device = torch.device(device)

    def _grid(self, i):
        return self.grids[i]

    def green(self, eps_r, tan_delta, h, grid: int = 0, out=None, stream=None):
        gd = self._grid(grid)
        g = out if out is not None else torch.empty((3, gd.ny, gd.nx), dtype=torch.complex128, device=self.device)
        _check_buffer(g, (3, gd.ny, gd.nx), torch.complex128, "out")
        slab_green_eval(self.plan, grid, eps_r, tan_delta, h, g, stream)
        return g

    def _table_dtype(self, grid):
        return torch.complex128 if self._grid(grid).precision == FP64 else torch.complex64

    def _check_table(self, z, grid):
        """A table as cfft_tabulate writes it for this grid: [npairs][ny][nx] in the grid's precision."""
        gd = self._grid(grid)
        if z.dim() != 3:
            raise ValueError(f"z must be a table [npairs][{gd.ny}][{gd.nx}], got shape {tuple(z.shape)}")
        _check_buffer(z, (z.shape[0], gd.ny, gd.nx), self._table_dtype(grid), "z")

    def spectra(self, q, grid: int = 0, out=None, stream=None):
        gd = self._grid(grid)
        if q.dim() != 2:
            raise ValueError(f"q must be complex128 [M][{self.nbasis}], got shape {tuple(q.shape)}")
        _check_buffer(q, (q.shape[0], self.nbasis), torch.complex128, "q")
        sdt = torch.complex128 if gd.precision == FP64 else torch.complex64
        spec = out if out is not None else torch.empty((q.shape[0], 4, gd.ny, gd.nx), dtype=sdt, device=self.device)
        _check_buffer(spec, (q.shape[0], 4, gd.ny, gd.nx), sdt, "out")
        mbf_spectra(self.plan, grid, self.basis, q, spec, stream)
        return spec

    def tabulate(self, spec, g, pairs, grid: int = 0, out=None, stream=None):
        gd = self._grid(grid)
        dt = torch.complex128 if gd.precision == FP64 else torch.complex64
        z = out if out is not None else torch.empty((len(pairs), gd.ny, gd.nx), dtype=dt, device=self.device)
        _check_buffer(z, (len(pairs), gd.ny, gd.nx), dt, "out")
        _check_buffer(g, (3, gd.ny, gd.nx), torch.complex128, "g")
        _check_buffer(spec, (spec.shape[0], 4, gd.ny, gd.nx), dt, "spec")
        cfft_tabulate(self.plan, grid, spec, spec.shape[0], g, pairs, z, stream)
        return z

    def lookup(self, z, pts, grid: int = 0, out=None, stream=None, order: int = 1):
        """Table values at displacements pts [Q][2]: bilinear (order 1) or
        second-order Lagrange (order 2) interpolation."""
        self._check_table(z, grid)
        if pts.dim() != 2:
            raise ValueError(f"pts must be float64 [Q][2], got shape {tuple(pts.shape)}")
        out = out if out is not None else torch.empty((z.shape[0], pts.shape[0]), dtype=torch.complex128,
                                                      device=self.device)
        _check_buffer(out, (z.shape[0], pts.shape[0]), torch.complex128, "out")
        _check_buffer(pts, (pts.shape[0], 2), torch.float64, "pts")
        if order == 2:
            cfft_lookup_quadratic(self.plan, grid, z, z.shape[0], pts, out, stream)
        elif order == 1:
            cfft_lookup(self.plan, grid, z, z.shape[0], pts, out, stream)
        else:
            raise ValueError("order must be 1 or 2")
        return out

    def fill(self, z, pairs, nmbf: int, pos, order: int = 2, grid: int = 0, out=None, stream=None):
        """Reduced matrix [A*M][A*M] of the element layout pos [A][2] read from
        the table z of the listed pairs; self blocks and unlisted (m, n) keep
        the contents of out (NaN when out is allocated here)."""
        self._check_table(z, grid)
        if pos.dim() != 2:
            raise ValueError(f"pos must be float64 [A][2], got shape {tuple(pos.shape)}")
        am = pos.shape[0] * nmbf
        if out is None:
            out = torch.full((am, am), complex(float("nan"), float("nan")), dtype=torch.complex128,
                             device=self.device)
        _check_buffer(out, (am, am), torch.complex128, "out")
        _check_buffer(pos, (pos.shape[0], 2), torch.float64, "pos")
        if z.shape[0] != len(pairs):
            raise ValueError(f"z holds {z.shape[0]} tables for {len(pairs)} pairs")
        cfft_fill(self.plan, grid, z, pairs, nmbf, pos, order, out, stream)
        return out

    def close(self):
        self.plan.close()


class TableFunction(torch.autograd.Function):
    """Z = table(eps_r, h, q) with the adjoint of cfft_backward.

    eps_r and h are real 0-d float64 tensors, q complex128 [M][B].  The
    forward keeps the sampled Green's function and spectra (the checkpoint of
    the sampled integrand) for the backward.
    """

    @staticmethod
    def forward(ctx, eps_r, h, q, tab: Tabulator, tan_delta: float, pairs, grid: int):
        e = float(eps_r.item())
        hh = float(h.item())
        g = tab.green(e, tan_delta, hh, grid)
        spec = tab.spectra(q.detach(), grid)
        z = tab.tabulate(spec, g, pairs, grid)
        ctx.save_for_backward(q.detach(), g, spec)
        ctx.meta = (tab, tan_delta, list(pairs), grid, e, hh)
        return z

    @staticmethod
    def backward(ctx, gz):
        q, g, spec = ctx.saved_tensors
        tab, tan_delta, pairs, grid, e, hh = ctx.meta
        gz = gz.contiguous().to(torch.complex128)
        grad_sub = torch.empty(2, dtype=torch.float64, device=gz.device)
        grad_q = torch.empty_like(q)
        cfft_backward(tab.plan, grid, gz, e, tan_delta, hh, tab.basis, q, pairs, g, spec, grad_sub, grad_q)
        return grad_sub[0], grad_sub[1], grad_q, None, None, None, None


class FillFunction(torch.autograd.Function):
    """Reduced-matrix fill of an element layout with its scatter-add adjoint
    (entries the fill does not write are zero here)."""

    @staticmethod
    def forward(ctx, z, pos, tab: Tabulator, pairs, nmbf: int, order: int = 2, grid: int = 0):
        am = pos.shape[0] * nmbf
        out = torch.zeros((am, am), dtype=torch.complex128, device=z.device)
        tab.fill(z, pairs, nmbf, pos, order=order, grid=grid, out=out)
        ctx.save_for_backward(pos)
        ctx.meta = (tab, list(pairs), nmbf, order, grid, z.shape)
        return out

    @staticmethod
    def backward(ctx, gout):
        (pos,) = ctx.saved_tensors
        tab, pairs, nmbf, order, grid, shape = ctx.meta
        dz = torch.zeros(shape, dtype=torch.complex128, device=gout.device)
        cfft_fill_backward(tab.plan, grid, gout.contiguous().to(torch.complex128), pairs, nmbf, pos, order, dz)
        return dz, None, None, None, None, None, None


class LookupFunction(torch.autograd.Function):
    """Table lookup (bilinear, order 1, or second order, order 2) with its
    scatter-add adjoint."""

    @staticmethod
    def forward(ctx, z, pts, tab: Tabulator, grid: int, order: int = 1):
        out = tab.lookup(z, pts, grid, order=order)
        ctx.save_for_backward(pts)
        ctx.meta = (tab, grid, z.shape, order)
        return out

    @staticmethod
    def backward(ctx, gout):
        (pts,) = ctx.saved_tensors
        tab, grid, shape, order = ctx.meta
        dz = torch.zeros(shape, dtype=torch.complex128, device=gout.device)
        back = cfft_lookup_quadratic_backward if order == 2 else cfft_lookup_backward
        back(tab.plan, grid, gout.contiguous().to(torch.complex128), shape[0], pts, dz)
        return dz, None, None, None, None
