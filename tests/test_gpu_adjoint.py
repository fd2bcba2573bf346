"""GPU adjoint (cfft_backward + lookup adjoint) against central finite
differences of the GPU FP64 forward and against the oracle's gradient.

Loss: L = sum_points sum_pairs |Z_mn(r_i) - Z_target|^2 with bilinear lookup,
as in the differentiation workload; gradients w.r.t. eps_r, h and every MBF
coefficient (d/dRe + i d/dIm convention, the one torch uses for complex
leaves).
"""
import math
import sys

import numpy as np
import pytest

from oracle import cfft_oracle as co
from workloads import Grid, Substrate, gaussian_coefficients, rooftop_lattice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K0 = 2 * math.pi


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _problem(n=64, m=2, seed=41, npts=32, truncation=0):
    rng = np.random.default_rng(seed)
    grid = Grid(n, n, 6 * K0, 6 * K0, K0, truncation=truncation)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, m, basis.shape[0])
    pairs = [(a, b) for a in range(m) for b in range(m)]
    dxa = co.displacement_axis(n, grid.kx_max)
    pts = rng.uniform(dxa[1], dxa[-3], (npts, 2))
    qt = q + 0.1 * gaussian_coefficients(rng, m, basis.shape[0])
    zt = co.lookup_direct(grid, Substrate(2.3, 0.0, 0.05), basis, qt, np.array(pairs), pts)
    return grid, sub, basis, q, pairs, pts, zt


def _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt, eps=None, h=None, qv=None, need_grad=True, order=1):
    from paper_1404_7357_amd import FLAG_ZERO_PAD2, LookupFunction, TableFunction, Tabulator
    tab = Tabulator(grid, basis, max_mbf=q.shape[0], flags=FLAG_ZERO_PAD2 if getattr(grid, "zero_pad", 0) else 0)
    e = torch.tensor(sub.eps_r if eps is None else eps, dtype=torch.float64, device="cuda", requires_grad=True)
    hh = torch.tensor(sub.h if h is None else h, dtype=torch.float64, device="cuda", requires_grad=True)
    qq = torch.tensor(q if qv is None else qv, device="cuda", requires_grad=True)
    z = TableFunction.apply(e, hh, qq, tab, sub.tan_delta, pairs, 0)
    v = LookupFunction.apply(z, torch.tensor(pts, device="cuda"), tab, 0, order)
    loss = (v - torch.tensor(zt, device="cuda")).abs().pow(2).sum()
    out = [float(loss.item())]
    if need_grad:
        loss.backward()
        out += [float(e.grad.item()), float(hh.grad.item()), qq.grad.cpu().numpy()]
    tab.close()
    return out


def test_gradient_vs_central_differences():
    _say("adjoint vs FD 64^2")
    grid, sub, basis, q, pairs, pts, zt = _problem()
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    step = 1e-6

    def L(**kw):
        return _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt, need_grad=False, **kw)[0]
    fd_e = (L(eps=sub.eps_r + step) - L(eps=sub.eps_r - step)) / (2 * step)
    fd_h = (L(h=sub.h + step) - L(h=sub.h - step)) / (2 * step)
    assert abs(de - fd_e) < 1e-6 * abs(fd_e), (de, fd_e)
    assert abs(dh - fd_h) < 1e-6 * abs(fd_h), (dh, fd_h)
    rng = np.random.default_rng(3)
    for _ in range(6):
        m = int(rng.integers(q.shape[0]))
        j = int(rng.integers(q.shape[1]))
        d = np.zeros_like(q)
        d[m, j] = step
        fr = (L(qv=q + d) - L(qv=q - d)) / (2 * step)
        fi = (L(qv=q + 1j * d) - L(qv=q - 1j * d)) / (2 * step)
        assert abs(dq[m, j] - (fr + 1j * fi)) < 1e-6 * np.abs(dq).max(), (m, j, dq[m, j], fr, fi)


def test_gradient_vs_oracle():
    _say("adjoint vs oracle gradient 128^2")
    grid, sub, basis, q, pairs, pts, zt = _problem(n=128, npts=64, seed=43)
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, zt)
    assert abs(loss - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * max(abs(o_de), 1e-300), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * max(abs(o_dh), 1e-300), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()


def test_gradient_five_mbfs_vs_oracle():
    """More than four MBFs, an uneven pair list (the integrand adjoint's
    generic kernel, which reads each pair's gradient once per MBF), against
    the oracle's gradient."""
    _say("adjoint 5 MBFs vs oracle 32^2")
    rng = np.random.default_rng(59)
    n, m = 32, 5
    grid = Grid(n, n, 6 * K0, 6 * K0, K0)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, m, basis.shape[0])
    pairs = [(0, 0), (1, 4), (4, 2), (3, 3), (2, 1), (4, 4), (0, 3)]
    dxa = co.displacement_axis(n, grid.kx_max)
    pts = rng.uniform(dxa[1], dxa[-3], (16, 2))
    qt = q + 0.1 * gaussian_coefficients(rng, m, basis.shape[0])
    zt = co.lookup_direct(grid, Substrate(2.3, 0.0, 0.05), basis, qt, np.array(pairs), pts)
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, zt)
    assert abs(loss - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * max(abs(o_de), 1e-300), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * max(abs(o_dh), 1e-300), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()


def test_tensor_truncation_gradient_vs_oracle_and_differences():
    """Adjoint of the tensor-product truncation (one stored intermediate per
    pair): against the oracle's gradient of the same mode and central
    differences of the GPU forward."""
    _say("adjoint tensor truncation 64^2")
    grid, sub, basis, q, pairs, pts, zt = _problem(n=64, npts=24, seed=53, truncation=1)
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, zt)
    assert abs(loss - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * abs(o_de), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * abs(o_dh), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()
    step = 1e-6

    def L(**kw):
        return _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt, need_grad=False, **kw)[0]
    fd_e = (L(eps=sub.eps_r + step) - L(eps=sub.eps_r - step)) / (2 * step)
    assert abs(de - fd_e) < 1e-6 * abs(fd_e), (de, fd_e)


@pytest.mark.parametrize("order,truncation", [(0, 0), (7, 0), (7, 1)])
def test_gradient_at_the_extreme_orders_vs_oracle(order, truncation):
    """The adjoint at Taylor order 0 (one term: the plain transform) and at
    the largest order the library takes (7: eight intermediates, or one with
    the tensor truncation), against the oracle's gradient."""
    import dataclasses
    _say(f"adjoint order {order} truncation {truncation} 32^2")
    grid, sub, basis, q, pairs, pts, zt = _problem(n=32, npts=16, seed=61 + order, truncation=truncation)
    grid = dataclasses.replace(grid, order=order)
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, zt)
    assert abs(loss - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * max(abs(o_de), 1e-300), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * max(abs(o_dh), 1e-300), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()


def test_backward_many_pairs_chunked(monkeypatch):
    """Pair chunks accumulate the Green's and spectra gradients (ragged last chunk)."""
    _say("adjoint chunked pairs")
    grid, sub, basis, q, pairs, pts, zt = _problem(n=32, m=3, seed=47, npts=16)
    full = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    monkeypatch.setenv("CFFT_PAIR_CHUNK", "2")        # 9 pairs -> chunks 2,2,2,2,1
    chunked = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    assert abs(full[1] - chunked[1]) < 1e-12 * abs(full[1])
    assert abs(full[2] - chunked[2]) < 1e-12 * abs(full[2])
    assert np.abs(full[3] - chunked[3]).max() < 1e-12 * np.abs(full[3]).max()


def test_full_size_gradient_vs_central_differences():
    """Differentiation workload at full size (1024^2, 16 pairs, 4096 lookups):
    adjoint vs central differences of the GPU FP64 forward (relative 1e-6)."""
    _say("adjoint full size 1024^2")
    from paper_1404_7357_amd import LookupFunction, TableFunction, Tabulator
    from workloads import c5_gradient
    wl = c5_gradient()
    gd, sub = wl.grids[0], wl.substrates[0]
    tab = Tabulator(gd, wl.basis, max_mbf=wl.M)
    pairs = [tuple(int(v) for v in p) for p in wl.pairs]
    pts = torch.tensor(wl.queries, device="cuda")
    # target: the table at eps_r 2.3 and perturbed coefficients, through the same path
    with torch.no_grad():
        zt = LookupFunction.apply(
            TableFunction.apply(torch.tensor(wl.target_eps_r, dtype=torch.float64, device="cuda"),
                                torch.tensor(sub.h, dtype=torch.float64, device="cuda"),
                                torch.tensor(wl.target_q, device="cuda"), tab, sub.tan_delta, pairs, 0),
            pts, tab, 0)

    def loss_of(e, h, q, grad):
        ee = torch.tensor(e, dtype=torch.float64, device="cuda", requires_grad=grad)
        hh = torch.tensor(h, dtype=torch.float64, device="cuda", requires_grad=grad)
        qq = torch.tensor(q, device="cuda", requires_grad=grad)
        v = LookupFunction.apply(TableFunction.apply(ee, hh, qq, tab, sub.tan_delta, pairs, 0), pts, tab, 0)
        loss = (v - zt).abs().pow(2).sum()
        if not grad:
            return float(loss.item())
        loss.backward()
        return float(loss.item()), float(ee.grad.item()), float(hh.grad.item()), qq.grad.cpu().numpy()

    _, de, dh, dq = loss_of(sub.eps_r, sub.h, wl.q, True)
    step = 1e-6
    fd_e = (loss_of(sub.eps_r + step, sub.h, wl.q, False) - loss_of(sub.eps_r - step, sub.h, wl.q, False)) / (2 * step)
    fd_h = (loss_of(sub.eps_r, sub.h + step, wl.q, False) - loss_of(sub.eps_r, sub.h - step, wl.q, False)) / (2 * step)
    assert abs(de - fd_e) < 1e-6 * abs(fd_e), (de, fd_e)
    assert abs(dh - fd_h) < 1e-6 * abs(fd_h), (dh, fd_h)
    rng = np.random.default_rng(17)
    for _ in range(3):
        m, j = int(rng.integers(wl.M)), int(rng.integers(wl.B))
        d = np.zeros_like(wl.q)
        d[m, j] = step
        fr = (loss_of(sub.eps_r, sub.h, wl.q + d, False) - loss_of(sub.eps_r, sub.h, wl.q - d, False)) / (2 * step)
        fi = (loss_of(sub.eps_r, sub.h, wl.q + 1j * d, False) - loss_of(sub.eps_r, sub.h, wl.q - 1j * d, False)) / (2 * step)
        assert abs(dq[m, j] - (fr + 1j * fi)) < 1e-6 * np.abs(dq).max(), (m, j)
    tab.close()


def test_second_order_lookup_adjoint_is_the_transpose():
    """<dout, L z> = <L^T dout, z> for the second-order lookup L (random
    table and cotangent), with points on the table edges and outside."""
    _say("second-order lookup adjoint identity")
    from paper_1404_7357_amd import Tabulator
    rng = np.random.default_rng(61)
    grid = Grid(64, 32, 8 * K0, 6 * K0, K0)
    tab = Tabulator(grid, rooftop_lattice(1, 1), 1)
    z = torch.tensor(rng.standard_normal((3, 32, 64)) + 1j * rng.standard_normal((3, 32, 64)), device="cuda")
    dxa = co.displacement_axis(64, grid.kx_max)
    dya = co.displacement_axis(32, grid.ky_max)
    pts = np.stack([rng.uniform(dxa[0], dxa[-1], 300), rng.uniform(dya[0], dya[-1], 300)], 1)
    pts = np.concatenate([pts, [[dxa[0], dya[0]], [dxa[-1], dya[-1]], [dxa[-1] + 1.0, 0.0]]])
    p = torch.tensor(pts, device="cuda")
    dout = torch.tensor(rng.standard_normal((3, len(pts))) + 1j * rng.standard_normal((3, len(pts))), device="cuda")
    dout[:, -1] = 0                                   # the outside point has no value to weigh
    from paper_1404_7357_amd import cfft_lookup_quadratic_backward
    v = tab.lookup(z, p, order=2)
    dz = torch.zeros_like(z)
    cfft_lookup_quadratic_backward(tab.plan, 0, dout, 3, p, dz)
    torch.cuda.synchronize()
    tab.close()
    lhs = torch.sum(torch.conj(dout[:, :-1]) * v[:, :-1]).item()
    rhs = torch.sum(torch.conj(dz) * z).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_refined_second_order_gradient_vs_oracle_and_differences():
    """The paper's table use made differentiable: a x2 zero-padded grid read
    by second-order lookups; the gradient (band samples only) against the
    oracle's and central differences of the GPU forward."""
    import dataclasses
    _say("adjoint refined grid + second-order lookups")
    rng = np.random.default_rng(67)
    base = Grid(32, 32, 6 * K0, 6 * K0, K0)
    grid = dataclasses.replace(base, nx=64, ny=64, kx_max=12 * K0, ky_max=12 * K0, zero_pad=1)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = [(0, 0), (0, 1), (1, 0), (1, 1)]
    dxa = co.displacement_axis(64, grid.kx_max)
    pts = rng.uniform(dxa[1], dxa[-2], (24, 2))
    qt = q + 0.1 * gaussian_coefficients(rng, 2, basis.shape[0])
    zt = co.lookup_direct(grid, Substrate(2.3, 0.0, 0.05), basis, qt, np.array(pairs), pts, order=2)
    loss, de, dh, dq = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt, order=2)
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, zt, order=2)
    assert abs(loss - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * abs(o_de), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * abs(o_dh), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()
    step = 1e-6

    def L(**kw):
        return _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt, need_grad=False, order=2, **kw)[0]
    fd_h = (L(h=sub.h + step) - L(h=sub.h - step)) / (2 * step)
    assert abs(dh - fd_h) < 1e-6 * abs(fd_h), (dh, fd_h)


def test_fill_adjoint_is_the_transpose():
    """<dout, F z> = <F^T dout, z> for the reduced-matrix fill F, orders 1 and
    2, with self blocks, unlisted pairs and displacements outside the table."""
    _say("fill adjoint identity")
    from paper_1404_7357_amd import Tabulator, cfft_fill_backward
    rng = np.random.default_rng(71)
    grid = Grid(64, 32, 8 * K0, 6 * K0, K0)
    tab = Tabulator(grid, rooftop_lattice(1, 1), 3)
    pairs = [(0, 0), (0, 2), (1, 1), (2, 1)]
    z = torch.tensor(rng.standard_normal((4, 32, 64)) + 1j * rng.standard_normal((4, 32, 64)), device="cuda")
    pos = torch.tensor(rng.uniform([-1.1, -0.75], [1.1, 0.75], (23, 2)), device="cuda")
    am = 23 * 3
    for order in (1, 2):
        fz = torch.zeros((am, am), dtype=torch.complex128, device="cuda")
        tab.fill(z, pairs, 3, pos, order=order, out=fz)
        dout = torch.tensor(rng.standard_normal((am, am)) + 1j * rng.standard_normal((am, am)), device="cuda")
        outside = torch.isnan(fz)
        assert 0 < int(outside.sum().item()) < am * am // 4
        fz[outside] = 0
        dz = torch.zeros_like(z)
        cfft_fill_backward(tab.plan, 0, dout, pairs, 3, pos, order, dz)
        torch.cuda.synchronize()
        lhs = torch.sum(torch.conj(dout) * fz).item()
        rhs = torch.sum(torch.conj(dz) * z).item()
        assert abs(lhs - rhs) < 1e-12 * abs(lhs), (order, lhs, rhs)
    tab.close()


def test_fill_loss_gradient_vs_oracle():
    """A loss over the reduced matrix of a layout filled from a refined table
    (second-order interpolation): its gradient equals the oracle's gradient
    of the same loss written as lookups at the layout's displacements."""
    import dataclasses
    _say("fill loss gradient vs oracle")
    from paper_1404_7357_amd import FLAG_ZERO_PAD2, FillFunction, TableFunction, Tabulator
    rng = np.random.default_rng(73)
    base = Grid(32, 32, 6 * K0, 6 * K0, K0)
    grid = dataclasses.replace(base, nx=64, ny=64, kx_max=12 * K0, ky_max=12 * K0, zero_pad=1)
    sub = Substrate(2.2, 0.0, 0.05)
    basis = rooftop_lattice(2, 3)
    q = gaussian_coefficients(rng, 2, basis.shape[0])
    pairs = [(0, 0), (0, 1), (1, 1)]
    nel, nmbf = 5, 2
    lay = rng.uniform(-0.35, 0.35, (nel, 2))
    ii, jj = np.nonzero(~np.eye(nel, dtype=bool))
    target = rng.standard_normal((len(pairs), len(ii))) + 1j * rng.standard_normal((len(pairs), len(ii)))
    tmat = np.zeros((nel * nmbf, nel * nmbf), dtype=np.complex128)
    for p, (m, n) in enumerate(pairs):
        tmat[ii * nmbf + m, jj * nmbf + n] = target[p] * 1e-9
    tab = Tabulator(grid, basis, max_mbf=2, flags=FLAG_ZERO_PAD2)
    e = torch.tensor(sub.eps_r, dtype=torch.float64, device="cuda", requires_grad=True)
    hh = torch.tensor(sub.h, dtype=torch.float64, device="cuda", requires_grad=True)
    qq = torch.tensor(q, device="cuda", requires_grad=True)
    z = TableFunction.apply(e, hh, qq, tab, sub.tan_delta, pairs, 0)
    mat = FillFunction.apply(z, torch.tensor(lay, device="cuda"), tab, pairs, nmbf, 2, 0)
    written = torch.zeros_like(mat, dtype=torch.bool)
    for m, n in pairs:
        written[torch.tensor(ii * nmbf + m), torch.tensor(jj * nmbf + n)] = True
    loss = ((mat - torch.tensor(tmat, device="cuda")).abs().pow(2) * written).sum()
    loss.backward()
    de, dh, dq = float(e.grad.item()), float(hh.grad.item()), qq.grad.cpu().numpy()
    tab.close()
    pts = lay[ii] - lay[jj]
    o_loss, o_de, o_dh, o_dq = co.loss_gradient(grid, sub, basis, q, np.array(pairs), pts, target * 1e-9, order=2)
    assert abs(float(loss.item()) - o_loss) < 1e-9 * abs(o_loss)
    assert abs(de - o_de) < 1e-9 * abs(o_de), (de, o_de)
    assert abs(dh - o_dh) < 1e-9 * abs(o_dh), (dh, o_dh)
    assert np.abs(dq - o_dq).max() < 1e-9 * np.abs(o_dq).max()


def _clustered_points(rng, grid, count):
    """Points packed into a few table cells (many share a cell), plus some
    spread over the table, on its edges and outside it."""
    dxa = co.displacement_axis(grid.nx, grid.kx_max)
    dya = co.displacement_axis(grid.ny, grid.ky_max)
    cx, cy = dxa[grid.nx // 3], dya[grid.ny // 2]
    dd = dxa[1] - dxa[0]
    tight = np.stack([cx + rng.uniform(0, 2.5 * dd, count), cy + rng.uniform(0, 2.5 * dd, count)], 1)
    spread = np.stack([rng.uniform(dxa[0], dxa[-1], count // 4), rng.uniform(dya[0], dya[-1], count // 4)], 1)
    edges = [[dxa[0], dya[0]], [dxa[-1], dya[-1]], [dxa[-2], dya[0]], [dxa[-1] + 1.0, 0.0]]
    return np.concatenate([tight, spread, edges])


def test_interpolation_adjoints_are_deterministic():
    """The bilinear and second-order lookup adjoints and the fill adjoint give
    the same bits on every run (sorted per-cell sums, no atomics), with
    thousands of points sharing a few cells; the bilinear adjoint is the
    transpose of the lookup."""
    _say("interpolation adjoints: run-twice determinism")
    from paper_1404_7357_amd import Tabulator, cfft_fill_backward, cfft_lookup_backward, cfft_lookup_quadratic_backward
    rng = np.random.default_rng(91)
    grid = Grid(64, 32, 8 * K0, 6 * K0, K0)
    tab = Tabulator(grid, rooftop_lattice(1, 1), 3)
    pts = _clustered_points(rng, grid, 6000)
    p = torch.tensor(pts, device="cuda")
    dout = torch.tensor(rng.standard_normal((3, len(pts))) + 1j * rng.standard_normal((3, len(pts))), device="cuda")
    for name, fn in (("bilinear", cfft_lookup_backward), ("second order", cfft_lookup_quadratic_backward)):
        runs = []
        for _ in range(3):
            dz = torch.zeros((3, 32, 64), dtype=torch.complex128, device="cuda")
            fn(tab.plan, 0, dout, 3, p, dz)
            torch.cuda.synchronize()
            runs.append(dz.cpu())
        assert torch.equal(runs[0], runs[1]) and torch.equal(runs[0], runs[2]), name
        assert float(runs[0].abs().max()) > 0
    # bilinear transpose identity <dout, L z> = <L^T dout, z> on the same points
    z = torch.tensor(rng.standard_normal((3, 32, 64)) + 1j * rng.standard_normal((3, 32, 64)), device="cuda")
    v = tab.lookup(z, p)
    inside = ~torch.isnan(v[0])
    dz = torch.zeros_like(z)
    cfft_lookup_backward(tab.plan, 0, dout, 3, p, dz)
    lhs = torch.sum(torch.conj(dout[:, inside]) * v[:, inside]).item()
    rhs = torch.sum(torch.conj(dz) * z).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # fill adjoint: a layout with many repeated displacements
    pos = torch.tensor(rng.integers(-3, 4, (60, 2)) * 0.21 + rng.uniform(0, 1e-3, (60, 2)), device="cuda")
    pairs = [(0, 0), (0, 2), (1, 1), (2, 1)]
    am = 60 * 3
    doutf = torch.tensor(rng.standard_normal((am, am)) + 1j * rng.standard_normal((am, am)), device="cuda")
    for order in (1, 2):
        runs = []
        for _ in range(3):
            dz = torch.zeros((4, 32, 64), dtype=torch.complex128, device="cuda")
            cfft_fill_backward(tab.plan, 0, doutf, pairs, 3, pos, order, dz)
            torch.cuda.synchronize()
            runs.append(dz.cpu())
        assert torch.equal(runs[0], runs[1]) and torch.equal(runs[0], runs[2]), order
    tab.close()


def test_backward_is_deterministic():
    """The whole adjoint (lookup adjoint, adjoint passes, integrand, Green's
    function and spectra adjoints) run twice gives identical gradients."""
    _say("backward run-twice determinism")
    grid, sub, basis, q, pairs, pts, zt = _problem(n=128, m=3, npts=512)
    a = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    b = _gpu_loss_and_grad(grid, sub, basis, q, pairs, pts, zt)
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]
    assert np.array_equal(a[3], b[3])


def test_backward_rejects_a_spectra_adjoint_beyond_lds():
    """A basis set with 600 distinct x-centres and 4 MBFs needs 76.8 kB of LDS
    in the spectra adjoint: cfft_backward refuses it on the host, before any
    adjoint kernel runs, and leaves the gradient buffers untouched."""
    _say("backward LDS limit")
    from paper_1404_7357_amd import CfftError, Tabulator, cfft_backward
    from workloads import ROOFTOP_X, basis_array
    rng = np.random.default_rng(5)
    basis = basis_array([(ROOFTOP_X, -0.3 + 0.001 * i, 0.0, 0.01, 0.02) for i in range(600)])
    grid = Grid(32, 32, 6 * K0, 6 * K0, K0)
    tab = Tabulator(grid, basis, max_mbf=4)
    q = torch.tensor(gaussian_coefficients(rng, 4, 600), device="cuda")
    g = tab.green(2.2, 0.0, 0.05)
    spec = tab.spectra(q)
    pairs = [(0, 1), (2, 3)]
    z = tab.tabulate(spec, g, pairs)
    dz = torch.ones_like(z)
    grad_sub = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    grad_q = torch.full_like(q, 7.0)
    with pytest.raises(CfftError) as ei:
        cfft_backward(tab.plan, 0, dz, 2.2, 0.0, 0.05, tab.basis, q, pairs, g, spec, grad_sub, grad_q)
    assert "UNSUPPORTED" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((grad_sub == 7.0).all()) and bool((grad_q == 7.0).all())
    tab.close()
