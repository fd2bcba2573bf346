"""Frequency sweep with uneven grids (256^2, 512^2, 1024^2) in one plan,
replayed as one captured HIP graph, and the large 4096^2 launch
configuration, against the oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import cfft_oracle as co
from tolerances import FP64_TARGET, MIXED_TARGET
from workloads import (FP64, MIXED, Grid, c3_frequency_sweep, c4_large, gaussian_coefficients, random_smooth_field,
                       rooftop_lattice)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K0 = 2 * math.pi


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _sweep_calls(tab, wl, q, bufs):
    """The grids' chains (Green's function, spectra, table) one after the
    other on the current stream, through one plan holding all 8 grids."""
    pairs = [tuple(int(v) for v in p) for p in wl.pairs]
    for i, (gd, sub) in enumerate(zip(wl.grids, wl.substrates)):
        g, spec, z = bufs[i]
        tab.green(sub.eps_r, sub.tan_delta, sub.h, grid=i, out=g)
        tab.spectra(q, grid=i, out=spec)
        tab.tabulate(spec, g, pairs, grid=i, out=z)


def _sweep_buffers(wl):
    bufs = []
    for gd in wl.grids:
        dt = torch.complex128 if gd.precision == FP64 else torch.complex64
        bufs.append((torch.empty((3, gd.ny, gd.nx), dtype=torch.complex128, device="cuda"),
                     torch.empty((wl.M, 4, gd.ny, gd.nx), dtype=dt, device="cuda"),
                     torch.empty((len(wl.pairs), gd.ny, gd.nx), dtype=dt, device="cuda")))
    return bufs


def test_sweep_graph_replays_match_eager_and_oracle():
    """The frequency sweep through one plan holding all 8 grids, with
    autotuned schedules (tuned by the first eager calls, then captured, lanes
    included), replayed as one HIP graph: every replay equals the eager
    tables, and all 8 grids match the oracle at sampled outputs at the mixed
    bar."""
    from paper_1404_7357_amd import FLAG_AUTOTUNE, Tabulator
    wl = c3_frequency_sweep()
    _say("c3 sweep eager")
    tab = Tabulator(wl.grids, wl.basis, max_mbf=wl.M, flags=FLAG_AUTOTUNE)
    q = torch.tensor(wl.q, device="cuda")
    bufs = _sweep_buffers(wl)
    _sweep_calls(tab, wl, q, bufs)
    torch.cuda.synchronize()
    eager = [b[2].cpu().clone() for b in bufs]
    _say("c3 sweep graph capture")
    graph = torch.cuda.CUDAGraph()
    gbufs = _sweep_buffers(wl)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        _sweep_calls(tab, wl, q, gbufs)      # warm on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        _sweep_calls(tab, wl, q, gbufs)
    for rep in range(3):
        for b in gbufs:
            b[2].zero_()
        graph.replay()
        torch.cuda.synchronize()
        for i in range(len(wl.grids)):
            assert torch.equal(gbufs[i][2].cpu(), eager[i]), (rep, i)
        # eager work between replays
        _sweep_calls(tab, wl, q, bufs)
        torch.cuda.synchronize()
    tab.close()
    _say("c3 sweep oracle samples (8 grids)")
    rng = np.random.default_rng(9)
    for i in range(len(wl.grids)):
        gd, sub = wl.grids[i], wl.substrates[i]
        idx = np.unique(np.concatenate([rng.choice(gd.nx * gd.ny, 12, replace=False),
                                        [(gd.ny // 2) * gd.nx + gd.nx // 2, 0, gd.nx * gd.ny - 1]]))
        ref = co.tabulate(gd, sub, wl.basis, wl.q, wl.pairs, out_idx=idx, workers=8)
        got = eager[i].numpy().reshape(len(wl.pairs), -1)[:, idx]
        err = (np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max()
        _say(f"c3 grid {i} ({gd.nx}^2) err={err:.3e}")
        assert err < MIXED_TARGET, (i, err)


def _sample_points(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(nx * ny, count, replace=False).tolist())
    idx |= {(ny // 2) * nx + nx // 2, 0, nx * ny - 1}
    return np.array(sorted(idx))


def test_large_green_and_spectra_sampled():
    """4096^2 with the high-contrast slab and B = 1024, M = 6: sampled samples vs oracle."""
    from paper_1404_7357_amd import Tabulator
    wl = c4_large(precision=FP64)
    gd, sub = wl.grids[0], wl.substrates[0]
    _say("c4 4096^2 green + spectra")
    tab = Tabulator(gd, wl.basis, max_mbf=wl.M)
    g = tab.green(sub.eps_r, sub.tan_delta, sub.h).reshape(3, -1)
    spec = tab.spectra(torch.tensor(wl.q, device="cuda")).reshape(wl.M, 4, -1)
    idx = _sample_points(gd.nx, gd.ny, 2000, 5)
    it = torch.tensor(idx, device="cuda")
    gs = g[:, it].cpu().numpy()
    ss = spec[:, :, it].cpu().numpy()
    tab.close()
    kx, ky = co.grid_samples(gd.nx, gd.ny, gd.kx_max, gd.ky_max)
    kx, ky = kx[idx], ky[idx]
    ref_g = np.stack(co.green_remainder(kx, ky, gd.gamma, gd.k0, sub.eps_r, sub.tan_delta, sub.h))
    assert np.abs(gs - ref_g).max() < 1e-12 * np.abs(ref_g).max()
    kcx, kcy, _ = co.ray_contour(kx, ky, gd.gamma)
    mt, mh = co.mbf_spectra(wl.basis, wl.q, kcx, kcy)
    ref_s = np.concatenate([mt, mh], axis=1)
    assert np.abs(ss - ref_s).max() < 1e-12 * np.abs(ref_s).max()


@pytest.mark.parametrize("prec", [FP64, MIXED])
def test_large_table_sampled(prec):
    """4096^2 tabulation of all 36 pairs (the large launch configuration) from
    seeded Green's-function and spectra arrays; sampled outputs of 4 pairs vs
    the oracle's direct sum of the same integrands."""
    from paper_1404_7357_amd import Tabulator
    n, m = 4096, 6
    gd = Grid(n, n, math.pi * n / 200.0, math.pi * n / 200.0, K0, precision=prec)
    rng = np.random.default_rng(77)
    # smooth, decaying synthetic factors (spectra and Green's function of no
    # particular antenna): Gaussian envelope times seeded noise
    kx, ky = co.grid_samples(n, n, gd.kx_max, gd.ky_max)
    env = np.exp(-0.5 * (kx ** 2 + ky ** 2) / (3 * K0) ** 2)
    _say(f"c4 table prec={prec}: building inputs")
    g = np.stack([env * random_smooth_field(rng, n * n) for _ in range(3)])
    spec = np.stack([np.stack([env * random_smooth_field(rng, n * n) for _ in range(4)]) for _ in range(m)])
    tab = Tabulator(gd, rooftop_lattice(1, 1), max_mbf=m)
    pairs = [(a, b) for a in range(m) for b in range(m)]
    _say(f"c4 table prec={prec}: gpu")
    sdt = torch.complex128 if prec == FP64 else torch.complex64
    z = tab.tabulate(torch.tensor(spec.reshape(m, 4, n, n), device="cuda").to(sdt),
                     torch.tensor(g.reshape(3, n, n), device="cuda"), pairs)
    torch.cuda.synchronize()
    check = [0, 7, 20, 35]
    idx = _sample_points(n, n, 12, 13)
    it = torch.tensor(idx, device="cuda")
    got = z.reshape(len(pairs), -1)[:, it][check].cpu().numpy().astype(np.complex128)
    tab.close()
    del z
    _say(f"c4 table prec={prec}: oracle")
    sel = [pairs[p] for p in check]
    mt = spec[:, 0:2]
    mh = spec[:, 2:4]
    ref = co.tabulate_from_factors(gd, sel, tuple(g), mt, mh, out_idx=idx, workers=8)
    scale = np.abs(ref).max(axis=1)
    err = (np.abs(got - ref).max(axis=1) / scale).max()
    tol = FP64_TARGET if prec == FP64 else MIXED_TARGET
    print(f"[gpu-case] c4 table prec={prec} err={err:.3e}", flush=True)
    assert err < tol, err


def test_large_lookup_1e5_points():
    """Bilinear lookup of 36 tables of 4096^2 (complex64) at the 10^5 query points of
    the large workload, against the oracle's bilinear interpolation."""
    from paper_1404_7357_amd import Tabulator
    wl = c4_large()
    gd = wl.grids[0]
    _say("c4 lookup 1e5 points")
    tab = Tabulator(gd, rooftop_lattice(1, 1), max_mbf=6)
    z = torch.complex(torch.randn((36, gd.ny, gd.nx), device="cuda", dtype=torch.float32,
                                  generator=torch.Generator(device="cuda").manual_seed(5)),
                      torch.randn((36, gd.ny, gd.nx), device="cuda", dtype=torch.float32,
                                  generator=torch.Generator(device="cuda").manual_seed(6)))
    pts = torch.tensor(wl.queries, device="cuda")
    out = tab.lookup(z, pts).cpu().numpy()
    sel = [0, 17, 35]
    zc = z[sel].cpu().numpy().astype(np.complex128)
    tab.close()
    ref = co.bilinear_lookup(gd, zc, wl.queries)
    assert np.abs(out[sel] - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.isfinite(out).all()
