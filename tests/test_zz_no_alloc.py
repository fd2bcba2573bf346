"""The allocation-free entry point cfft_tabulate_noalloc against cfft_tabulate,
through the C ABI: two calls in a row on one plan (the second on a smaller
grid, with fewer pairs), each compared with cfft_tabulate on the same inputs;
the device's free memory is unchanged by the calls; a grid whose
intermediates exceed the fixed scratch is rejected before any launch."""
import math

import numpy as np
import pytest

from workloads import FP64, MIXED, Grid, gaussian_coefficients, rooftop_lattice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K0 = 2 * math.pi


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _inputs(tab, grid_i, gd, q, sub):
    g = tab.green(sub[0], sub[1], sub[2], grid=grid_i)
    spec = tab.spectra(q, grid=grid_i)
    return g, spec


def test_noalloc_matches_tabulate_on_two_calls():
    from paper_1404_7357_amd import Tabulator, _lib
    basis = rooftop_lattice(4, 6)
    rng = np.random.default_rng(404)
    q = torch.tensor(gaussian_coefficients(rng, 4, basis.shape[0]), device="cuda")
    grids = [Grid(512, 512, 10 * K0, 10 * K0, K0, precision=FP64),      # 16.8 MB per pair: two chunks of 15 + 1
             Grid(128, 64, 8 * K0, 6 * K0, K0, precision=MIXED)]
    tab = Tabulator(grids, basis, max_mbf=4)
    sub = (4.4, 0.002, 0.06)
    calls = [(0, [(m, n) for m in range(4) for n in range(4)]), (1, [(2, 1), (0, 3), (3, 3)])]
    outs = []
    # inputs and outputs of both calls allocated before measuring free memory
    for gi, pairs in calls:
        gd = grids[gi]
        g, spec = _inputs(tab, gi, gd, q, sub)
        dt = torch.complex128 if gd.precision == FP64 else torch.complex64
        z_ref = tab.tabulate(spec, g, pairs, grid=gi)
        z_na = torch.full_like(z_ref, complex(float("nan"), float("nan")))
        outs.append((gi, pairs, g, spec, z_ref, z_na, dt))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for gi, pairs, g, spec, z_ref, z_na, dt in outs:
        _say(f"noalloc grid {gi} {grids[gi].nx}x{grids[gi].ny} pairs={len(pairs)}")
        _lib.cfft_tabulate_noalloc(tab.plan, gi, spec, spec.shape[0], g, pairs, z_na)
        torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    for gi, pairs, g, spec, z_ref, z_na, dt in outs:
        a = z_na.cpu().numpy()
        b = z_ref.cpu().numpy()
        assert np.isfinite(a).all()
        err = float(np.abs(a - b).max() / np.abs(b).max())
        _say(f"noalloc grid {gi} err vs cfft_tabulate {err:.3e}")
        assert err == 0.0, err
    tab.close()


def test_noalloc_rejects_grids_beyond_the_scratch():
    from paper_1404_7357_amd import CfftError, Tabulator, _lib
    basis = rooftop_lattice(1, 1)
    gd = Grid(4096, 4096, 10 * K0, 10 * K0, K0, precision=FP64)     # 1 GiB of intermediates per pair
    tab = Tabulator(gd, basis, max_mbf=1)
    # full-size buffers: the call must fail on the host, but nothing it could
    # launch would reach outside them
    spec = torch.zeros((1, 4, gd.ny, gd.nx), dtype=torch.complex128, device="cuda")
    g = torch.zeros((3, gd.ny, gd.nx), dtype=torch.complex128, device="cuda")
    z = torch.zeros((1, gd.ny, gd.nx), dtype=torch.complex128, device="cuda")
    with pytest.raises(CfftError) as ei:
        _lib.cfft_tabulate_noalloc(tab.plan, 0, spec, 1, g, [(0, 0)], z)
    assert "UNSUPPORTED" in str(ei.value) and "allocation-free" in str(ei.value)
    tab.close()
