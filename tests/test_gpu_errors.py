"""Error paths of the C ABI that need a device: an allocation the device
refuses (forced from the host with the CFFT_TEST_FAIL_ALLOC hook) is reported
as CFFT_ERR_ALLOC, by plan creation and by a call that must grow the plan's
workspace, and the plan stays usable afterwards."""
import math

import numpy as np
import pytest

from workloads import Grid, Substrate, gaussian_coefficients, rooftop_lattice

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K0 = 2 * math.pi


def test_refused_allocation_reports_alloc(monkeypatch):
    from paper_1404_7357_amd import CfftError, Tabulator
    print("[gpu-case] refused allocation", flush=True)
    grid = Grid(64, 64, 8 * K0, 8 * K0, K0)
    basis = rooftop_lattice(2, 3)
    monkeypatch.setenv("CFFT_TEST_FAIL_ALLOC", "1")
    with pytest.raises(CfftError) as ei:
        Tabulator(grid, basis, max_mbf=2)
    assert "ALLOC" in str(ei.value)
    monkeypatch.delenv("CFFT_TEST_FAIL_ALLOC")
    tab = Tabulator(grid, basis, max_mbf=2)
    q = torch.tensor(gaussian_coefficients(np.random.default_rng(3), 2, basis.shape[0]), device="cuda")
    sub = Substrate(2.2, 0.0, 0.05)
    g = tab.green(sub.eps_r, sub.tan_delta, sub.h)
    spec = tab.spectra(q)
    # the first tabulate must allocate the pass workspace: refused
    monkeypatch.setenv("CFFT_TEST_FAIL_ALLOC", "1")
    with pytest.raises(CfftError) as ei:
        tab.tabulate(spec, g, [(0, 1)])
    assert "ALLOC" in str(ei.value)
    monkeypatch.delenv("CFFT_TEST_FAIL_ALLOC")
    z = tab.tabulate(spec, g, [(0, 1)])
    torch.cuda.synchronize()
    assert bool(torch.isfinite(z).all())
    tab.close()
