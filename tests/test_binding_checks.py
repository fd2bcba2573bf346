"""Host-side buffer checks of the Python binding: a caller mistake in a
table, coefficient, query or layout tensor (wrong dtype, shape, device or
memory layout) raises ValueError before anything reaches the library, so it
can never become an out-of-bounds device access.  Runs without a GPU: the
Tabulator is built without a plan, so a check that let a bad buffer through
would reach the C ABI with a NULL plan and raise CfftError instead."""
import math

import pytest

torch = pytest.importorskip("torch")


def _tab(precision):
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(root, "paper_1404_7357_amd", "libcfft.so")):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1404_7357_amd import Tabulator, _lib
    from workloads import Grid, rooftop_lattice
    tab = Tabulator.__new__(Tabulator)
    tab.grids = [Grid(64, 32, 30.0, 30.0, 2 * math.pi, precision=precision)]
    tab.plan = _lib.Plan.__new__(_lib.Plan)
    tab.plan.handle = None
    tab.basis = _lib.basis_array(rooftop_lattice(2, 3))
    tab.nbasis = len(tab.basis)
    tab.device = torch.device("cuda")
    return tab


def _raises(fn, *words):
    with pytest.raises(ValueError) as ei:
        fn()
    for w in words:
        assert w in str(ei.value), str(ei.value)


@pytest.mark.parametrize("precision", [0, 1])
def test_lookup_rejects_bad_tables(precision):
    tab = _tab(precision)
    want = "complex128" if precision == 0 else "complex64"
    other = torch.complex64 if precision == 0 else torch.complex128
    pts = torch.zeros((5, 2), dtype=torch.float64)
    # wrong precision for the grid (would read 16-byte elements from an 8-byte table or vice versa)
    _raises(lambda: tab.lookup(torch.zeros((3, 32, 64), dtype=other), pts), "z", want)
    # smaller table than the grid
    _raises(lambda: tab.lookup(torch.zeros((3, 16, 64), dtype=other), pts), "z", "(3, 32, 64)")
    # a 2-d tensor is not a table
    _raises(lambda: tab.lookup(torch.zeros((32, 64), dtype=other), pts), "z")
    # host memory (the kernels would dereference a host pointer)
    good_dtype = torch.complex128 if precision == 0 else torch.complex64
    _raises(lambda: tab.lookup(torch.zeros((3, 32, 64), dtype=good_dtype), pts), "z", "cuda")
    _raises(lambda: tab.lookup(torch.zeros((3, 32, 64), dtype=good_dtype), pts, order=2), "z", "cuda")


@pytest.mark.parametrize("precision", [0, 1])
def test_fill_rejects_bad_tables(precision):
    tab = _tab(precision)
    want = "complex128" if precision == 0 else "complex64"
    other = torch.complex64 if precision == 0 else torch.complex128
    pos = torch.zeros((4, 2), dtype=torch.float64)
    _raises(lambda: tab.fill(torch.zeros((1, 32, 64), dtype=other), [(0, 0)], 1, pos,
                             out=torch.zeros((4, 4), dtype=torch.complex128)), "z", want)
    _raises(lambda: tab.fill(torch.zeros((1, 32, 32), dtype=other), [(0, 0)], 1, pos,
                             out=torch.zeros((4, 4), dtype=torch.complex128)), "z")


def test_spectra_rejects_bad_coefficients():
    tab = _tab(0)
    nb = tab.nbasis
    # host coefficients: the spectra kernel would read a host pointer
    _raises(lambda: tab.spectra(torch.zeros((2, nb), dtype=torch.complex128)), "q", "cuda")
    # wrong dtype and wrong basis count
    _raises(lambda: tab.spectra(torch.zeros((2, nb), dtype=torch.complex64)), "q", "complex128")
    _raises(lambda: tab.spectra(torch.zeros((2, nb + 1), dtype=torch.complex128)), "q")
    _raises(lambda: tab.spectra(torch.zeros((nb,), dtype=torch.complex128)), "q")


def test_non_contiguous_buffers_are_rejected():
    from paper_1404_7357_amd import _check_buffer
    t = torch.zeros((4, 6), dtype=torch.float64).t()
    _raises(lambda: _check_buffer(t, (6, 4), torch.float64, "t"), "contiguous")
