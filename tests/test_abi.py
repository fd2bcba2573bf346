"""Host-side checks of the C ABI: the library loads, exports every entry point
declared in include/cfft.h, and rejects bad arguments before touching a device.
No compute call is made here (this suite runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfft.h")


def _lib():
    import torch  # noqa: F401  (binds the library to torch's HIP runtime)
    if not os.path.exists(os.path.join(ROOT, "paper_1404_7357_amd", "libcfft.so")):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1404_7357_amd import _lib as L
    return L, L.load()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:cfft_status_t|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    names = _declared()
    assert {"c_fft_plan", "mbf_spectra", "slab_green_eval", "cfft_tabulate", "cfft_backward"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.ENTRY_POINTS) == set(names)


def test_struct_layouts_match_header():
    L, _ = _lib()
    assert ctypes.sizeof(L.GridDesc) == 64
    assert ctypes.sizeof(L.Basis) == 40
    assert L.GridDesc.precision.offset == 56 and L.GridDesc.beta_end.offset == 48
    assert L.GridDesc.truncation.offset == 60
    from workloads import BASIS_DTYPE
    assert BASIS_DTYPE.itemsize == 40


def _grid(**kw):
    from workloads import Grid
    g = Grid(64, 64, 50.0, 50.0, 6.283185307179586)
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("field,value", [("nx", 48), ("ny", 8), ("nx", 8192), ("gamma", 0.0), ("gamma", -1.0),
                                         ("order", -1), ("order", 8), ("kx_max", 0.0), ("k0", float("nan")),
                                         ("precision", 7), ("contour", 9), ("truncation", 2), ("truncation", -1)])
def test_plan_rejects_invalid_grids(field, value):
    L, lib = _lib()
    desc = (L.GridDesc * 1)(L.grid_desc(_grid(**{field: value})))
    h = ctypes.c_void_p()
    st = lib.c_fft_plan(desc, 1, 4, 0, ctypes.byref(h))
    assert st == 1, (field, value, st)
    assert lib.cfft_last_error().decode()
    assert not h.value


def test_plan_checks_parabolic_contour_arguments():
    """The parabolic contour needs a finite beta_end > 0 (INVALID_ARG) and
    excludes the tensor-product truncation (UNSUPPORTED); both are caught on
    the host before any device call."""
    L, lib = _lib()
    h = ctypes.c_void_p()
    for bad in (0.0, -1.0, float("inf")):
        desc = (L.GridDesc * 1)(L.grid_desc(_grid(contour=1, beta_end=bad)))
        assert lib.c_fft_plan(desc, 1, 4, 0, ctypes.byref(h)) == 1
    desc = (L.GridDesc * 1)(L.grid_desc(_grid(contour=1, beta_end=20.0, truncation=1)))
    assert lib.c_fft_plan(desc, 1, 4, 0, ctypes.byref(h)) == 2


def test_plan_argument_checks():
    L, lib = _lib()
    desc = (L.GridDesc * 1)(L.grid_desc(_grid()))
    h = ctypes.c_void_p()
    assert lib.c_fft_plan(None, 1, 4, 0, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 0, 4, 0, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 1, 0, 0, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 1, 17, 0, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 1, 4, 0x100, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 1, 4, 8, ctypes.byref(h)) == 1
    assert lib.c_fft_plan(desc, 1, 4, 0, None) == 1


def test_calls_on_unknown_plan_are_rejected():
    L, lib = _lib()
    bogus = ctypes.c_void_p(0x1234)
    assert lib.slab_green_eval(None, 0, 2.2, 0.0, 0.05, ctypes.c_void_p(8), None) == 1
    assert lib.slab_green_eval(bogus, 0, 2.2, 0.0, 0.05, ctypes.c_void_p(8), None) == 1
    assert "destroyed" in lib.cfft_last_error().decode() or "unknown" in lib.cfft_last_error().decode()
    assert lib.c_fft_plan_destroy(None) == 0
    assert lib.c_fft_plan_destroy(bogus) == 1


def test_every_entry_point_rejects_a_null_plan():
    """Each plan-taking entry point returns CFFT_ERR_INVALID_ARG for a NULL
    plan before touching any pointer or device."""
    L, lib = _lib()
    nul = ctypes.c_void_p(0)
    pairs = (ctypes.c_int32 * 2)(0, 0)
    basis = (L.Basis * 1)()
    calls = {
        "slab_green_eval": lambda: lib.slab_green_eval(None, 0, 2.2, 0.0, 0.05, nul, None),
        "mbf_spectra": lambda: lib.mbf_spectra(None, 0, basis, 1, nul, 1, nul, None),
        "cfft_tabulate": lambda: lib.cfft_tabulate(None, 0, nul, 1, nul, pairs, 1, nul, None),
        "cfft_lookup": lambda: lib.cfft_lookup(None, 0, nul, 1, nul, 1, nul, None),
        "cfft_lookup_quadratic": lambda: lib.cfft_lookup_quadratic(None, 0, nul, 1, nul, 1, nul, None),
        "cfft_fill": lambda: lib.cfft_fill(None, 0, nul, pairs, 1, 1, nul, 2, 2, nul, None),
        "cfft_fill_backward": lambda: lib.cfft_fill_backward(None, 0, nul, pairs, 1, 1, nul, 2, 2, nul, None),
        "cfft_lookup_backward": lambda: lib.cfft_lookup_backward(None, 0, nul, 1, nul, 1, nul, None),
        "cfft_backward": lambda: lib.cfft_backward(None, 0, nul, 2.2, 0.0, 0.05, basis, 1, nul, 1, pairs, 1, nul, nul,
                                                   nul, nul, None),
        "cfft_profile": lambda: lib.cfft_profile(None, 1),
    }
    for name, call in calls.items():
        assert call() == 1, name
        assert lib.cfft_last_error().decode(), name
    ms, n = ctypes.c_double(), ctypes.c_int64()
    assert lib.cfft_profile_read(None, 0, ctypes.byref(ms), ctypes.byref(n)) == 1


def test_no_device_is_reported_not_faked():
    """Without a GPU a valid plan request fails with CFFT_ERR_HIP (no CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    L, lib = _lib()
    desc = (L.GridDesc * 1)(L.grid_desc(_grid()))
    h = ctypes.c_void_p()
    assert lib.c_fft_plan(desc, 1, 4, 0, ctypes.byref(h)) == 4
