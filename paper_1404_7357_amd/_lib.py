"""ctypes binding of libcfft.so (argument marshalling only).

Every function here converts torch tensors to device pointers and forwards to
the C ABI declared in include/cfft.h; no arithmetic of the method happens in
Python.  torch is imported first so that the library binds to the HIP runtime
that torch already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfft.so")

CFFT_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "ALLOC", 4: "HIP", 5: "NONFINITE"}

CONTOUR_RAY, CONTOUR_PARABOLIC = 0, 1
FP64, MIXED = 0, 1
TRUNC_TOTAL, TRUNC_TENSOR = 0, 1
FLAG_CHECK_FINITE = 1
FLAG_AUTOTUNE = 2
FLAG_ZERO_PAD2 = 4

ENTRY_POINTS = ("c_fft_plan", "c_fft_plan_destroy", "slab_green_eval", "mbf_spectra", "cfft_tabulate",
                "cfft_tabulate_noalloc",
                "cfft_lookup", "cfft_lookup_quadratic", "cfft_fill", "cfft_fill_backward", "cfft_lookup_backward",
                "cfft_lookup_quadratic_backward", "cfft_backward", "cfft_profile",
                "cfft_profile_read",
                "cfft_last_error", "cfft_version")

PROFILE_CLASSES = {"green": 0, "spectra": 1, "row_pass": 2, "col_pass": 3, "lookup": 4, "adj_col_pass": 5,
                   "adj_row_pass": 6, "adj_integrand": 7, "adj_green": 8, "adj_spectra": 9}


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("kx_max", ctypes.c_double), ("ky_max", ctypes.c_double),
                ("k0", ctypes.c_double), ("gamma", ctypes.c_double),
                ("contour", ctypes.c_int32), ("order", ctypes.c_int32),
                ("beta_end", ctypes.c_double),
                ("precision", ctypes.c_int32), ("truncation", ctypes.c_int32)]


class Basis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("a", ctypes.c_double), ("b", ctypes.c_double)]


class CfftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libcfft.so once; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcfft.so not built at {path}; run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.c_fft_plan.argtypes = [ctypes.POINTER(GridDesc), i32, i32, i32, ctypes.POINTER(vp)]
    lib.c_fft_plan_destroy.argtypes = [vp]
    lib.slab_green_eval.argtypes = [vp, i32, dbl, dbl, dbl, vp, vp]
    lib.mbf_spectra.argtypes = [vp, i32, ctypes.POINTER(Basis), i32, vp, i32, vp, vp]
    lib.cfft_tabulate.argtypes = [vp, i32, vp, i32, vp, ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
    lib.cfft_tabulate_noalloc.argtypes = [vp, i32, vp, i32, vp, ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
    lib.cfft_lookup.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cfft_lookup_quadratic.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cfft_fill.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_int32), i32, i32, vp, i32, i32, vp, vp]
    lib.cfft_fill_backward.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_int32), i32, i32, vp, i32, i32, vp, vp]
    lib.cfft_lookup_backward.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cfft_lookup_quadratic_backward.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
    lib.cfft_backward.argtypes = [vp, i32, vp, dbl, dbl, dbl, ctypes.POINTER(Basis), i32, vp, i32,
                                  ctypes.POINTER(ctypes.c_int32), i32, vp, vp, vp, vp, vp]
    lib.cfft_profile.argtypes = [vp, i32]
    lib.cfft_profile_read.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for name in ENTRY_POINTS:
        fn = getattr(lib, name)
        fn.restype = ctypes.c_char_p if name in ("cfft_last_error", "cfft_version") else ctypes.c_int
    _lib = lib
    return lib


def check(status: int):
    if status != CFFT_OK:
        raise CfftError(status, load().cfft_last_error().decode())


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(t.data_ptr())
    return ctypes.c_void_p(int(t))


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def grid_desc(g) -> GridDesc:
    """GridDesc from any object with the cfft_grid_desc_t field names."""
    return GridDesc(int(g.nx), int(g.ny), float(g.kx_max), float(g.ky_max), float(g.k0), float(g.gamma),
                    int(getattr(g, "contour", CONTOUR_RAY)), int(g.order), float(getattr(g, "beta_end", 0.0)),
                    int(g.precision), int(getattr(g, "truncation", TRUNC_TOTAL)))


def basis_array(records):
    """ctypes array of Basis from a numpy structured array (kind, pad, cx, cy, a, b)."""
    arr = (Basis * len(records))()
    for i, r in enumerate(records):
        arr[i] = Basis(int(r["kind"]), 0, float(r["cx"]), float(r["cy"]), float(r["a"]), float(r["b"]))
    return arr


def pairs_array(pairs):
    flat = [int(v) for p in pairs for v in p]
    return (ctypes.c_int32 * len(flat))(*flat)


class Plan:
    """Owns a cfft plan handle (c_fft_plan / c_fft_plan_destroy)."""

    def __init__(self, grids, max_mbf: int, flags: int = 0):
        lib = load()
        descs = (GridDesc * len(grids))(*[grid_desc(g) for g in grids])
        handle = ctypes.c_void_p()
        check(lib.c_fft_plan(descs, len(grids), int(max_mbf), int(flags), ctypes.byref(handle)))
        self.handle = handle
        self.grids = list(grids)

    def close(self):
        if self.handle is not None and self.handle.value:
            check(load().c_fft_plan_destroy(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def slab_green_eval(plan: Plan, grid: int, eps_r: float, tan_delta: float, h: float, g, stream=None):
    check(load().slab_green_eval(plan.handle, grid, float(eps_r), float(tan_delta), float(h), _ptr(g),
                                 _stream(stream)))


def mbf_spectra(plan: Plan, grid: int, basis, q, spec, stream=None):
    b = basis if isinstance(basis, ctypes.Array) else basis_array(basis)
    check(load().mbf_spectra(plan.handle, grid, b, len(b), _ptr(q), int(q.shape[0]), _ptr(spec), _stream(stream)))


def cfft_tabulate(plan: Plan, grid: int, spec, nmbf: int, g, pairs, z, stream=None):
    pa = pairs_array(pairs)
    check(load().cfft_tabulate(plan.handle, grid, _ptr(spec), int(nmbf), _ptr(g), pa, len(pa) // 2, _ptr(z),
                               _stream(stream)))


def cfft_tabulate_noalloc(plan: Plan, grid: int, spec, nmbf: int, g, pairs, z, stream=None):
    pa = pairs_array(pairs)
    check(load().cfft_tabulate_noalloc(plan.handle, grid, _ptr(spec), int(nmbf), _ptr(g), pa, len(pa) // 2,
                                       _ptr(z), _stream(stream)))


def cfft_lookup(plan: Plan, grid: int, z, npairs: int, pts, out, stream=None):
    check(load().cfft_lookup(plan.handle, grid, _ptr(z), int(npairs), _ptr(pts), int(pts.shape[0]), _ptr(out),
                             _stream(stream)))


def cfft_lookup_quadratic(plan: Plan, grid: int, z, npairs: int, pts, out, stream=None):
    check(load().cfft_lookup_quadratic(plan.handle, grid, _ptr(z), int(npairs), _ptr(pts), int(pts.shape[0]),
                                       _ptr(out), _stream(stream)))


def cfft_fill(plan: Plan, grid: int, z, pairs, nmbf: int, pos, order: int, out, stream=None):
    pa = pairs_array(pairs)
    check(load().cfft_fill(plan.handle, grid, _ptr(z), pa, len(pa) // 2, int(nmbf), _ptr(pos), int(pos.shape[0]),
                           int(order), _ptr(out), _stream(stream)))


def cfft_fill_backward(plan: Plan, grid: int, dout, pairs, nmbf: int, pos, order: int, dz, stream=None):
    pa = pairs_array(pairs)
    check(load().cfft_fill_backward(plan.handle, grid, _ptr(dout), pa, len(pa) // 2, int(nmbf), _ptr(pos),
                                    int(pos.shape[0]), int(order), _ptr(dz), _stream(stream)))


def cfft_lookup_backward(plan: Plan, grid: int, dout, npairs: int, pts, dz, stream=None):
    check(load().cfft_lookup_backward(plan.handle, grid, _ptr(dout), int(npairs), _ptr(pts), int(pts.shape[0]),
                                      _ptr(dz), _stream(stream)))


def cfft_lookup_quadratic_backward(plan: Plan, grid: int, dout, npairs: int, pts, dz, stream=None):
    check(load().cfft_lookup_quadratic_backward(plan.handle, grid, _ptr(dout), int(npairs), _ptr(pts),
                                                int(pts.shape[0]), _ptr(dz), _stream(stream)))


def cfft_backward(plan: Plan, grid: int, dz, eps_r, tan_delta, h, basis, q, pairs, g, spec, grad_sub, grad_q,
                  stream=None):
    b = basis if isinstance(basis, ctypes.Array) else basis_array(basis)
    pa = pairs_array(pairs)
    check(load().cfft_backward(plan.handle, grid, _ptr(dz), float(eps_r), float(tan_delta), float(h), b, len(b),
                               _ptr(q), int(q.shape[0]), pa, len(pa) // 2, _ptr(g), _ptr(spec), _ptr(grad_sub),
                               _ptr(grad_q), _stream(stream)))


def profile(plan: Plan, enable: bool):
    check(load().cfft_profile(plan.handle, 1 if enable else 0))


def profile_read(plan: Plan, kernel: str):
    """(total_ms, launches) of one kernel class since the last read."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(load().cfft_profile_read(plan.handle, PROFILE_CLASSES[kernel], ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def last_error() -> str:
    return load().cfft_last_error().decode()


def version() -> str:
    return load().cfft_version().decode()
