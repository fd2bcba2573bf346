#!/usr/bin/env python3
"""Throughput of the contour-FFT tabulation on one MI355X.

One step = the whole forward hot path for one antenna/substrate: the slab
Green's function on the contour, the spectra of the M = 4 MBFs (B = 256
rooftops each), and the C-FFT table of all 16 MBF pairs on a 512 x 512 grid
(P = 3, gamma = 1/130), in FP64.  Inputs (basis geometry, coefficients,
substrate) are resident before the timed region.

Printed: one JSON line with the headline (table entries per second), the
roofline of the dominant kernel (per-kernel HIP event timing), side
measurements (mixed precision, the other workloads, adjoint/forward time on
the 1024^2 differentiation workload), and, from a last host-CPU leg, the
oracle timed on a bounded sample with each GPU result's error against it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _ensure_built():
    if not os.path.exists(os.path.join(ROOT, "paper_1404_7357_amd", "libcfft.so")):
        import __graft_entry__
        __graft_entry__.build()


def _source_hash(files=("cfft_passes.hip", "cfft_device.h")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1404_7357_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel, launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", "traffic_c2_fp64.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != _source_hash() or kernel not in rec.get("kernels", {}):
        return None
    return rec["kernels"][kernel].get("hbm_bytes_per_launch")


class Step:
    """Resident inputs and one Tabulator for a workload grid."""

    def __init__(self, wl, torch):
        from paper_1404_7357_amd import FLAG_AUTOTUNE, FLAG_ZERO_PAD2, Tabulator, _lib
        self.torch = torch
        self.wl = wl
        self.grid = wl.grids[0]
        self.sub = wl.substrates[0]
        # the pair-chunk schedule is autotuned on the first (warm-up) call
        flags = FLAG_AUTOTUNE | (FLAG_ZERO_PAD2 if self.grid.zero_pad else 0)
        self.tab = Tabulator(self.grid, wl.basis, max_mbf=wl.M, flags=flags)
        self.q = torch.tensor(wl.q, device="cuda")
        self.pairs = [tuple(int(v) for v in p) for p in wl.pairs]
        gd = self.grid
        dt = torch.complex128 if gd.precision == 0 else torch.complex64
        self.g = torch.empty((3, gd.ny, gd.nx), dtype=torch.complex128, device="cuda")
        self.spec = torch.empty((wl.M, 4, gd.ny, gd.nx), dtype=dt, device="cuda")
        self.z = torch.empty((len(self.pairs), gd.ny, gd.nx), dtype=dt, device="cuda")
        self._lib = _lib

    def run(self):
        # One stream: running the (independent) Green's function on a second
        # stream beside the spectra measured slower at every size, the
        # fork/join costing more than the overlap saves (512^2: 185 vs 177 us;
        # 64^2: 93 vs 34 us).
        s = self.sub
        self.tab.green(s.eps_r, s.tan_delta, s.h, out=self.g)
        self.tab.spectra(self.q, out=self.spec)
        self.tab.tabulate(self.spec, self.g, self.pairs, out=self.z)

    def entries(self):
        return self.grid.nx * self.grid.ny * len(self.pairs)


def _time_steps(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _kernel_times(st, steps):
    """Average duration per launch (ms) of every kernel class, by HIP events on the launch stream."""
    lib = st._lib
    lib.profile(st.tab.plan, True)
    for _ in range(steps):
        st.run()
    st.torch.cuda.synchronize()
    lib.profile(st.tab.plan, False)
    out = {}
    for name in ("green", "spectra", "row_pass", "col_pass"):
        ms, n = lib.profile_read(st.tab.plan, name)
        if n:
            out[name] = {"avg_ms": ms / n, "launches_per_step": n / steps}
    return out


def _copy_rate(torch, mib=1024, reps=20):
    """Device-to-device copy (read + write) GB/s on this GPU: the practical ceiling for a streaming pass."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def _cpu_cfft(wl, z_gpu, workers):
    """The CPU C-FFT baseline (eq. fftarry taken literally with scipy FFT2) on
    the whole workload, with the GPU table's deviation from it."""
    import numpy as np

    from oracle import cfft_cpu
    from oracle import cfft_oracle as co
    grid, sub = wl.grids[0], wl.substrates[0]
    t0 = time.perf_counter()
    fac = co.sampled_factors(grid, sub, wl.basis, wl.q)
    t1 = time.perf_counter()
    z = cfft_cpu.tabulate_cfft(grid, sub, wl.basis, wl.q, wl.pairs, workers=workers, factors=fac)
    t2 = time.perf_counter()
    entries = z.size
    dev = float((np.abs(z_gpu.reshape(z.shape) - z).reshape(len(wl.pairs), -1).max(axis=1)
                 / np.abs(z).reshape(len(wl.pairs), -1).max(axis=1)).max())
    return {"value": entries / (t2 - t0), "unit": "entries/s", "cores": workers, "kind": "cpu-cfft",
            "seconds": t2 - t0, "seconds_factors": t1 - t0, "seconds_fft": t2 - t1,
            "sample": f"whole table ({len(wl.pairs)} pairs x {grid.nx}x{grid.ny}), "
                      f"{len(cfft_cpu.terms(grid.order))} FFT2 per pair, scipy.fft",
            "rel_dev_gpu": dev}


def _cpu_cfft_paper_pair(workers):
    """The FFT work of one pair of the paper's table setup on the CPU: eq.
    fftarry with scipy FFT2 (10 transforms of 2048^2, complex128) on a
    synthetic integrand; the like-for-like figure for the paper's 1.56 s per
    pair (FFT time only, one i7-3770).  The Green's function and spectra
    are not part of that figure and are replaced by seeded noise here."""
    import numpy as np

    from oracle import cfft_cpu
    from oracle import cfft_oracle as co
    from workloads import paper_array_2048
    wl = paper_array_2048()
    grid = wl.grids[0]
    rng = np.random.default_rng(5)
    n = grid.nx * grid.ny
    kx, ky = co.grid_samples(grid.nx, grid.ny, grid.kx_max, grid.ky_max)
    w = np.full(n, (1 + 1j * grid.gamma) ** 2)
    noise = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)   # noqa: E731
    fac = (kx, ky, w, noise(3, n), noise(1, 2, n), noise(1, 2, n))
    t0 = time.perf_counter()
    cfft_cpu.tabulate_cfft(grid, wl.substrates[0], wl.basis, wl.q[:1], np.array([(0, 0)]), workers=workers,
                           factors=fac)
    sec = time.perf_counter() - t0
    return {"seconds_per_pair": sec, "cores": workers, "kind": "cpu-cfft",
            "sample": "one pair, 2048^2 incl. zero padding, 10 FFT2 + weighting, synthetic integrand",
            "paper_seconds_per_pair": 1.56, "paper_hardware": "one i7-3770"}


def _green_flops():
    """FP64 flops of one Green's-function launch (512^2 grid) from the committed rocprofv3 counters, if current."""
    path = os.path.join(ROOT, "profiles", "traffic_c2_fp64.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("green_source_hash") != _source_hash(("cfft_green.hip", "cfft_device.h")):
        return None
    return rec.get("green_fp64_flops_per_launch")


def _green_alu(st, steps):
    """Green's-function kernel alone on the launch stream (HIP events), against the FP64 vector peak."""
    lib = st._lib
    s = st.sub
    lib.profile(st.tab.plan, True)
    for _ in range(steps):
        st.tab.green(s.eps_r, s.tan_delta, s.h, out=st.g)
    st.torch.cuda.synchronize()
    lib.profile(st.tab.plan, False)
    ms, n = lib.profile_read(st.tab.plan, "green")
    avg_ms = ms / n
    flops = _green_flops()
    achieved = flops / (avg_ms * 1e-3) / 1e12 if flops else None
    gd = st.grid
    return {"bound": "alu", "kernel": "green", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "avg_ms": avg_ms,
            "fp64_flops_per_launch": flops, "samples_evaluated": (gd.nx // 2 + 1) * (gd.ny // 2 + 1),
            "samples_written": gd.nx * gd.ny}


def _cpu_baseline(wl, z_gpu, n_out, workers):
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np

    from oracle import cfft_oracle as co
    grid, sub = wl.grids[0], wl.substrates[0]
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(grid.nx * grid.ny, n_out, replace=False))
    idx[0] = (grid.ny // 2) * grid.nx + grid.nx // 2          # Delta = 0 (table maximum)
    idx = np.unique(idx)
    t0 = time.perf_counter()
    ref = co.tabulate(grid, sub, wl.basis, wl.q, wl.pairs, out_idx=idx, workers=workers)
    dt = time.perf_counter() - t0
    entries = ref.size
    zs = z_gpu.reshape(len(wl.pairs), -1)[:, idx]
    err = float((np.abs(zs - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())
    return {"value": entries / dt, "unit": "entries/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(idx)} output displacements x {len(wl.pairs)} pairs of the 512x512 table "
                      f"(Green's function and spectra on all 262144 samples, direct sum per output), "
                      f"{dt:.1f} s"}, err, (idx, ref)


def _rel_err(got, ref):
    """Largest error over pairs, relative to each pair's largest oracle value."""
    import numpy as np
    return float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())


def _cpu_leg(out, tables, n_out, workers):
    """The host-CPU leg, run after every GPU leg: the oracle timed on a bounded
    sample of the benchmark workload (cpu_baseline) and the CPU C-FFT
    baselines.  The oracle's values on that sample, and on sampled outputs of
    the other legs' tables (collected in `tables`), state each GPU result's
    error against the FP64 oracle.  Nothing else in this script runs the
    oracle."""
    import numpy as np

    from oracle import cfft_oracle as co
    wl, z_fp64 = tables["c2"]
    npairs = len(wl.pairs)
    _log(f"cpu oracle on {n_out} outputs x {npairs} pairs, {workers} threads")
    base, err, (idx, ref) = _cpu_baseline(wl, z_fp64, n_out, workers)
    out["cpu_baseline"] = base
    out["rel_err_vs_oracle"] = err
    _log("cpu C-FFT baseline (eq. fftarry with scipy FFT2, whole table)")
    out["cpu_cfft"] = _cpu_cfft(wl, z_fp64, workers)
    _log("cpu C-FFT, one pair of the paper's 2048^2 setup")
    out["cpu_cfft_paper_pair"] = _cpu_cfft_paper_pair(workers)
    if "mixed" in tables:
        out["mixed"]["rel_err_vs_oracle"] = _rel_err(tables["mixed"].reshape(npairs, -1)[:, idx], ref)
    # other legs: the oracle at 64 sampled outputs per pair plus Delta = 0
    for key, seed, target in (("tensor_fp64", 77, ("tensor", "fp64")), ("tensor_mixed", 77, ("tensor", "mixed")),
                              ("parabolic", 78, ("parabolic",))):
        if key not in tables:
            continue
        wlx, z = tables[key]
        grid, sub = wlx.grids[0], wlx.substrates[0]
        rng = np.random.default_rng(seed)
        sidx = np.unique(np.concatenate([rng.choice(grid.nx * grid.ny, 64, replace=False),
                                         [(grid.ny // 2) * grid.nx + grid.nx // 2]]))
        sref = co.tabulate(grid, sub, wlx.basis, wlx.q, wlx.pairs, out_idx=sidx, workers=workers)
        leg = out
        for k in target:
            leg = leg[k]
        leg["rel_err_vs_oracle"] = _rel_err(z[:, sidx], sref)
        leg["oracle_sample"] = f"{len(sidx)} outputs x {len(wlx.pairs)} pairs"
    if "c1" in tables:
        wl1, z1 = tables["c1"]
        r1 = co.tabulate(wl1.grids[0], wl1.substrates[0], wl1.basis, wl1.q, wl1.pairs)
        out["c1_latency"]["rel_err_vs_oracle"] = float(np.abs(z1 - r1).max() / np.abs(r1).max())


def _adjoint_ratio(torch, steps, warmup):
    """Forward (table + lookup + loss) vs backward (lookup adjoint + cfft_backward) on 1024^2."""
    from paper_1404_7357_amd import LookupFunction, TableFunction, Tabulator
    from workloads import c5_gradient
    wl = c5_gradient()
    grid, sub = wl.grids[0], wl.substrates[0]
    tab = Tabulator(grid, wl.basis, max_mbf=wl.M)
    pairs = [tuple(int(v) for v in p) for p in wl.pairs]
    pts = torch.tensor(wl.queries, device="cuda")
    q = torch.tensor(wl.q, device="cuda", requires_grad=True)
    eps = torch.tensor(sub.eps_r, dtype=torch.float64, device="cuda", requires_grad=True)
    h = torch.tensor(sub.h, dtype=torch.float64, device="cuda", requires_grad=True)
    zt = torch.zeros((len(pairs), pts.shape[0]), dtype=torch.complex128, device="cuda")

    def fwd():
        z = TableFunction.apply(eps, h, q, tab, sub.tan_delta, pairs, 0)
        v = LookupFunction.apply(z, pts, tab, 0)
        return (v - zt).abs().pow(2).sum()

    def fwd_only():
        with torch.no_grad():
            fwd()

    t_f = _time_steps(torch, fwd_only, steps, warmup)

    def fwd_bwd():
        eps.grad = h.grad = q.grad = None
        loss = fwd()
        loss.backward()

    t_fb = _time_steps(torch, fwd_bwd, steps, warmup)
    tab.close()
    return {"workload": wl.name, "forward_ms": t_f * 1e3, "backward_ms": (t_fb - t_f) * 1e3,
            "adjoint_forward_ratio": (t_fb - t_f) / t_f, "entries": grid.nx * grid.ny * len(pairs),
            "queries": int(pts.shape[0])}


def _tensor_leg(torch, steps, warmup, precision):
    """The 512^2 workload with the tensor-product truncation (one intermediate
    per pair; not in the paper).  Returns the leg's figures and (workload,
    table) for the CPU leg, which states its error against the oracle's
    tensor mode."""
    import dataclasses

    from workloads import TRUNC_TENSOR, c2_rooftop_512
    wl = c2_rooftop_512(precision=precision)
    wl = dataclasses.replace(wl, grids=[dataclasses.replace(wl.grids[0], truncation=TRUNC_TENSOR)])
    st = Step(wl, torch)
    sec = _time_steps(torch, st.run, steps, warmup)
    sec_tab = _time_steps(torch, lambda: st.tab.tabulate(st.spec, st.g, st.pairs, out=st.z), steps, 2)
    km = _kernel_times(st, steps)
    torch.cuda.synchronize()
    z = st.z.cpu().numpy().reshape(len(wl.pairs), -1)
    st.tab.close()
    return {"value": st.entries() / sec, "ms_per_step": sec * 1e3,
            "passes_only": {"ms": sec_tab * 1e3, "value": st.entries() / sec_tab, "unit": "entries/s"},
            "dtype": "f64" if precision == 0 else "fp32 FFT / fp64 rest", "kernels_ms": km}, (wl, z)


def _parabolic_leg(torch, steps, warmup):
    """The 512^2 workload on the parabolic contour (beta_end = 2 k0 sqrt(eps_r)):
    per-sample spectra, (P+1)(P+2)/2 row transforms; FP64.  Returns the
    leg's figures and (workload, table) for the CPU leg's error statement."""
    import dataclasses
    import math as _m

    from workloads import CONTOUR_PARABOLIC, c2_rooftop_512
    wl = c2_rooftop_512()
    sub = wl.substrates[0]
    grid = dataclasses.replace(wl.grids[0], contour=CONTOUR_PARABOLIC,
                               beta_end=2.0 * wl.grids[0].k0 * _m.sqrt(sub.eps_r))
    wl = dataclasses.replace(wl, grids=[grid])
    st = Step(wl, torch)
    sec = _time_steps(torch, st.run, steps, warmup)
    sec_tab = _time_steps(torch, lambda: st.tab.tabulate(st.spec, st.g, st.pairs, out=st.z), steps, 2)
    km = _kernel_times(st, steps)
    torch.cuda.synchronize()
    z = st.z.cpu().numpy().reshape(len(wl.pairs), -1)
    st.tab.close()
    return {"value": st.entries() / sec, "ms_per_step": sec * 1e3, "beta_end": grid.beta_end,
            "passes_only": {"ms": sec_tab * 1e3, "value": st.entries() / sec_tab, "unit": "entries/s"},
            "dtype": "f64", "kernels_ms": km}, (wl, z)


def _large_leg(torch, steps, warmup):
    """The large configuration: 4096^2, 36 pairs (M = 6, B = 1024), mixed
    precision, followed by the bilinear lookup of 10^5 displacements."""
    from workloads import c4_large
    wl = c4_large()
    st = Step(wl, torch)
    pts = torch.tensor(wl.queries, device="cuda")
    vals = torch.empty((len(wl.pairs), pts.shape[0]), dtype=torch.complex128, device="cuda")

    def step():
        st.run()
        st.tab.lookup(st.z, pts, out=vals)

    sec = _time_steps(torch, step, steps, warmup)
    sec_lookup = _time_steps(torch, lambda: st.tab.lookup(st.z, pts, out=vals), steps, 1)
    km = _kernel_times(st, steps)
    st.tab.close()
    return {"workload": wl.name, "entries": st.entries(), "value": st.entries() / sec, "ms_per_step": sec * 1e3,
            "lookup_ms": sec_lookup * 1e3, "lookups": int(pts.shape[0]) * len(wl.pairs),
            "dtype": "fp32 FFT / fp64 rest", "kernels_ms": km}


def _c1_latency(torch, steps, warmup):
    """The smallest configuration (64^2, one MBF, one pair, FP64): launch-bound, so its step latency is
    the figure of merit.  Returns (workload, table) too: the CPU leg states its error against the
    oracle's whole table."""
    from workloads import c1_single_cosine
    wl = c1_single_cosine()
    st = Step(wl, torch)
    sec = _time_steps(torch, st.run, steps, warmup)
    torch.cuda.synchronize()
    z = st.z.cpu().numpy()
    st.tab.close()
    return {"workload": wl.name, "latency_us": sec * 1e6, "entries": st.entries(), "dtype": "f64"}, (wl, z)


def _paper_leg(torch, steps, warmup):
    """The paper's own table setup (Sec. IV-F): a 2048^2 FFT including the x2
    zero padding, M = 9 MBFs (81 pairs), FP64; then the fill of the reduced
    matrix of the 25 x 25 regular array at 0.58 lambda0 (Sec. IV-E) by
    second-order interpolation in the refined table (390 000 element pairs
    x 81 MBF pairs)."""
    from workloads import paper_array_2048
    wl = paper_array_2048()
    st = Step(wl, torch)
    pos = torch.tensor(wl.layout, device="cuda")
    am = pos.shape[0] * wl.M
    mat = torch.zeros((am, am), dtype=torch.complex128, device="cuda")   # self blocks stay zero here
    sec = _time_steps(torch, st.run, steps, warmup)
    sec_tab = _time_steps(torch, lambda: st.tab.tabulate(st.spec, st.g, st.pairs, out=st.z), steps, 1)
    sec_fill = _time_steps(torch, lambda: st.tab.fill(st.z, st.pairs, wl.M, pos, out=mat), steps, 1)
    km = _kernel_times(st, steps)
    finite = bool(torch.isfinite(mat).all().item())
    st.tab.close()
    a_count = pos.shape[0]
    return {"workload": wl.name, "entries": st.entries(), "value": st.entries() / sec, "ms_per_step": sec * 1e3,
            "passes_only": {"ms": sec_tab * 1e3, "value": st.entries() / sec_tab, "unit": "entries/s"},
            "fill_ms": sec_fill * 1e3, "fill_element_pairs": a_count * (a_count - 1),
            "fill_interpolations": a_count * (a_count - 1) * len(wl.pairs), "fill_all_finite": finite,
            "paper_cpu": {"fft_s_81_pairs": 126.36, "interp_s_390000": 1.62, "hardware": "one i7-3770"},
            "dtype": "f64", "kernels_ms": km}


def _sweep(torch, steps, warmup):
    """Frequency sweep, 8 uneven grids x 16 pairs (mixed), eager and as one replayed HIP graph; the
    schedules are autotuned per grid by the first (warm-up) calls, before the capture."""
    from paper_1404_7357_amd import FLAG_AUTOTUNE, Tabulator
    from workloads import c3_frequency_sweep
    wl = c3_frequency_sweep()
    tab = Tabulator(wl.grids, wl.basis, max_mbf=wl.M, flags=FLAG_AUTOTUNE)
    q = torch.tensor(wl.q, device="cuda")
    pairs = [tuple(int(v) for v in p) for p in wl.pairs]
    bufs = []
    for gd in wl.grids:
        bufs.append((torch.empty((3, gd.ny, gd.nx), dtype=torch.complex128, device="cuda"),
                     torch.empty((wl.M, 4, gd.ny, gd.nx), dtype=torch.complex64, device="cuda"),
                     torch.empty((len(pairs), gd.ny, gd.nx), dtype=torch.complex64, device="cuda")))

    def calls():
        for i, (gd, sub) in enumerate(zip(wl.grids, wl.substrates)):
            g, spec, z = bufs[i]
            tab.green(sub.eps_r, sub.tan_delta, sub.h, grid=i, out=g)
            tab.spectra(q, grid=i, out=spec)
            tab.tabulate(spec, g, pairs, grid=i, out=z)

    t_eager = _time_steps(torch, calls, steps, warmup)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls()
    t_graph = _time_steps(torch, graph.replay, steps, warmup)
    entries = sum(gd.nx * gd.ny for gd in wl.grids) * len(pairs)
    tab.close()
    return {"workload": wl.name, "entries": entries, "value_graph": entries / t_graph,
            "ms_graph": t_graph * 1e3, "value_eager": entries / t_eager, "ms_eager": t_eager * 1e3,
            "dtype": "fp32 FFT / fp64 rest"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-outputs", type=int, default=1024, help="oracle sample size (outputs per pair)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the mixed-precision and adjoint legs")
    ap.add_argument("--copy-calibration", action="store_true", help="run one 256 MiB device copy (counter scale)")
    ap.add_argument("--only", choices=("large", "paper_setup", "sweep", "adjoint"),
                    help="run one extra leg alone and print its JSON (for profiling it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    _ensure_built()
    import torch

    from workloads import MIXED, c2_rooftop_512
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X (no device visible)", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.only:
        leg = {"large": _large_leg, "paper_setup": _paper_leg, "sweep": _sweep, "adjoint": _adjoint_ratio}[args.only]
        print(json.dumps({"leg": args.only, **leg(torch, args.steps, args.warmup)}), flush=True)
        return

    wl = c2_rooftop_512()
    _log(f"workload {wl.name}: warmup {args.warmup}, steps {args.steps}")
    st = Step(wl, torch)
    sec = _time_steps(torch, st.run, args.steps, args.warmup)
    value = st.entries() / sec
    _log(f"fp64 step {sec * 1e3:.3f} ms -> {value:.4e} entries/s")
    # the row and column passes alone (cfft_tabulate on resident G and spectra)
    sec_tab = _time_steps(torch, lambda: st.tab.tabulate(st.spec, st.g, st.pairs, out=st.z), args.steps, 2)
    passes_only = {"ms": sec_tab * 1e3, "value": st.entries() / sec_tab, "unit": "entries/s"}
    kernels = _kernel_times(st, args.steps)
    green_alu = _green_alu(st, args.steps)
    torch.cuda.synchronize()
    z_fp64 = st.z.cpu().numpy()

    # roofline of the dominant kernel (row or column pass); a launch covers
    # npairs / launches pairs (the autotuned pair chunk)
    n = wl.grids[0].nx * wl.grids[0].ny
    P = wl.grids[0].order
    npairs = len(wl.pairs)
    s = 16
    per_launch = {k: npairs / kernels[k]["launches_per_step"] for k in ("row_pass", "col_pass")}
    # row pass inputs of one launch: G (3 arrays) plus the testing spectra
    # (Mx, My) of the launch's distinct m and the reflected ones (Mx#, My#) of
    # its distinct n, each read once
    chunk = int(round(per_launch["row_pass"]))
    plist = [tuple(p) for p in wl.pairs]
    in_arrays = []
    for c0 in range(0, npairs, chunk):
        part = plist[c0:c0 + chunk]
        in_arrays.append(3 + 2 * len({m for m, _ in part}) + 2 * len({q for _, q in part}))
    launch_bytes = {
        "row_pass": sum(in_arrays) / len(in_arrays) * n * 16 + (P + 1) * n * s * per_launch["row_pass"],
        "col_pass": (P + 1) * n * s * per_launch["col_pass"] + n * s * per_launch["col_pass"],
    }
    dom = max(("row_pass", "col_pass"), key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
    avg_s = kernels[dom]["avg_ms"] * 1e-3
    achieved = launch_bytes[dom] / avg_s / 1e9
    # the device copy rate (skipped in the short profiling runs, whose copy
    # calibration must be the only large copy)
    copy_gbs = None if args.no_extras else _copy_rate(torch)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic(dom, launch_bytes[dom]),
                "algorithmic_bytes_per_launch": launch_bytes[dom],
                "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None}
    for k in ("row_pass", "col_pass"):
        kernels[k]["pairs_per_launch"] = per_launch[k]
        kernels[k]["algorithmic_bytes_per_launch"] = launch_bytes[k]
        kernels[k]["achieved_GBs"] = launch_bytes[k] / (kernels[k]["avg_ms"] * 1e-3) / 1e9

    out = {"metric": "MBF reaction terms tabulated/s at stated rel. error vs FP64; adjoint/forward time",
           "value": value, "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl.name, "grid": "512x512", "pairs": npairs, "mbf": wl.M, "rooftops": wl.B,
                      "order": P, "gamma": wl.grids[0].gamma, "eps_r": wl.substrates[0].eps_r,
                      "tan_delta": wl.substrates[0].tan_delta, "h": wl.substrates[0].h,
                      "precision": "fp64"},
           "roofline": roofline, "green_fp64": green_alu, "passes_only": passes_only, "kernels_ms": kernels}
    st.tab.close()
    del st

    # GPU tables kept for the CPU leg's error statements
    tables = {"c2": (wl, z_fp64)}

    if not args.no_extras:
        wlm = c2_rooftop_512(precision=MIXED)
        stm = Step(wlm, torch)
        secm = _time_steps(torch, stm.run, args.steps, args.warmup)
        secm_tab = _time_steps(torch, lambda: stm.tab.tabulate(stm.spec, stm.g, stm.pairs, out=stm.z), args.steps, 2)
        km = _kernel_times(stm, args.steps)
        mixed = {"value": stm.entries() / secm, "ms_per_step": secm * 1e3, "dtype": "fp32 FFT / fp64 rest",
                 "passes_only": {"ms": secm_tab * 1e3, "value": stm.entries() / secm_tab, "unit": "entries/s"},
                 "kernels_ms": km}
        torch.cuda.synchronize()
        tables["mixed"] = stm.z.cpu().numpy()
        stm.tab.close()
        del stm
        out["mixed"] = mixed
        _log("tensor-product truncation legs (FP64, mixed)")
        tf, tables["tensor_fp64"] = _tensor_leg(torch, args.steps, args.warmup, 0)
        tm, tables["tensor_mixed"] = _tensor_leg(torch, args.steps, args.warmup, MIXED)
        out["tensor"] = {"fp64": tf, "mixed": tm}
        _log("parabolic-contour leg (FP64)")
        out["parabolic"], tables["parabolic"] = _parabolic_leg(torch, max(3, args.steps // 5), 2)
        _log("large leg (4096^2, 36 pairs, 10^5 lookups)")
        out["large"] = _large_leg(torch, 3, 1)
        _log("64^2 single-pair latency leg")
        out["c1_latency"], tables["c1"] = _c1_latency(torch, args.steps, args.warmup)
        _log("paper-setup leg (2048^2 incl. zero padding, 81 pairs, 25 x 25 array fill)")
        out["paper_setup"] = _paper_leg(torch, 3, 1)
        _log("sweep leg (8 grids, one graph)")
        out["sweep"] = _sweep(torch, max(3, args.steps // 5), 2)
        _log("adjoint leg (1024^2, 16 pairs, 4096 lookups)")
        out["adjoint"] = _adjoint_ratio(torch, max(3, args.steps // 5), 2)

    if not args.no_cpu_baseline:
        _cpu_leg(out, tables, args.cpu_outputs, min(16, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
