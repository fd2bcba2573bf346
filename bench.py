#!/usr/bin/env python3
"""Throughput of the contour-FFT tabulation on one MI355X.

Headline step: the large configuration, 4096 x 4096 grid over 200 x 200
lambda0, M = 6 MBFs of B = 1024 rooftops (36 MBF pairs), eps_r 10.2 slab,
P = 3, gamma = 1/130, FP64 (the paper's complex128): the slab Green's
function on the contour, the spectra of the 6 MBFs, the C-FFT tables of all
36 pairs (604 M entries) and the bilinear lookup of 10^5 displacements.
Inputs (basis geometry, coefficients, substrate, query points) are resident
before the timed region; every kernel is bracketed by HIP events on its own
stream during the timed steps.

Printed: one JSON line with the headline (table entries per second), its
error against the FP64 oracle, the roofline of the dominant kernel, the
oracle timed on the host (cpu_baseline), and side legs (the same workload
in mixed precision, the 512^2 workload, tensor truncation, parabolic
contour, 64^2 latency, the paper's own 2048^2 setup, the frequency sweep,
adjoint/forward time), each with its error against the oracle.  The oracle
runs only in the last, host-CPU leg.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector
HOST_THREADS = 16            # the host CPU share of one GPU on the benchmark boxes


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _ensure_built():
    if not os.path.exists(os.path.join(ROOT, "paper_1404_7357_amd", "libcfft.so")):
        import __graft_entry__
        __graft_entry__.build()


def _code_text(text):
    """Source text without comments and blank lines (a comment edit leaves the kernels unchanged)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.strip() for line in text.splitlines() if line.strip())


def _source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1404_7357_amd", "csrc", f)) as fh:
            h.update(_code_text(fh.read()).encode())
    return h.hexdigest()[:16]


PASS_SOURCES = ("cfft_passes.hip", "cfft_device.h")
GREEN_SOURCES = ("cfft_green.hip", "cfft_device.h")


def _counter_record(name):
    """A committed rocprofv3 counter record (profiles/<name>.json) if it still describes the current sources."""
    try:
        with open(os.path.join(ROOT, "profiles", name + ".json")) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("pass_source_hash") not in (None, _source_hash(PASS_SOURCES)):
        rec["kernels"] = {}
    if rec.get("green_source_hash") not in (None, _source_hash(GREEN_SOURCES)):
        rec.pop("green_fp64_flops_per_launch", None)
    return rec


def _host_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model or platform.processor()}


# --------------------------------------------------------------------------- GPU legs
class Leg:
    """Resident inputs and one plan for one grid of a workload."""

    def __init__(self, torch, wl, flags=0):
        from paper_1404_7357_amd import FLAG_ZERO_PAD2, Tabulator, _lib
        self.torch, self.wl, self._lib = torch, wl, _lib
        self.grid, self.sub = wl.grids[0], wl.substrates[0]
        flags |= FLAG_ZERO_PAD2 if self.grid.zero_pad else 0
        self.tab = Tabulator(self.grid, wl.basis, max_mbf=wl.M, flags=flags)
        self.q = torch.tensor(wl.q, device="cuda")
        self.pairs = [tuple(int(v) for v in p) for p in wl.pairs]
        gd = self.grid
        dt = torch.complex128 if gd.precision == 0 else torch.complex64
        self.g = torch.empty((3, gd.ny, gd.nx), dtype=torch.complex128, device="cuda")
        self.spec = torch.empty((wl.M, 4, gd.ny, gd.nx), dtype=dt, device="cuda")
        self.z = torch.empty((len(self.pairs), gd.ny, gd.nx), dtype=dt, device="cuda")
        self.pts = self.vals = None
        if wl.queries is not None:
            self.pts = torch.tensor(wl.queries, device="cuda")
            self.vals = torch.empty((len(self.pairs), self.pts.shape[0]), dtype=torch.complex128, device="cuda")

    def run(self, lookup=True):
        s = self.sub
        self.tab.green(s.eps_r, s.tan_delta, s.h, out=self.g)
        self.tab.spectra(self.q, out=self.spec)
        self.tab.tabulate(self.spec, self.g, self.pairs, out=self.z)
        if lookup and self.pts is not None:
            self.tab.lookup(self.z, self.pts, out=self.vals)

    def tabulate(self):
        self.tab.tabulate(self.spec, self.g, self.pairs, out=self.z)

    def entries(self):
        return self.grid.nx * self.grid.ny * len(self.pairs)

    def sampled_outputs(self, idx):
        """The table at flattened output indices idx, [npairs][len(idx)] complex128 on the host."""
        import numpy as np
        it = self.torch.tensor(idx, device="cuda")
        return self.z.reshape(len(self.pairs), -1)[:, it].cpu().numpy().astype(np.complex128)

    def sampled_factors(self, idx):
        """G and the spectra at flattened sample indices idx (host, complex128)."""
        import numpy as np
        it = self.torch.tensor(idx, device="cuda")
        g = self.g.reshape(3, -1)[:, it].cpu().numpy()
        s = self.spec.reshape(self.wl.M, 4, -1)[:, :, it].cpu().numpy().astype(np.complex128)
        return g, s

    def close(self):
        self.tab.close()


def _timed(torch, fn, steps, warmup, plan=None):
    """W untimed steps, then exactly K timed steps bracketed by synchronisations;
    with a plan, every kernel of the K steps is bracketed by HIP events on its
    launch stream.  Returns (seconds per step, per-class kernel times)."""
    from paper_1404_7357_amd import _lib
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if plan is not None:
        _lib.profile(plan, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    kernels = {}
    if plan is not None:
        _lib.profile(plan, False)
        for name in ("green", "spectra", "row_pass", "col_pass", "lookup"):
            ms, n = _lib.profile_read(plan, name)
            if n:
                kernels[name] = {"avg_ms": ms / n, "launches_per_step": n / steps}
        # a two-lane schedule runs one chunk's column pass beside the next
        # chunk's row pass: the event spans then overlap and are not
        # exclusive durations (their sum exceeds the step)
        busy = sum(k["avg_ms"] * k["launches_per_step"] for k in kernels.values())
        if busy > 1.02 * sec * 1e3:
            for name in ("row_pass", "col_pass"):
                if name in kernels:
                    kernels[name]["overlapping_lanes"] = True
    return sec, kernels


def _pass_bytes(gd, M, npairs_launch):
    """Algorithmic HBM bytes of one row-pass and one column-pass launch covering
    npairs_launch pairs (P+1 intermediates written and read, the table
    written; the Green's function (FP64) and the 4 spectra of each MBF in the
    grid's storage precision, each read once per launch that covers all M^2
    pairs, i.e. (3 + 4 M) arrays amortised over the M^2 pairs)."""
    s = 16 if gd.precision == 0 else 8
    P = gd.order
    inputs = (3 * 16 + 4 * M * s) / (M * M)
    inter = (P + 1) * s
    if gd.zero_pad:
        # a x2 zero-padded grid: the row pass reads the band samples (a
        # quarter) and writes the band rows (half); the column pass reads the
        # band rows and writes the whole table
        inputs /= 4
        inter /= 2
    e = gd.nx * gd.ny * npairs_launch
    return {"row_pass": e * (inter + inputs), "col_pass": e * (inter + s),
            "per_entry": {"row_pass": inter + inputs, "col_pass": inter + s}}


def _roofline(kernels, gd, M, npairs, copy_gbs, counters):
    per_launch = {k: npairs / kernels[k]["launches_per_step"] for k in ("row_pass", "col_pass")}
    out = {}
    for k in ("row_pass", "col_pass"):
        b = _pass_bytes(gd, M, per_launch[k])
        kernels[k]["pairs_per_launch"] = per_launch[k]
        kernels[k]["algorithmic_bytes_per_launch"] = b[k]
        kernels[k]["algorithmic_bytes_per_entry"] = b["per_entry"][k]
        kernels[k]["achieved_GBs"] = b[k] / (kernels[k]["avg_ms"] * 1e-3) / 1e9
        out[k] = b[k]
    dom = max(("row_pass", "col_pass"), key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches_per_step"])
    achieved = out[dom] / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = None
    if counters and dom in counters.get("kernels", {}):
        rec = counters["kernels"][dom]
        if abs(rec.get("pairs_per_launch", 0) - per_launch[dom]) < 1e-9:
            traffic = rec["hbm_bytes_per_launch"]
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes_per_launch": out[dom],
            "avg_launch_ms": kernels[dom]["avg_ms"], "copy_GBs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs if copy_gbs else None}


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


def _sample_idx(nx, ny, count, seed):
    """Seeded flattened indices including Delta = 0 and the four table corners."""
    import numpy as np
    rng = np.random.default_rng(seed)
    idx = set(rng.choice(nx * ny, count, replace=False).tolist())
    idx |= {(ny // 2) * nx + nx // 2, 0, nx - 1, (ny - 1) * nx, nx * ny - 1}
    return np.array(sorted(idx))


_SEEDED = {}


def _seeded_factors(gd, M, seed):
    """Synthetic, seeded Green's function and spectra arrays of a grid's shape:
    a smooth Gaussian envelope times seeded noise (no particular antenna).  They
    let the oracle's direct sum check the passes at sizes where its own
    Green's function and spectra would take hours (4096^2, B = 1024)."""
    import numpy as np
    from workloads import random_smooth_field
    from oracle.cfft_oracle import grid_samples  # sample coordinates only
    key = (gd.nx, gd.ny, gd.kx_max, gd.ky_max, M, seed)
    if key in _SEEDED:
        return _SEEDED[key]
    rng = np.random.default_rng(seed)
    kx, ky = grid_samples(gd.nx, gd.ny, gd.kx_max, gd.ky_max)
    env = np.exp(-0.5 * (kx ** 2 + ky ** 2) / (0.3 * max(gd.kx_max, gd.ky_max)) ** 2)
    n = gd.nx * gd.ny
    g = np.stack([env * random_smooth_field(rng, n) for _ in range(3)])
    spec = np.stack([np.stack([env * random_smooth_field(rng, n) for _ in range(4)]) for _ in range(M)])
    _SEEDED[key] = (g, spec)
    return g, spec


def _seeded_table(torch, leg, seed, check_pairs, nout):
    """The leg's launch configuration (grid, pair list, schedule) run on seeded
    factors: returns what the host leg needs to state the passes' error."""
    import numpy as np
    gd, M = leg.grid, leg.wl.M
    g, spec = _seeded_factors(gd, M, seed)
    sdt = torch.complex128 if gd.precision == 0 else torch.complex64
    gt = torch.tensor(g.reshape(3, gd.ny, gd.nx), device="cuda")
    st = torch.tensor(spec.reshape(M, 4, gd.ny, gd.nx), device="cuda").to(sdt)
    z = leg.tab.tabulate(st, gt, leg.pairs)
    idx = _sample_idx(gd.nx, gd.ny, nout, seed + 1)
    it = torch.tensor(idx, device="cuda")
    got = z.reshape(len(leg.pairs), -1)[:, it][check_pairs].cpu().numpy().astype(np.complex128)
    del z, gt, st
    if gd.precision != 0:
        spec = spec.astype(np.complex64).astype(np.complex128)   # the spectra the GPU read
    return {"grid": gd, "pairs": [leg.pairs[p] for p in check_pairs], "g": g, "spec": spec, "idx": idx, "got": got}


def _headline(torch, steps, warmup, precision=0, with_checks=True):
    """The large configuration in one precision: timed steps, kernel times,
    and the data for the host leg's error statement."""
    from workloads import c4_large
    wl = c4_large(precision=precision)
    leg = Leg(torch, wl)
    _log(f"{wl.name} prec={precision}: warmup {warmup}, steps {steps}")
    sec, kernels = _timed(torch, leg.run, steps, warmup, leg.tab.plan)
    sec_tab, _ = _timed(torch, leg.tabulate, max(2, steps // 2), 1)
    out = {"workload": wl.name, "entries": leg.entries(), "value": leg.entries() / sec, "ms_per_step": sec * 1e3,
           "passes_only": {"ms": sec_tab * 1e3, "value": leg.entries() / sec_tab, "unit": "entries/s"},
           "lookups": int(leg.pts.shape[0]) * len(leg.pairs), "kernels_ms": kernels,
           "schedule": "all 36 pairs in one row-pass and one column-pass launch, one stream"}
    checks = None
    if with_checks:
        sidx = _sample_idx(wl.grids[0].nx, wl.grids[0].ny, 8192, 11)
        g_s, s_s = leg.sampled_factors(sidx)
        checks = {"factors": (wl, sidx, g_s, s_s),
                  "table": _seeded_table(torch, leg, 77, [0, 7, 20, 35], 12)}
    return leg, out, checks


def _c2_leg(torch, steps, warmup, precision, truncation=0, contour=None):
    """The 512^2 workload (M = 4, B = 256, 16 pairs), autotuned schedule."""
    import dataclasses

    from paper_1404_7357_amd import FLAG_AUTOTUNE
    from workloads import c2_rooftop_512
    wl = c2_rooftop_512(precision=precision)
    grid = dataclasses.replace(wl.grids[0], truncation=truncation)
    if contour is not None:
        grid = dataclasses.replace(grid, contour=contour, beta_end=2.0 * grid.k0 * math.sqrt(wl.substrates[0].eps_r))
    wl = dataclasses.replace(wl, grids=[grid])
    leg = Leg(torch, wl, flags=FLAG_AUTOTUNE)
    sec, kernels = _timed(torch, leg.run, steps, warmup, leg.tab.plan)
    sec_tab, _ = _timed(torch, leg.tabulate, steps, 2)
    idx = _sample_idx(grid.nx, grid.ny, 64, 21)
    got = leg.sampled_outputs(idx)
    out = {"workload": wl.name, "value": leg.entries() / sec, "ms_per_step": sec * 1e3,
           "passes_only": {"ms": sec_tab * 1e3, "value": leg.entries() / sec_tab, "unit": "entries/s"},
           "dtype": "f64" if precision == 0 else "fp32 storage", "kernels_ms": kernels}
    leg.close()
    return out, {"wl": wl, "idx": idx, "got": got}


def _c1_latency(torch, steps, warmup):
    """64^2, one MBF, one pair, FP64: launch-bound, so the step latency is the figure of merit."""
    from workloads import c1_single_cosine
    wl = c1_single_cosine()
    leg = Leg(torch, wl)
    sec, _ = _timed(torch, leg.run, steps, warmup)
    z = leg.z.cpu().numpy()
    leg.close()
    return {"workload": wl.name, "latency_us": sec * 1e6, "entries": wl.grids[0].nx * wl.grids[0].ny,
            "dtype": "f64"}, {"wl": wl, "z": z}


def _paper_leg(torch, steps, warmup):
    """The paper's table setup (Sec. IV-F): 2048^2 FFT including the x2 zero
    padding, M = 9 MBFs (81 pairs), FP64; then the fill of the reduced matrix
    of the 25 x 25 regular array at 0.58 lambda0 by second-order interpolation
    in the refined table (390 000 element pairs x 81 MBF pairs)."""
    from paper_1404_7357_amd import FLAG_AUTOTUNE
    from workloads import paper_array_2048
    wl = paper_array_2048()
    leg = Leg(torch, wl, flags=FLAG_AUTOTUNE)
    pos = torch.tensor(wl.layout, device="cuda")
    am = pos.shape[0] * wl.M
    mat = torch.zeros((am, am), dtype=torch.complex128, device="cuda")
    sec, kernels = _timed(torch, leg.run, steps, warmup, leg.tab.plan)
    sec_tab, _ = _timed(torch, leg.tabulate, steps, 1)
    sec_fill, _ = _timed(torch, lambda: leg.tab.fill(leg.z, leg.pairs, wl.M, pos, out=mat), steps, 1)
    finite = bool(torch.isfinite(mat).all().item())
    del mat
    gd = wl.grids[0]
    idx = _sample_idx(gd.nx, gd.ny, 40, 31)
    got = leg.sampled_outputs(idx)
    sel = [0, 40, 80]
    leg.close()
    a_count = pos.shape[0]
    return {"workload": wl.name, "entries": leg.entries(), "value": leg.entries() / sec, "ms_per_step": sec * 1e3,
            "passes_only": {"ms": sec_tab * 1e3, "value": leg.entries() / sec_tab, "unit": "entries/s"},
            "fill_ms": sec_fill * 1e3, "fill_element_pairs": a_count * (a_count - 1),
            "fill_interpolations": a_count * (a_count - 1) * len(wl.pairs), "fill_all_finite": finite,
            "paper_cpu": {"fft_s_81_pairs": 126.36, "interp_s_390000": 1.62, "hardware": "one i7-3770"},
            "dtype": "f64", "kernels_ms": kernels}, {"wl": wl, "idx": idx, "got": got[sel], "sel": sel}


def _sweep(torch, steps, warmup):
    """Frequency sweep, 8 uneven grids x 16 pairs (mixed), eager and as one replayed HIP graph; the
    schedules are autotuned per grid by the first (warm-up) calls, before the capture.  Eager calls
    and replays are timed in two alternating rounds after their warm-ups (the first replays after a
    capture run slower), and each figure is the mean of its two rounds."""
    import numpy as np

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

    for _ in range(warmup):
        calls()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        calls()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls()
    te, tg = [], []
    for _ in range(2):
        te.append(_timed(torch, calls, steps, warmup)[0])
        tg.append(_timed(torch, graph.replay, steps, warmup)[0])
    t_eager, t_graph = sum(te) / 2, sum(tg) / 2
    samples = []
    for i, gd in enumerate(wl.grids):
        idx = _sample_idx(gd.nx, gd.ny, 16, 40 + i)
        it = torch.tensor(idx, device="cuda")
        samples.append((idx, bufs[i][2].reshape(len(pairs), -1)[:, it].cpu().numpy().astype(np.complex128)))
    entries = sum(gd.nx * gd.ny for gd in wl.grids) * len(pairs)
    tab.close()
    return {"workload": wl.name, "entries": entries, "value_graph": entries / t_graph,
            "ms_graph": t_graph * 1e3, "value_eager": entries / t_eager, "ms_eager": t_eager * 1e3,
            "dtype": "fp32 storage"}, {"wl": wl, "samples": samples}


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
    keep = {}

    def fwd():
        z = TableFunction.apply(eps, h, q, tab, sub.tan_delta, pairs, 0)
        keep["z"] = z
        v = LookupFunction.apply(z, pts, tab, 0)
        return (v - zt).abs().pow(2).sum()

    def fwd_only():
        with torch.no_grad():
            fwd()

    t_f, _ = _timed(torch, fwd_only, steps, warmup)

    def fwd_bwd():
        eps.grad = h.grad = q.grad = None
        loss = fwd()
        loss.backward()

    t_fb, _ = _timed(torch, fwd_bwd, steps, warmup)
    idx = _sample_idx(grid.nx, grid.ny, 32, 51)
    it = torch.tensor(idx, device="cuda")
    got = keep["z"].detach().reshape(len(pairs), -1)[:, it].cpu().numpy()
    tab.close()
    return {"workload": wl.name, "forward_ms": t_f * 1e3, "backward_ms": (t_fb - t_f) * 1e3,
            "adjoint_forward_ratio": (t_fb - t_f) / t_f, "entries": grid.nx * grid.ny * len(pairs),
            "queries": int(pts.shape[0])}, {"wl": wl, "idx": idx, "got": got}


def _green_alu(torch, leg, steps, counters):
    """Green's-function kernel alone on its launch stream (HIP events), against the FP64 vector peak."""
    s = leg.sub
    _, k = _timed(torch, lambda: leg.tab.green(s.eps_r, s.tan_delta, s.h, out=leg.g), steps, 2, leg.tab.plan)
    avg_ms = k["green"]["avg_ms"]
    flops = (counters or {}).get("green_fp64_flops_per_launch")
    achieved = flops / (avg_ms * 1e-3) / 1e12 if flops else None
    gd = leg.grid
    return {"bound": "alu", "kernel": "green", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS if achieved else None, "avg_ms": avg_ms,
            "fp64_flops_per_launch": flops, "samples_evaluated": (gd.nx // 2 + 1) * (gd.ny // 2 + 1),
            "samples_written": gd.nx * gd.ny}


# --------------------------------------------------------------------------- host-CPU leg
def _oracle_factors(grid, sub, basis, q, workers, idx=None):
    """The oracle's Green's function and spectra on every sample of a grid (or
    at flattened sample indices idx), its functions called on chunks of
    samples in parallel threads."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    from oracle import cfft_oracle as co
    kx, ky = co.grid_samples(grid.nx, grid.ny, grid.kx_max, grid.ky_max)
    if idx is not None:
        kx, ky = kx[idx], ky[idx]
    n = kx.size
    step = max(1, -(-n // workers))

    def chunk(i0):
        sl = slice(i0, min(n, i0 + step))
        kcx, kcy, _, gam = co.grid_contour(kx[sl], ky[sl], grid)
        g = co.green_remainder(kx[sl], ky[sl], gam, grid.k0, sub.eps_r, sub.tan_delta, sub.h)
        mt, mh = co.mbf_spectra(basis, q, kcx, kcy)
        return g, mt, mh

    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(chunk, range(0, n, step)))
    g = tuple(np.concatenate([p[0][c] for p in parts]) for c in range(3))
    mt = np.concatenate([p[1] for p in parts], axis=-1)
    mh = np.concatenate([p[2] for p in parts], axis=-1)
    return g, mt, mh


def _block(nout, workers):
    """Outputs per direct-sum task so that a few outputs still spread over the workers."""
    return max(1, -(-nout // workers))


def _rel_err(got, ref):
    """Largest error over pairs, relative to each pair's largest oracle value (the paper's max-normalised error)."""
    import numpy as np
    got, ref = np.asarray(got).reshape(len(ref), -1), np.asarray(ref).reshape(len(ref), -1)
    return float((np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)).max())


def _table_err_real(chk, workers):
    """A leg's sampled outputs against the oracle's direct sum on its own Green's function and spectra."""
    from oracle import cfft_oracle as co
    import numpy as np
    wl = chk["wl"]
    grid, sub = wl.grids[0], wl.substrates[0]
    mask = co.band_mask(grid)
    if mask is None:
        g, mt, mh = _oracle_factors(grid, sub, wl.basis, wl.q, workers)
    else:
        # a zero-padded grid carries the integrand on its band only: the
        # factors elsewhere are multiplied by zero, so only the band is evaluated
        band = np.nonzero(mask)[0]
        gb, mtb, mhb = _oracle_factors(grid, sub, wl.basis, wl.q, workers, idx=band)
        n = grid.nx * grid.ny
        g = tuple(np.zeros(n, dtype=np.complex128) for _ in range(3))
        for c in range(3):
            g[c][band] = gb[c]
        mt = np.zeros(mtb.shape[:-1] + (n,), dtype=np.complex128)
        mh = np.zeros_like(mt)
        mt[..., band] = mtb
        mh[..., band] = mhb
    pairs = chk.get("pairs", wl.pairs)
    sel = chk.get("sel")
    if sel is not None:
        pairs = [wl.pairs[p] for p in sel]
    ref = co.tabulate_from_factors(grid, pairs, g, mt, mh, out_idx=chk["idx"], workers=workers,
                                   block=_block(len(chk["idx"]), workers))
    return _rel_err(chk["got"], ref)


def _factor_err(factors, workers):
    """G and spectra at sampled samples against the oracle's (one max-normalised error each)."""
    import numpy as np
    wl, sidx, g_s, s_s = factors
    grid, sub = wl.grids[0], wl.substrates[0]
    t0 = time.perf_counter()
    g, mt, mh = _oracle_factors(grid, sub, wl.basis, wl.q, workers, idx=sidx)
    dt = time.perf_counter() - t0
    ref_g = np.stack(g)
    ref_s = np.concatenate([mt, mh], axis=1)
    return (float(np.abs(g_s - ref_g).max() / np.abs(ref_g).max()),
            float(np.abs(s_s - ref_s).max() / np.abs(ref_s).max()), dt / len(sidx))


def _cpu_baseline(checks, workers):
    """The oracle as it stands, on bounded samples of the large configuration,
    extrapolated to its whole table: (i) the Green's function and spectra on
    the sampled spectral samples of the headline's factor check (seconds per
    sample), (ii) the direct sum of eq. fftexp at the sampled outputs of the
    seeded-factor check, each over all 16.8 M samples (seconds per entry).
    The whole-table time is N_samples x (i) + entries x (ii)."""
    from oracle import cfft_oracle as co
    tab = checks["table"]
    t0 = time.perf_counter()
    ref = co.tabulate_from_factors(tab["grid"], tab["pairs"], tuple(tab["g"]), tab["spec"][:, 0:2],
                                   tab["spec"][:, 2:4], out_idx=tab["idx"], workers=workers,
                                   block=_block(len(tab["idx"]), workers))
    t_sum = time.perf_counter() - t0
    err_table = _rel_err(tab["got"], ref)
    err_g, err_s, t_fac_per_sample = _factor_err(checks["factors"], workers)
    gd = tab["grid"]
    n = gd.nx * gd.ny
    entries = n * 36
    sum_per_entry = t_sum / ref.size
    total = n * t_fac_per_sample + entries * sum_per_entry
    return {"value": entries / total, "unit": "entries/s", "cores": workers, "kind": "oracle",
            "sample": (f"{ref.size} outputs ({len(tab['idx'])} displacements x {len(tab['pairs'])} pairs) of the "
                       f"4096^2 table, each a direct sum over all {n} samples ({t_sum:.1f} s), plus the Green's "
                       f"function and spectra (B = 1024, M = 6) at {len(checks['factors'][1])} samples "
                       f"({t_fac_per_sample * len(checks['factors'][1]):.1f} s); extrapolated to the whole table "
                       f"({total / 3600:.1f} h)"),
            "seconds_direct_sum_per_entry": sum_per_entry, "seconds_factors_per_sample": t_fac_per_sample,
            **_host_info()}, {"table_seeded_factors": err_table, "green_sampled": err_g, "spectra_sampled": err_s}


def _cpu_cfft_paper_pair(workers):
    """The FFT work of one pair of the paper's table setup on the CPU: eq.
    fftarry with scipy FFT2 (10 transforms of 2048^2, complex128) on a
    synthetic integrand; the like-for-like figure for the paper's 1.56 s per
    pair (FFT time only, one i7-3770)."""
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


def _cpu_cfft_headline_pair(workers):
    """The passes of one pair of the headline workload on the CPU: eq. fftarry
    literally, scipy FFT2 (10 transforms of 4096^2, complex128) on a synthetic
    integrand of the same size, with every worker thread of the host; scaled
    to the 36 pairs of the step as passes-only entries/s (the analogue of the
    GPU's passes_only figure)."""
    import numpy as np

    from oracle import cfft_cpu
    from oracle import cfft_oracle as co
    from workloads import c4_large
    wl = c4_large(precision=0)
    grid = wl.grids[0]
    rng = np.random.default_rng(6)
    n = grid.nx * grid.ny
    kx, ky = co.grid_samples(grid.nx, grid.ny, grid.kx_max, grid.ky_max)
    w = np.full(n, (1 + 1j * grid.gamma) ** 2)
    noise = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)   # noqa: E731
    fac = (kx, ky, w, noise(3, n), noise(1, 2, n), noise(1, 2, n))
    t0 = time.perf_counter()
    cfft_cpu.tabulate_cfft(grid, wl.substrates[0], wl.basis, wl.q[:1], np.array([(0, 0)]), workers=workers,
                           factors=fac)
    sec = time.perf_counter() - t0
    npairs = len(wl.pairs)
    return {"seconds_per_pair": sec, "passes_entries_per_s": n / sec, "seconds_all_pairs": sec * npairs,
            "cores": workers, "kind": "cpu-cfft",
            "sample": f"one pair of the {grid.nx}^2 FP64 headline grid, 10 FFT2 + weighting, synthetic integrand; "
                      f"x {npairs} pairs for the step (passes only: no Green's function or spectra)"}


def _cpu_leg(out, checks, workers):
    """The host-CPU leg, run after every GPU leg: the oracle timed on bounded
    samples of the headline workload (cpu_baseline) and each GPU result's error
    against it.  Nothing else in this script runs the oracle."""
    _log(f"cpu oracle: headline sample, {workers} threads")
    base, comp = _cpu_baseline(checks["headline"], workers)
    out["cpu_baseline"] = base
    out["oracle_check"] = {**comp, "how": ("the passes on seeded factors of the headline's shape and launch "
                                           "configuration at 12 sampled displacements (corners and Delta = 0 "
                                           "included) x 4 pairs; the Green's function and spectra of the "
                                           "workload itself at 8197 sampled samples")}
    out["rel_err_vs_oracle"] = max(comp.values())
    if "mixed" in checks:
        _, cm = _cpu_baseline(checks["mixed"], workers)
        out["mixed"]["oracle_check"] = cm
        out["mixed"]["rel_err_vs_oracle"] = max(cm.values())
    for key in ("c2", "c2_mixed", "tensor_fp64", "tensor_mixed", "parabolic"):
        if key in checks:
            _log(f"cpu oracle: {key}")
            leg = out
            for k in {"c2": ("c2",), "c2_mixed": ("c2", "mixed"), "tensor_fp64": ("tensor", "fp64"),
                      "tensor_mixed": ("tensor", "mixed"), "parabolic": ("parabolic",)}[key]:
                leg = leg[k]
            leg["rel_err_vs_oracle"] = _table_err_real(checks[key], workers)
            leg["oracle_sample"] = f"{len(checks[key]['idx'])} outputs x 16 pairs, the oracle's own factors"
    if "c1" in checks:
        from oracle import cfft_oracle as co
        wl1, z1 = checks["c1"]["wl"], checks["c1"]["z"]
        r1 = co.tabulate(wl1.grids[0], wl1.substrates[0], wl1.basis, wl1.q, wl1.pairs)
        out["c1_latency"]["rel_err_vs_oracle"] = _rel_err(z1, r1)
    if "paper_setup" in checks:
        _log("cpu oracle: paper setup")
        out["paper_setup"]["rel_err_vs_oracle"] = _table_err_real(checks["paper_setup"], workers)
        out["paper_setup"]["oracle_sample"] = "band factors of the oracle itself; 45 outputs x 3 pairs"
    if "sweep" in checks:
        _log("cpu oracle: sweep (8 grids)")
        import dataclasses
        wl = checks["sweep"]["wl"]
        errs = []
        for i, (idx, got) in enumerate(checks["sweep"]["samples"]):
            wli = dataclasses.replace(wl, grids=[wl.grids[i]], substrates=[wl.substrates[i]])
            errs.append(_table_err_real({"wl": wli, "idx": idx, "got": got}, workers))
        out["sweep"]["rel_err_vs_oracle"] = max(errs)
        out["sweep"]["rel_err_per_grid"] = errs
    if "adjoint" in checks:
        _log("cpu oracle: differentiation workload forward table")
        out["adjoint"]["rel_err_vs_oracle"] = _table_err_real(checks["adjoint"], workers)
    _log("cpu C-FFT, one pair of the paper's 2048^2 setup")
    out["cpu_cfft_paper_pair"] = _cpu_cfft_paper_pair(workers)
    _log("cpu C-FFT, one pair of the headline 4096^2 grid")
    out["cpu_cfft_headline_pair"] = _cpu_cfft_headline_pair(workers)


# --------------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline only (no side legs)")
    ap.add_argument("--copy-calibration", action="store_true", help="run one 256 MiB device copy (counter scale)")
    ap.add_argument("--only", choices=("headline", "mixed", "c2", "paper_setup", "sweep", "adjoint"),
                    help="run one GPU leg alone and print its JSON (for profiling it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    _ensure_built()
    import torch

    from workloads import CONTOUR_PARABOLIC, MIXED, TRUNC_TENSOR
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X (no device visible)", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.only and args.only != "headline":
        fn = {"mixed": lambda: _headline(torch, args.steps, args.warmup, MIXED, False)[1],
              "c2": lambda: _c2_leg(torch, args.steps, args.warmup, 0)[0],
              "paper_setup": lambda: _paper_leg(torch, args.steps, args.warmup)[0],
              "sweep": lambda: _sweep(torch, max(20, args.steps), max(5, args.warmup))[0],
              "adjoint": lambda: _adjoint_ratio(torch, args.steps, args.warmup)[0]}[args.only]
        print(json.dumps({"leg": args.only, **fn()}), flush=True)
        return

    counters = _counter_record("counters_c4_fp64")
    leg, head, hchk = _headline(torch, args.steps, args.warmup, 0, with_checks=not args.only)
    gd, M = leg.grid, leg.wl.M
    green = _green_alu(torch, leg, args.steps, counters)
    leg.close()
    del leg
    torch.cuda.empty_cache()
    copy_gbs = None if (args.no_extras or args.only) else _copy_rate(torch)
    kernels = head.pop("kernels_ms")
    roofline = _roofline(kernels, gd, M, 36, copy_gbs, counters)
    out = {"metric": "MBF reaction terms tabulated/s at stated rel. error vs FP64; adjoint/forward time",
           "value": head["value"], "unit": "entries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": head["workload"], "grid": f"{gd.nx}x{gd.ny}", "span_lambda0": 200.0,
                      "pairs": 36, "mbf": M, "rooftops": 1024, "order": gd.order, "gamma": gd.gamma,
                      "eps_r": 10.2, "tan_delta": 0.0, "h": 0.12, "lookups": 100000, "precision": "fp64",
                      "schedule": head["schedule"]},
           "rel_err_vs_oracle": None, "roofline": roofline, "green_fp64": green,
           "passes_only": head["passes_only"], "kernels_ms": kernels}
    if args.only:
        print(json.dumps(out), flush=True)
        return
    checks = {"headline": hchk}

    if not args.no_extras:
        _log("mixed-precision large leg")
        mleg, mixed, checks["mixed"] = _headline(torch, max(3, args.steps // 2), 1, MIXED)
        mleg.close()
        del mleg
        torch.cuda.empty_cache()
        mixed["dtype"] = "fp32 storage, fp64 transforms (4096-point axes)"
        out["mixed"] = mixed
        _log("512^2 legs")
        out["c2"], checks["c2"] = _c2_leg(torch, args.steps, args.warmup, 0)
        out["c2"]["mixed"], checks["c2_mixed"] = _c2_leg(torch, args.steps, args.warmup, MIXED)
        tf, checks["tensor_fp64"] = _c2_leg(torch, args.steps, args.warmup, 0, truncation=TRUNC_TENSOR)
        tm, checks["tensor_mixed"] = _c2_leg(torch, args.steps, args.warmup, MIXED, truncation=TRUNC_TENSOR)
        out["tensor"] = {"fp64": tf, "mixed": tm}
        out["parabolic"], checks["parabolic"] = _c2_leg(torch, max(3, args.steps // 4), 2, 0,
                                                        contour=CONTOUR_PARABOLIC)
        _log("64^2 single-pair latency leg")
        out["c1_latency"], checks["c1"] = _c1_latency(torch, 50, 10)
        _log("paper-setup leg (2048^2 incl. zero padding, 81 pairs, 25 x 25 array fill)")
        out["paper_setup"], checks["paper_setup"] = _paper_leg(torch, 3, 1)
        _log("sweep leg (8 grids, one graph)")
        out["sweep"], checks["sweep"] = _sweep(torch, max(20, args.steps), max(5, args.warmup))
        _log("adjoint leg (1024^2, 16 pairs, 4096 lookups)")
        out["adjoint"], checks["adjoint"] = _adjoint_ratio(torch, max(3, args.steps // 4), 2)

    if not args.no_cpu_baseline:
        _cpu_leg(out, checks, min(HOST_THREADS, os.cpu_count() or 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
