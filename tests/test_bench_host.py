"""Host-side parts of bench.py (no GPU): the one-GPU guard, the comment-
insensitive source hash that ties the committed counter record to the kernel
sources, and that record's consistency with the algorithmic bytes the
benchmark line reports for the 4096^2 FP64 passes."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_source_hash_ignores_comments_only():
    b = _bench()
    code = "int f(int x) {\n  return x + 1;\n}\n"
    commented = "// a note\nint f(int x) {  // trailing\n  /* block\n     comment */ return x + 1;\n\n}\n"
    assert b._code_text(code) == b._code_text(commented)
    assert b._code_text(code) != b._code_text(code.replace("+ 1", "+ 2"))


def test_counter_record_matches_sources_and_algorithmic_bytes():
    b = _bench()
    with open(os.path.join(ROOT, "profiles", "counters_c4_fp64.json")) as fh:
        raw = json.load(fh)
    rec = b._counter_record("counters_c4_fp64")
    assert rec is not None
    # the record describes the kernel sources as committed (else the line reports traffic = null)
    assert raw["pass_source_hash"] == b._source_hash(b.PASS_SOURCES)
    assert raw["green_source_hash"] == b._source_hash(b.GREEN_SOURCES)
    cal = rec["calibration"]
    assert abs(cal["fetch_scale"] - 2.0) < 0.05 and abs(cal["write_scale"] - 1.0) < 0.05
    entries = 36 * 4096 * 4096
    # algorithmic bytes per entry of one launch of all 36 pairs: row 76 B, column 80 B (FP64, M = 6, P = 3)
    for kernel, per_entry in (("row_pass", 76), ("col_pass", 80)):
        k = rec["kernels"][kernel]
        assert k["pairs_per_launch"] == 36
        ratio = k["hbm_bytes_per_launch"] / (per_entry * entries)
        assert 0.95 < ratio < 1.1, (kernel, ratio)
    assert rec["green_fp64_flops_per_launch"] > 0
