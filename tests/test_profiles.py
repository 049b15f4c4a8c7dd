"""The committed measurement records match the kernels they describe (CPU check).

Each HBM-traffic record under profiles/ carries a hash of its kernel source's code
(comments and blank lines left out); bench.py reports that record's traffic only while
the hash matches, and null once the kernel has changed.  Each rocprofv3 summary names the
command that made it, and that command runs committed files only.
"""
import glob
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

SRC = {"fp64": "chi0_f64.hip", "fp32": "chi0_mixed.hip", "bf16x3": "chi0_bf16.hip", "f16x3": "chi0_bf16.hip"}
RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "chi0_*_traffic.json")))
SUMMARIES = sorted(glob.glob(os.path.join(ROOT, "profiles", "chi0_*.txt")))


def parse(path):
    name = os.path.basename(path)[len("chi0_"):]
    prec, workload = name.split("_", 1)
    return prec, workload.replace("_traffic.json", "").replace(".txt", "")


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_traffic_record_is_reported_only_for_its_kernel(path):
    rec = json.load(open(path))
    prec, workload = parse(path)
    t = bench.traffic_from_profiles(workload, prec)
    if rec["kernel_source_sha256_16"] == bench.kernel_source_hash(SRC[prec]):
        assert t is not None and t >= rec["algorithmic_bytes_per_launch"]
    else:
        assert t is None
    assert all("rocprofv3 --pmc" in c and "_work" not in c and "bench.py" in c for c in rec["commands"])


def test_default_workload_has_current_records():
    # the bench's default line (3x3x1, N_aux 2400, FP64) has a kernel trace summary and a
    # traffic record taken with the committed contraction kernel
    assert os.path.exists(os.path.join(ROOT, "profiles", "chi0_fp64_slab3x3_naux2400.txt"))
    assert bench.traffic_from_profiles("slab3x3_naux2400", "fp64") is not None


@pytest.mark.parametrize("path", SUMMARIES, ids=[os.path.basename(p) for p in SUMMARIES])
def test_kernel_trace_summary_names_its_command(path):
    text = open(path).read()
    prec, workload = parse(path)
    cmd = [ln for ln in text.splitlines() if "rocprofv3 --kernel-trace --stats" in ln]
    assert cmd and "bench.py" in cmd[0] and "_work" not in cmd[0]
    # the command reproduces the summary's workload and precision
    if workload != "slab3x3_naux2400":
        assert f"--workload {workload}" in cmd[0]
    if prec != "fp64":
        assert f"--prec {prec}" in cmd[0]
    assert "AverageNs" in text


def test_code_hash_ignores_comments_only():
    a = "int f() {\n  return 1;  // one\n}\n"
    b = "// header\nint f() {\n\n  return 1;\n}\n"
    c = "int f() {\n  return 2;\n}\n"
    assert bench.code_hash(a) == bench.code_hash(b)
    assert bench.code_hash(a) != bench.code_hash(c)
