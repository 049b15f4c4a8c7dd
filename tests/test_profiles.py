"""The committed measurement records match the kernels they describe (CPU check).

Each HBM-traffic record under profiles/ carries a hash of its kernel source's code
(comments and blank lines left out); bench.py reports that record's traffic only while
the hash matches.  Each rocprofv3 summary names the command that made it, and that
command runs committed files only.
"""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

PRECS = ("fp64", "fp32", "bf16x3")


@pytest.mark.parametrize("prec", PRECS)
def test_traffic_record_matches_kernel_source(prec):
    path = os.path.join(ROOT, "profiles", f"chi0_{prec}_slab3x3_naux384_traffic.json")
    rec = json.load(open(path))
    src = {"fp64": "chi0_f64.hip", "fp32": "chi0_mixed.hip", "bf16x3": "chi0_bf16.hip"}[prec]
    assert rec["kernel_source_sha256_16"] == bench.kernel_source_hash(src)
    t = bench.traffic_from_profiles("slab3x3_naux384", prec)
    assert t is not None and t >= rec["algorithmic_bytes_per_launch"]
    assert all("rocprofv3 --pmc" in c and "_work" not in c for c in rec["commands"])


@pytest.mark.parametrize("prec", PRECS)
def test_kernel_trace_summary_names_its_command(prec):
    text = open(os.path.join(ROOT, "profiles", f"chi0_{prec}_slab3x3_naux384.txt")).read()
    cmd = [ln for ln in text.splitlines() if "rocprofv3 --kernel-trace --stats" in ln]
    assert cmd and "bench.py" in cmd[0] and "_work" not in cmd[0]
    assert "chi0" in text and "AverageNs" in text


def test_code_hash_ignores_comments_only():
    a = "int f() {\n  return 1;  // one\n}\n"
    b = "// header\nint f() {\n\n  return 1;\n}\n"
    c = "int f() {\n  return 2;\n}\n"
    assert bench.code_hash(a) == bench.code_hash(b)
    assert bench.code_hash(a) != bench.code_hash(c)
