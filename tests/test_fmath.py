"""The library's double exp, log and division (csrc/fmath.h), built for the host and checked
against long double references: at most 1.5 ulp (exp), 2 ulp (log) and 2 ulp (division, from a
reciprocal seed no better than float) over argument sweeps, and the special cases (saturation,
exact values, non-finite arguments; a NaN exp argument saturates to the lower bound)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    out = tmp_path_factory.mktemp("fmath") / "fmath_check"
    src = os.path.join(ROOT, "tests", "fmath_check.cpp")
    inc = os.path.join(ROOT, "paper_2210_08024_amd", "csrc")
    subprocess.run([hipcc, "-O2", "-x", "hip", "--offload-arch=gfx950", "-I", inc, src, "-o", str(out)],
                   check=True, capture_output=True)
    res = subprocess.run([str(out)], check=True, capture_output=True, text=True).stdout
    return {ln.split()[0]: ln.split()[1] for ln in res.strip().splitlines()}


def test_exp_accuracy(report):
    assert float(report["exp_max_ulp"]) <= 1.5, report
    assert report["exp_special"] == "1"


def test_division_accuracy(report):
    assert float(report["div_max_ulp"]) <= 2.0, report


def test_log_accuracy(report):
    assert float(report["log_max_ulp"]) <= 2.0, report
    assert report["log_special"] == "1"
