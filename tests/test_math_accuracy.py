"""The kernels' FP64 elementary functions (paper_1905_02241_amd/csrc/mech_math.h)
built for the host and checked against long-double references.

The rate functions, the Nernst potential and the clamp waveform of every
FP64 kernel go through exp_d, expm1_d, log_d and sin_d, so their accuracy
bounds the FP64 parity bars from below.  Measured worst cases over 2e7
arguments: e^x 0.99 ulp, e^x - 1 1.79 ulp (x just above ln2/2, where the
result is about half the series term it is formed from), ln x 1.12 ulp,
sin x 1.48 ulp; the bars below sit just above those.  The host build runs the same operations in the same
order (fma_s is a plain fused multiply-add there)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "math_host.cpp")
INC = os.path.join(ROOT, "paper_1905_02241_amd", "csrc")


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("math") / "math_host")
    subprocess.run([cxx, "-O2", "-ffp-contract=off", "-I", INC, SRC, "-o", exe, "-lm"], check=True)
    out = subprocess.run([exe, "400000"], check=True, capture_output=True, text=True).stdout
    return {k: float(v) for k, v in (line.split() for line in out.strip().splitlines())}


def test_exp_within_one_ulp(report):
    assert report["exp"] <= 1.0


def test_expm1_within_two_ulp(report):
    assert report["expm1"] <= 2.0


def test_log_within_one_and_a_half_ulp(report):
    assert report["log"] <= 1.5


def test_sin_within_two_ulp(report):
    assert report["sin"] <= 2.0
    assert report["sin_abs"] <= 2.5e-16


def test_special_values(report):
    assert report["exp(-800)"] == 0.0
    assert report["exp(800)"] == float("inf")
    assert report["expm1(-800)"] == -1.0
    assert report["expm1(0)"] == 0.0
    assert report["log(1)"] == 0.0
    assert report["log(0)"] == float("-inf")
    assert report["log(-1)"] != report["log(-1)"]   # NaN
    assert report["sin(0)"] == 0.0
    assert report["exp(nan)"] != report["exp(nan)"]
