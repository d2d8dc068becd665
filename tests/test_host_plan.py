"""The planner's work plans checked on the host (no GPU): the bispectrum
kernel's LDS offsets, staged regions and output indices, and the
least-squares rounds' accumulator windows, for the benchmark's parameters
and others (tests/plan_check.cpp, built here with the host compiler)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1701_00581_amd", "csrc")

CASES = ["128:63:12:16", "128:63:10:16", "128:63:16:16", "128:40:16:16", "128:3:2:16",
         "64:31:8:16", "64:20:5:16", "64:31:3:16", "64:5:2:16", "128:63:12:24", "64:31:8:24"]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "plan_check.cpp"),
                    os.path.join(CSRC, "plan.cpp"), "-o", exe], check=True, capture_output=True)
    return exe


def test_work_plans_are_in_bounds_and_cover_every_sample_once(checker):
    r = subprocess.run([checker, *CASES], check=True, capture_output=True, text=True)
    lines = r.stdout.strip().splitlines()
    assert len(lines) == len(CASES)
    for line in lines:
        assert line.endswith(" bad=0"), line
