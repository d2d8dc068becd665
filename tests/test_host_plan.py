"""The planner's work plans checked on the host (no GPU): the bispectrum
kernel's LDS offsets, staged regions and output indices, the least-squares
rounds' accumulator windows, and the phase solve's groups and units, for
the benchmark's parameters and others (tests/plan_check.cpp, built here with
the host compiler)."""
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


def test_phase_solve_groups_join_only_independent_shells(checker):
    """The solve's barriers fall between groups of shells.  Re-planned with
    one group per shell (the order of the recursion itself) the units still
    pass the checks; with the first two groups after the seeds joined, where
    the second reads phasors of the first, the check must flag the plan, and
    the planner's own grouping must need fewer units than one group per shell."""
    geos = ["128:63:12:16", "64:31:3:16", "64:5:2:16", "128:40:16:16"]
    cases = geos + [f"shells:{g}" for g in geos] + [f"merge:{g}" for g in geos]
    r = subprocess.run([checker, *cases], check=True, capture_output=True, text=True)
    lines = dict(zip(cases, r.stdout.strip().splitlines()))
    assert len(lines) == len(cases)

    def field(line, name):
        return int(line.split(f" {name}=")[1].split()[0])

    for g in geos:
        assert lines[g].endswith(" bad=0"), lines[g]
        assert lines[f"shells:{g}"].endswith(" bad=0"), lines[f"shells:{g}"]
        assert field(lines[f"merge:{g}"], "units bad") > 0, lines[f"merge:{g}"]
        assert field(lines[g], "groups") < field(lines[g], "shells")
        assert field(lines[g], "units") < field(lines[f"shells:{g}"], "units")
