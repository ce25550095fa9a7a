"""Host logic of the iteration issue planner (IssuePlan, in
paper_2206_14780_amd/csrc/issue_plan.hpp): tests/issue_plan_sim.cpp runs the
solver's issue loop (two polls in flight, the older one read before more is
queued) against synthetic residual histories; here it is compiled with the
host compiler and its results checked.  No GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def sim(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("issue_plan") / "sim")
    subprocess.run([cxx, "-O1", "-std=c++17", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2206_14780_amd", "csrc"),
                    os.path.join(HERE, "issue_plan_sim.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        name, h, issued, maxb = line.split()
        res[name] = (int(h), int(issued), int(maxb))
    return res


KMAX = {"geometric_kmax1": 1, "geometric_kmax16": 16}


def test_every_batch_within_its_limit_and_the_halt_always_issued(sim):
    for name, (h, issued, maxb) in sim.items():
        assert maxb <= KMAX.get(name, 8), name
        assert issued >= h, name  # the halting p-update must run


def test_a_predictable_decay_issues_nothing_past_the_halt(sim):
    # geometric decay of r.r: the predicted halt is exact, and no iteration
    # is queued past it, whatever the batch limit
    for name in ("geometric", "geometric_kmax1", "geometric_kmax16", "slow", "one_component", "plateau"):
        h, issued, _ = sim[name]
        assert issued == h, (name, h, issued)


def test_a_noisy_decay_issues_little_past_the_halt(sim):
    h, issued, _ = sim["noisy"]
    assert h > 100 and issued - h <= 8


def test_a_converged_start_wastes_only_the_blind_batches(sim):
    # before the first poll is read nothing is known: the batches of 2 and 4
    h, issued, _ = sim["converged_start"]
    assert h == 1 and issued <= 6
