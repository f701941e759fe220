"""The compiler's resource report for every kernel of the last build
(paper_1605_05508_amd/_build/resources.json, written by build_lib): no
kernel may keep much in scratch memory.

A kernel's by-value argument structure is copied to scratch when the
optimiser gives up proving the copy redundant (1.3 KB per lane for the
building's arguments), which made the score kernel three times slower
without any error; the building kernels are held to a few spilled
registers, and every kernel stays below the size of such a copy.  The fit's
autotuner trials at tight register budgets spill by design (up to a few
hundred bytes), which the second limit allows.
"""
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT = os.path.join(ROOT, "paper_1605_05508_amd", "_build", "resources.json")

BUILD_KERNELS = ("build_", "bin_", "seed_")  # name parts of the building's kernels
BUILD_SCRATCH_MAX = 64   # bytes per lane
ANY_SCRATCH_MAX = 1024   # bytes per lane, below a copy of an argument structure


@pytest.fixture(scope="module")
def kernels():
    if not os.path.exists(REPORT):
        pytest.skip("no resource report: build the library first")
    with open(REPORT) as f:
        d = json.load(f)
    assert d["kernels"], "empty resource report"
    return d["kernels"]


def test_building_kernels_stay_out_of_scratch(kernels):
    bad = {n: k["scratch"] for n, k in kernels.items()
           if any(p in n for p in BUILD_KERNELS) and k.get("scratch", 0) > BUILD_SCRATCH_MAX}
    assert not bad, f"building kernels in scratch (bytes per lane): {bad}"


def test_no_kernel_holds_an_argument_copy(kernels):
    bad = {n: k["scratch"] for n, k in kernels.items() if k.get("scratch", 0) > ANY_SCRATCH_MAX}
    assert not bad, f"kernels with more scratch than {ANY_SCRATCH_MAX} bytes per lane: {bad}"


def test_hot_kernels_keep_their_occupancy(kernels):
    """The float building's score kernel runs at three waves per SIMD and its
    merge at six or more; the headline fit's tuned shapes at three."""
    def find(*parts):
        hits = [k for n, k in kernels.items() if all(p in n for p in parts)]
        assert hits, f"no kernel named with {parts}"
        return hits
    for k in find("build_score_kernelIffLb0ELb1ELb0E"):
        assert k["occupancy"] >= 3 and k["scratch"] == 0
    for k in find("build_merge_kernelIfLi2ELi5E"):
        assert k["occupancy"] >= 6 and k["scratch"] == 0
    for k in find("fit_fused_kernelIffd", "Li3ELb0ELb0ELi1E"):
        assert k["occupancy"] >= 3
