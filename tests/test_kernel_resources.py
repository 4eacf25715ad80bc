"""Compile-time guard on the gfx950 kernels: no kernel may spill to scratch,
and the PageRank sweeps must keep enough waves resident to hide gather
latency.  A spill turns the sweep's register traffic into HBM traffic (a
scratch-spilling slot sweep measured tens of times slower), and it is only
visible in the compiler's resource report, not in any result."""
import shutil

import pytest

from paper_2210_01465_amd import build

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None and not
                                __import__("os").path.exists("/opt/rocm/bin/hipcc"),
                                reason="hipcc not available")


@pytest.fixture(scope="module")
def resources():
    return build.kernel_resources("fl_kernels.hip")


def test_report_covers_the_kernels(resources):
    names = " ".join(resources)
    for k in ("k_pr_iter_slots", "k_pr_iter_csr", "k_batch_sweep", "k_degree_slots", "k_fill_slots",
              "k_compact_place", "k_seg_compact_write", "k_pr_finish"):
        assert k in names, k
    assert all("scratch" in r and "vgprs" in r for r in resources.values())


def test_no_kernel_spills(resources):
    spilled = {k: r["scratch"] for k, r in resources.items() if r["scratch"] != 0}
    assert not spilled, spilled


def test_sweeps_keep_occupancy(resources):
    low = {k: r for k, r in resources.items()
           if ("k_pr_iter" in k or "k_batch_sweep" in k) and r.get("occupancy", 0) < 4}
    assert not low, low
