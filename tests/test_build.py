"""The compiler's resource report of the last build (no GPU): no product
kernel keeps values in scratch memory.

A spill puts per-lane loads and stores to scratch on the critical path
and shows up as HBM writes in the counters; the pair kernel's register
budget at three wavefronts per SIMD is the usual cause. Only the pair
kernel's counting variants (diagnostic counters on, never used for
timing) may spill."""
import os
import re

import pytest

from paper_1607_02427_amd import build as B

REPORTS = {src: B.resources_path(src) for src in B.SOURCES}
pytestmark = pytest.mark.skipif(not all(os.path.exists(p) for p in REPORTS.values()),
                                reason="no resource report: libdem.so was not built by build.py")

COUNTING = re.compile(r"k_pairsI[fd]Li\dELi\d+ELb1E")


def _kernels(path):
    """(mangled name, scratch bytes per lane, VGPRs) of each kernel in one report."""
    out = []
    for blk in open(path).read().split("Function Name: ")[1:]:
        name = blk.split("\n", 1)[0].strip()
        scratch = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", blk)
        vgpr = re.search(r"VGPRs: (\d+)", blk)
        assert scratch and vgpr, name
        out.append((name, int(scratch.group(1)), int(vgpr.group(1))))
    return out


def test_every_source_reports_its_kernels():
    names = [n for p in REPORTS.values() for n, _, _ in _kernels(p)]
    for k in ("k_pairs", "k_gather", "k_kick_drift", "k_nbr", "k_fill", "k_assign", "k_replica_tail"):
        assert any(k in n for n in names), k


def test_no_product_kernel_spills():
    spills = [(n, s) for p in REPORTS.values() for n, s, _ in _kernels(p) if s > 0 and not COUNTING.search(n)]
    assert not spills, spills


def test_pair_kernels_fit_their_occupancy():
    """Three wavefronts per SIMD leave 168 VGPRs per lane (512 / 3, in
    granules of 8); the variants built for three must fit them."""
    for n, _, v in _kernels(REPORTS["dem_force.hip"]):
        m = re.search(r"k_pairsI[fd]Li\dELi\d+ELb0ELi(\d)E", n)
        if m and m.group(1) == "3":
            assert v <= 168, (n, v)
