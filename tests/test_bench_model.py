"""The bench's algorithmic work model (roofline numerators): level splits,
multiply-add, MFMA-operation and HBM-byte counts per pass, and the guard that
drops measured traffic once the kernel sources differ from the profiled ones."""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def inter(levels):
    """Multiply-adds of a pass's levels: the last merge (with its quotient
    step, 32), and per inter-level twiddle an unreduced merge (24) plus one
    Shoup product (64 + 45 + 45)."""
    return 32 + (levels - 1) * (24 + 154)


def test_level_split_matches_the_library_rule():
    # fewest levels of radix <= 16, larger levels first, except that three
    # levels start with the smallest
    assert bench.level_split(12) == [4, 4, 4]
    assert bench.level_split(11) == [3, 4, 4]
    assert bench.level_split(10) == [3, 4, 3]
    assert bench.level_split(9) == [3, 3, 3]
    assert bench.level_split(8) == [4, 4]
    assert bench.level_split(5) == [3, 2]
    assert bench.level_split(4) == [4]


def test_work_per_element_2e20_forward():
    w = bench.algorithmic_work([10, 10], kind=0)
    # pass 0: 3 merges + 2 level twiddles (Shoup) + pass twiddle from the table (Montgomery)
    assert w[0]["mads"] == inter(3) + 162 and w[0]["hbm_bytes"] == 96
    # pass 1 (last, forward): 3 merges + 2 level twiddles, no epilogue
    assert w[1]["mads"] == inter(3) and w[1]["hbm_bytes"] == 64
    # even/odd split: rho/2 MFMAs of 32x32x32 per 32 vectors and output pair
    assert all(p["mfma_ops"] == 1024 * (16 + 8 + 8) for p in w)


def test_work_epilogues_and_large_passes():
    # N^-1 rides in the first pass's twiddle table: no product in the last pass
    inv = bench.algorithmic_work([12, 12], kind=1)
    assert inv[1]["mads"] == inter(3)
    cinv = bench.algorithmic_work([12, 12], kind=3)
    assert cinv[1]["mads"] == inter(3) + 162         # g^-K from the table's tail
    assert bench.algorithmic_work([6, 5, 5], kind=3)[2]["mads"] == inter(2) + 2 * 162
    # a single pass (no table) and a plan above the table limit keep it
    assert bench.algorithmic_work([12], kind=1)[0]["mads"] == inter(3) + 162
    assert bench.algorithmic_work([12], kind=3)[0]["mads"] == inter(3) + 3 * 162
    assert bench.algorithmic_work([9, 9, 8], kind=1)[2]["mads"] == inter(2) + 162
    coset = bench.algorithmic_work([12, 12], kind=2)
    assert coset[0]["mads"] == inter(3) + 162 + 162        # + coset pre-scale (table)
    assert bench.algorithmic_work([12], kind=2)[0]["mads"] == inter(3) + 2 * 162
    # above the table limit the pass twiddle takes two products and no table read
    big = bench.algorithmic_work([10, 9, 9], kind=0)
    assert big[0]["mads"] == inter(3) + 2 * 162 and big[0]["hbm_bytes"] == 64


def test_traffic_only_for_the_profiled_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "not-the-profiled-sources")
    assert bench.measured_traffic() is None


def test_msm_product_count():
    # 4 points, 1-bit windows: K = 256; prep 20, accumulation 7 * 4 * 256,
    # reduction 256 * 1 * 35, merge 256 * (8 + 10) + 6
    assert bench.msm_products(4, 1) == 16 + 7168 + 8960 + 4614
    # accumulation dominates at the benchmark's size
    n, c = 1 << 22, 16
    assert 7 * n * 16 / bench.msm_products(n, c) > 0.85
