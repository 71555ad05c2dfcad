"""Host-side logic of the MSM calls, without a device: the window width
frntt_msm picks, the scratch it reports, and the argument errors that are
returned before anything touches the GPU."""
from __future__ import annotations

import ctypes

import paper_2604_17808_amd as fr
from paper_2604_17808_amd import frntt as B


def _windows(c):
    return -(-256 // c)


def test_window_widths():
    ws = [fr.msm_window(1 << k) for k in range(0, 27)]
    assert all(1 <= w <= 20 for w in ws)
    # never narrower for more points
    assert ws == sorted(ws)
    # the measured widths at the benchmark's sizes
    assert [fr.msm_window(1 << k) for k in (20, 22, 24, 26)] == [15, 16, 16, 20]
    # a size between powers of two takes the width of its floor(log2)
    assert fr.msm_window((1 << 22) + 12345) == fr.msm_window(1 << 22)
    assert fr.lib().frntt_msm_window(-1) == B.EINVAL


def test_small_sizes_follow_the_addition_model():
    # below 2^13 points: the c that minimises K (n + 5 2^c)
    for n in (0, 1, 2, 17, 100, 1000, 4096, 8191):
        cost = {c: _windows(c) * (n + 5 * (1 << c)) for c in range(1, 21)}
        best = min(cost.values())
        assert cost[fr.msm_window(n)] == best, n


def test_workspace_bytes():
    sizes = [fr.msm_workspace_bytes(1 << k) for k in (10, 14, 18, 20, 22)]
    assert all(b > 0 for b in sizes) and sizes == sorted(sizes)
    for k in (16, 20, 22):
        n = 1 << k
        c = fr.msm_window(n)
        K = _windows(c)
        # at least the prepared points (128 B each), the sorted entries and
        # the sort keys (4 B per point and window), and two (B, W) pairs of
        # extended points per bucket
        assert fr.msm_workspace_bytes(n) >= n * 128 + 3 * K * n * 4 + 4 * (K << c) * 128
        assert fr.msm_workspace_bytes(n, c) == fr.msm_workspace_bytes(n)
    assert fr.msm_workspace_bytes(-1) == 0
    assert fr.msm_workspace_bytes(10, 21) == 0
    assert fr.msm_workspace_bytes((1 << 26) + 1) == 0


def test_argument_errors_without_device():
    L = fr.lib()
    vp = ctypes.c_void_p
    assert L.frntt_msm(None, None, None, 1, 0, None, None) == B.EINVAL
    assert L.frntt_msm_presort(None, None, None, 1, 0, None, None) == B.EINVAL
    assert L.frntt_ec_mul(None, None, None, 1, None, None) == B.EINVAL
    assert L.frntt_msm_batch(None, None, None, None, 1, 0, None, None) == B.EINVAL
    one = (vp * 1)(None)
    n = (ctypes.c_int64 * 1)(1)
    assert L.frntt_msm_batch(None, one, one, n, 1, 0, one, None) == B.EINVAL
