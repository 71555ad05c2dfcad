"""The allocation-free entry point (ntt_transform_noalloc) against
ntt_transform: two calls in a row, the second on a smaller input, every kind
and both forms; bit-exact, and checked against the oracle."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import cref

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64).copy()).to("cuda:0")


def _host(t):
    return t.cpu().numpy().view(np.uint64).reshape(-1, 4)


@pytest.mark.parametrize("algo", [fr.ALGO_BUTTERFLY, fr.ALGO_FOURSTEP_MFMA], ids=["butterfly", "mfma"])
def test_noalloc_matches_transform_two_calls(algo):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=20)
    L = fr.lib()
    try:
        c.set_algo(algo)
        s = torch.cuda.current_stream().cuda_stream
        for log_n, batch, seed in ((18, 2, 61), (13, 1, 62)):    # second call smaller
            x = np.concatenate([si.polynomial(seed, log_n, stream=b) for b in range(batch)])
            for kind in range(4):
                print(f"noalloc algo={algo} log_n={log_n} batch={batch} kind={kind}", flush=True)
                a, b = _dev(x), _dev(x)
                assert L.ntt_transform_noalloc(c.handle, a.data_ptr(), log_n, batch, kind, s) == 0
                assert L.ntt_transform(c.handle, b.data_ptr(), log_n, batch, kind, s) == 0
                torch.cuda.synchronize()
                got = _host(a)
                assert np.array_equal(got, _host(b)), (log_n, kind)
                assert np.array_equal(got, cref.transform(x, log_n, kind)), (log_n, kind)
        # sizes beyond the static scratch are refused, nothing enqueued
        t = torch.zeros(((1 << 20), 4), dtype=torch.int64, device="cuda:0")
        assert L.ntt_transform_noalloc(c.handle, t.data_ptr(), 20, 2, 0, s) == fr.frntt.ERANGE
        assert L.ntt_transform_noalloc(c.handle, t.data_ptr() + 8, 10, 1, 0, s) == fr.frntt.EALIGN
    finally:
        torch.cuda.synchronize()
        c.close()
