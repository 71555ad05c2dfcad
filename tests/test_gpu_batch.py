"""Uneven batches (one persistent launch), hipGraph replay and the autotuner:
bit-exact against the CPU oracle, and identical alone and in the mix."""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import cref

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=22)
    yield c
    torch.cuda.synchronize()
    c.close()


def host(t):
    return t.cpu().numpy().view(np.uint64).reshape(-1, 4)


def make_jobs(ctx, seed, sizes, kinds):
    """Device buffers filled by the device generator (stream = job index)."""
    bufs = []
    for j, l in enumerate(sizes):
        t = torch.empty((1 << l, 4), dtype=torch.int64, device="cuda:0")
        ctx.generate(t.data_ptr(), seed, j, 0, 1 << l)
        bufs.append(t)
    jobs = [(b.data_ptr(), l, k) for b, l, k in zip(bufs, sizes, kinds)]
    return bufs, jobs


def expect(seed, j, l, k):
    return cref.transform(si.polynomial(seed, l, stream=j), l, k)


def test_batch_mixed_small(ctx):
    sizes = [13, 10, 16, 1, 0, 12, 14, 8, 11, 15, 9, 2]
    kinds = [0, 1, 2, 3, 0, 2, 3, 1, 0, 1, 2, 3]
    _say("batch mixed small")
    bufs, jobs = make_jobs(ctx, 21, sizes, kinds)
    ctx.batch(jobs)
    torch.cuda.synchronize()
    for j, (l, k) in enumerate(zip(sizes, kinds)):
        assert np.array_equal(host(bufs[j]), expect(21, j, l, k)), (j, l, k)


def test_batch_alone_equals_mix(ctx):
    sizes = [14, 12, 16, 12, 10]
    kinds = [0, 2, 1, 3, 0]
    bufs, jobs = make_jobs(ctx, 22, sizes, kinds)
    ctx.batch(jobs)
    torch.cuda.synchronize()
    for j, (l, k) in enumerate(zip(sizes, kinds)):
        t = torch.empty((1 << l, 4), dtype=torch.int64, device="cuda:0")
        ctx.generate(t.data_ptr(), 22, j, 0, 1 << l)
        ctx.transform_checked(t.data_ptr(), l, 1, k)
        torch.cuda.synchronize()
        assert np.array_equal(host(t), host(bufs[j]))


def test_batch_errors(ctx):
    t = torch.empty((1024, 4), dtype=torch.int64, device="cuda:0")
    with pytest.raises(fr.FrnttError) as e:
        ctx.batch([(t.data_ptr() + 8, 10, 0)])
    assert e.value.status == fr.frntt.EALIGN
    with pytest.raises(fr.FrnttError) as e:
        ctx.batch([(t.data_ptr(), 23, 0)])
    assert e.value.status == fr.frntt.ERANGE
    with pytest.raises(fr.FrnttError) as e:
        ctx.batch([(t.data_ptr(), 10, 5)])
    assert e.value.status == fr.frntt.EINVAL
    ctx.batch([])                                            # empty batch: no-op


def test_c4_uneven_256_graph(ctx):
    """256 forward NTTs, sizes uniform over 2^12..2^20 (seed 4), one persistent
    launch captured in a hipGraph. The first replay is checked on every job
    against the oracle; later replays (inputs regenerated eagerly in between)
    and the same batch without the graph on a sample."""
    sizes = si.uneven_batch_sizes(4, 256, 12, 20)
    kinds = [0] * 256
    _say(f"c4: {sum(1 << l for l in sizes)} elements in 256 jobs")
    bufs, jobs = make_jobs(ctx, 4, sizes, kinds)
    ctx.batch(jobs, graph=True)
    torch.cuda.synchronize()
    got = [host(b) for b in bufs]
    _say("c4: first replay done, checking all 256 jobs")
    for j, l in enumerate(sizes):
        assert np.array_equal(got[j], expect(4, j, l, 0)), (j, l)
    del got
    rng = np.random.default_rng(4)
    sample = sorted(set(rng.choice(256, 10, replace=False).tolist()) | {int(np.argmax(sizes)),
                                                                          int(np.argmin(sizes))})
    wants = {j: expect(4, j, sizes[j], 0) for j in sample}
    for replay in range(1, 3):
        for j, l in enumerate(sizes):                  # eager regeneration between replays
            ctx.generate(bufs[j].data_ptr(), 4, j, 0, 1 << l)
        torch.cuda.synchronize()
        ctx.batch(jobs, graph=True)
        torch.cuda.synchronize()
        for j in sample:
            assert np.array_equal(host(bufs[j]), wants[j]), (replay, j, sizes[j])
    # the same batch without the graph gives the same bytes
    for j, l in enumerate(sizes):
        ctx.generate(bufs[j].data_ptr(), 4, j, 0, 1 << l)
    ctx.batch(jobs)
    torch.cuda.synchronize()
    for j in sample:
        assert np.array_equal(host(bufs[j]), wants[j])


def test_autotuner(ctx, tmp_path):
    _say("autotune 2^16")
    algo, passes, ms = ctx.tune(16, 2)
    assert algo in (fr.ALGO_BUTTERFLY, fr.ALGO_FOURSTEP_MFMA) and passes >= 1 and ms > 0
    plan = ctx.get_plan(fr.ALGO_AUTO, 16)
    assert sum(plan) == 16
    x = np.concatenate([si.polynomial(31, 16, stream=s) for s in range(2)])
    t = torch.from_numpy(x.view(np.int64).copy()).to("cuda:0")
    ctx.transform_checked(t.data_ptr(), 16, 2, fr.FWD)      # uses the tuned choice
    torch.cuda.synchronize()
    assert np.array_equal(host(t), cref.transform(x, 16, 0))
    path = str(tmp_path / "tune.json")
    ctx.tune_save(path)
    doc = json.load(open(path))
    assert doc["format"] == "frntt-tune-1"
    ent = [e for e in doc["entries"] if e["log_n"] == 16][0]
    assert sum(ent["passes"]) == 16 and ent["algo"] == algo
    assert len(ent["levels"]) == len(ent["passes"])
    c2 = fr.Context(0, max_log_n=16)
    try:
        c2.tune_load(path)
        assert c2.get_plan(fr.ALGO_AUTO, 16) == plan
    finally:
        c2.close()


def test_tuned_level_split_single_and_batch(ctx, tmp_path):
    """A tuned plan with non-default level orders ([4,3,3] and [3,3,4] in the
    two 2^10 passes of 2^20) is used by single transforms and by batches, and
    both stay bit-exact."""
    path = str(tmp_path / "tune20.json")
    with open(path, "w") as fh:
        json.dump({"format": "frntt-tune-1", "entries": [
            {"log_n": 20, "algo": 2, "passes": [10, 10], "ms": 0.1, "levels": [[4, 3, 3], [3, 3, 4]]}]}, fh)
    c = fr.Context(0, max_log_n=20)
    try:
        assert c.get_plan_levels(fr.ALGO_AUTO, 20, 0) == [3, 4, 3]         # default split
        c.tune_load(path)
        assert c.get_plan(fr.ALGO_AUTO, 20) == [10, 10]
        assert c.get_plan_levels(fr.ALGO_AUTO, 20, 0) == [4, 3, 3]
        assert c.get_plan_levels(fr.ALGO_AUTO, 20, 1) == [3, 3, 4]
        x = si.polynomial(33, 20)
        for kind in (fr.FWD, fr.COSET_INV):
            _say(f"tuned levels 2^20 kind={kind}")
            t = torch.from_numpy(x.view(np.int64).copy()).to("cuda:0")
            c.transform_checked(t.data_ptr(), 20, 1, kind)
            torch.cuda.synchronize()
            assert np.array_equal(host(t), cref.transform(x, 20, kind))
        bufs, jobs = make_jobs(c, 34, [20, 14, 20], [0, 1, 3])
        c.batch(jobs)
        torch.cuda.synchronize()
        for j, (l, k) in enumerate(zip([20, 14, 20], [0, 1, 3])):
            assert np.array_equal(host(bufs[j]), expect(34, j, l, k)), (j, l, k)
    finally:
        torch.cuda.synchronize()
        c.close()
