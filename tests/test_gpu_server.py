"""Continuous-batching server: every result bit-exact against the oracle and
identical to the same transform run alone; admission respects the budget."""
from __future__ import annotations

import ctypes
import sys
import time

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
    c = fr.Context(0, max_log_n=20)
    yield c
    torch.cuda.synchronize()
    c.close()


def fetch(srv, ticket, log_n):
    out = np.zeros(((1 << log_n), 4), dtype=np.uint64)
    srv.result(ticket, out.ctypes.data_as(ctypes.c_void_p).value)
    return out


def test_server_mix_matches_oracle_and_alone(ctx):
    srv = fr.Server(ctx, 4 << 30, slots=4)
    try:
        reqs = si.request_stream(5, 60, 10, 17, rate_per_s=3000.0)
        tickets = []
        t0 = time.perf_counter()
        for r in reqs:                        # paced arrivals: later ones land on running batches
            while time.perf_counter() - t0 < r["t_arrive_s"]:
                pass
            tickets.append(srv.submit(r["kind"], r["log_n"], 5))
        srv.drain(120)
        st = srv.stats()
        _say(f"server stats {st}")
        assert st["completed"] == len(reqs)
        for r, tk in zip(reqs, tickets):
            done, lat = srv.poll(tk)
            assert done and lat > 0
            got = fetch(srv, tk, r["log_n"])
            x = si.polynomial(5, r["log_n"], stream=tk)           # data = f(seed, request id)
            assert np.array_equal(got, cref.transform(x, r["log_n"], r["kind"])), (tk, r)
            # the same transform alone, through the plain entry point
            t = torch.empty((1 << r["log_n"], 4), dtype=torch.int64, device="cuda:0")
            ctx.generate(t.data_ptr(), 5, tk, 0, 1 << r["log_n"])
            ctx.transform_checked(t.data_ptr(), r["log_n"], 1, r["kind"])
            torch.cuda.synchronize()
            assert np.array_equal(t.cpu().numpy().view(np.uint64).reshape(-1, 4), got)
    finally:
        srv.close()


def test_server_two_pass_plan_at_2e12():
    """A 2^12 request under a two-pass plan needs a scratch region although
    its size fits one tile; the server sizes it from the plan that runs."""
    c = fr.Context(0, max_log_n=14)
    try:
        for algo in (fr.ALGO_FOURSTEP_MFMA, fr.ALGO_BUTTERFLY):
            c.set_plan(algo, 12, [6, 6])
        srv = fr.Server(c, 1 << 30, slots=2)
        try:
            kinds = [fr.FWD, fr.INV, fr.COSET, fr.COSET_INV] * 3
            tickets = [srv.submit(k, 12, 9) for k in kinds]
            srv.drain(60)
            for k, tk in zip(kinds, tickets):
                got = fetch(srv, tk, 12)
                x = si.polynomial(9, 12, stream=tk)
                assert np.array_equal(got, cref.transform(x, 12, k)), (tk, k)
        finally:
            srv.close()
        assert c.get_plan(fr.ALGO_FOURSTEP_MFMA, 12) == [6, 6]
    finally:
        torch.cuda.synchronize()
        c.close()


def test_server_release_on_done(ctx):
    srv = fr.Server(ctx, 1 << 30, slots=2)
    try:
        srv.set_release_on_done(True)
        tks = [srv.submit(k % 3, 14, 3) for k in range(40)]
        srv.drain(60)
        for tk in tks:
            done, lat = srv.poll(tk)
            assert done and lat > 0
        with pytest.raises(fr.FrnttError) as e:
            fetch(srv, tks[0], 14)                    # buffer already recycled
        assert e.value.status == fr.frntt.ESTATE
    finally:
        srv.close()


def test_server_destroy_cancels_queued(ctx):
    ctx.prepare(16, 0)
    srv = fr.Server(ctx, ctx.table_bytes() + (5 << 20), slots=1)
    for k in range(6):
        srv.submit(0, 16, 2)                          # only one fits; the rest stay queued
    time.sleep(0.2)
    srv.close()                                       # must return: queued requests are cancelled


def test_server_budget_and_errors(ctx):
    for kind in range(3):
        ctx.prepare(16, kind)                         # tables the requests below use
    tables = ctx.table_bytes()
    budget = tables + (6 << 20)
    srv = fr.Server(ctx, budget, slots=2)
    try:
        with pytest.raises(fr.FrnttError) as e:
            srv.submit(0, 20, 1)                      # 32 MiB + scratch alone exceeds the budget
        assert e.value.status == fr.frntt.EBUSY
        tks = [srv.submit(k % 3, 16, 9) for k in range(12)]   # 4 MiB each: must queue
        # finished results hold the budget until the client takes them: drain
        # reports the stall instead of waiting
        t0 = time.perf_counter()
        with pytest.raises(fr.FrnttError) as e:
            srv.drain(60)
        assert e.value.status == fr.frntt.EBUSY and time.perf_counter() - t0 < 30
        for i, tk in enumerate(tks):                  # consume in order: frees room for the rest
            deadline = time.perf_counter() + 60
            while not srv.poll(tk)[0]:
                assert time.perf_counter() < deadline
                time.sleep(0.001)
            got = fetch(srv, tk, 16)
            x = si.polynomial(9, 16, stream=tk)
            assert np.array_equal(got, cref.transform(x, 16, i % 3))
        st = srv.stats()
        assert st["completed"] == 12
        assert st["peak_bytes"] <= budget
        with pytest.raises(fr.FrnttError) as e:
            srv.poll(tks[0])                          # released by result()
        assert e.value.status == fr.frntt.ESTATE
        with pytest.raises(fr.FrnttError):
            srv.submit(7, 10, 1)                      # bad kind
        with pytest.raises(fr.FrnttError):
            srv.release(123456)                       # unknown ticket
    finally:
        srv.close()


def test_server_poisson_mix_at_scale(ctx):
    """400 Poisson-paced requests, NTT/INTT/coset-NTT 40/40/20, sizes
    2^14..2^18 (seed 15): every result bit-exact against the oracle, and a
    seeded sample of 100 identical when the same transform runs alone."""
    srv = fr.Server(ctx, 8 << 30, slots=4)          # all 400 results stay resident until fetched
    try:
        reqs = si.request_stream(15, 400, 14, 18, rate_per_s=3000.0)
        tickets = []
        t0 = time.perf_counter()
        for r in reqs:
            while time.perf_counter() - t0 < r["t_arrive_s"]:
                pass
            tickets.append(srv.submit(r["kind"], r["log_n"], 15))
        srv.drain(300)
        st = srv.stats()
        _say(f"server at scale: {st}")
        assert st["completed"] == len(reqs) and st["batches"] >= 1
        sample = {si.draw_u64(15, (1 << 23) + 99, j) % len(reqs) for j in range(100)}
        threads = cref.max_threads()
        for i, (r, tk) in enumerate(zip(reqs, tickets)):
            done, lat = srv.poll(tk)
            assert done and lat > 0
            got = fetch(srv, tk, r["log_n"])
            x = si.polynomial(15, r["log_n"], stream=tk)
            assert np.array_equal(got, cref.transform(x, r["log_n"], r["kind"], threads=threads)), (tk, r)
            if i in sample:
                t = torch.empty((1 << r["log_n"], 4), dtype=torch.int64, device="cuda:0")
                ctx.generate(t.data_ptr(), 15, tk, 0, 1 << r["log_n"])
                ctx.transform_checked(t.data_ptr(), r["log_n"], 1, r["kind"])
                torch.cuda.synchronize()
                assert np.array_equal(t.cpu().numpy().view(np.uint64).reshape(-1, 4), got), (tk, r)
    finally:
        srv.close()
