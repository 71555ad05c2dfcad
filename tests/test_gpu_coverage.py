"""Configurations beyond the basic parity sweep, each bit-exact against the C
oracle: every kind at 2^20 in both forms, the butterfly coset round trip at
2^24, the split-table twiddle path (FRNTT_SPLIT_TWIDDLES and sizes above the
pass-table limit), a 2^26 transform, the server at 2^19..2^22 and with
two-pass plans at 2^12, and the behaviour under a hipGraph stream capture."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import cref

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402

pytestmark = pytest.mark.gpu

ALGOS = [fr.ALGO_BUTTERFLY, fr.ALGO_FOURSTEP_MFMA]
ALGO_IDS = ["butterfly", "mfma"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64).copy()).to("cuda:0")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64).reshape(-1, 4)


def run(ctx, x, log_n, kind, algo=None, batch=1):
    t = to_dev(x)
    ctx.transform_checked(t.data_ptr(), log_n, batch, kind, torch.cuda.current_stream().cuda_stream, algo)
    torch.cuda.synchronize()
    return to_host(t)


@pytest.fixture(scope="module")
def ctx24():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=24)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_2e20_every_kind_both_forms(ctx24, algo, kind):
    _say(f"2^20 kind={kind} algo={algo}")
    x = si.polynomial(2, 20)
    assert np.array_equal(run(ctx24, x, 20, kind, algo), cref.transform(x, 20, kind))


def test_2e24_butterfly_coset_roundtrip_full(ctx24):
    """2^24 coset NTT then coset INTT in the butterfly form, every output."""
    _say("2^24 butterfly coset -> coset_inv")
    x = si.polynomial(3, 24)
    t = to_dev(x)
    s = torch.cuda.current_stream().cuda_stream
    ctx24.transform_checked(t.data_ptr(), 24, 1, fr.COSET, s, fr.ALGO_BUTTERFLY)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), cref.transform(x, 24, 2))
    ctx24.transform_checked(t.data_ptr(), 24, 1, fr.COSET_INV, s, fr.ALGO_BUTTERFLY)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), x)


def test_2e24_inverse_kinds_mfma(ctx24):
    """2^24 INTT and coset INTT (MFMA form) on fresh inputs, every output."""
    x = si.polynomial(1003, 24)
    for kind in (fr.INV, fr.COSET_INV):
        _say(f"2^24 kind={kind} mfma")
        assert np.array_equal(run(ctx24, x, 24, kind, fr.ALGO_FOURSTEP_MFMA), cref.transform(x, 24, kind))


# ------------------------------------------------------ split-table twiddles

@pytest.fixture(scope="module")
def ctx_split():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=20, flags=fr.frntt.SPLIT_TWIDDLES)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
@pytest.mark.parametrize("plan", [[8, 8], [4, 12], [12, 4], [6, 5, 5], [4, 6, 6]])
def test_split_twiddles_every_kind(ctx_split, algo, plan):
    """Without pass-twiddle tables every pass twiddle and coset factor comes
    from the split tables (two products): the matrix form's pass-twiddle level
    with split-table twiddles, the butterfly's store-time twiddle, the coset
    pre-scale from split tables, and the N^-1 / g^-k epilogues of the last pass."""
    _say(f"split twiddles algo={algo} plan={plan}")
    ctx_split.set_plan(algo, 16, plan)
    try:
        x = np.concatenate([si.polynomial(41, 16, stream=s) for s in range(2)])
        for kind in range(4):
            assert np.array_equal(run(ctx_split, x, 16, kind, algo, batch=2), cref.transform(x, 16, kind)), kind
        assert ctx_split.table_bytes() < 8 << 20     # no N-entry tables were built
    finally:
        ctx_split.set_plan(algo, 16, [])


def test_split_twiddles_2e20(ctx_split):
    x = si.polynomial(42, 20)
    for kind in (fr.FWD, fr.COSET_INV):
        _say(f"split twiddles 2^20 kind={kind}")
        assert np.array_equal(run(ctx_split, x, 20, kind, fr.ALGO_FOURSTEP_MFMA), cref.transform(x, 20, kind))


def test_2e26_above_the_table_limit():
    """2^26 (three passes, above the 2^25-entry pass-table limit, so the pass
    twiddles come from the split tables): sampled outputs against the
    definition and the round trip, both forms."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=26)
    try:
        x = si.polynomial(26, 26)
        rng = np.random.default_rng(26)
        ks = [0, 1, (1 << 26) - 1] + [int(k) for k in rng.integers(0, 1 << 26, 2)]
        for algo in ALGOS:
            _say(f"2^26 algo={algo}")
            t = to_dev(x)
            s = torch.cuda.current_stream().cuda_stream
            c.transform_checked(t.data_ptr(), 26, 1, fr.FWD, s, algo)
            torch.cuda.synchronize()
            y = to_host(t)
            for k in ks:
                assert np.array_equal(y[k], cref.eval_output(x, 26, k, 0)), (algo, k)
            c.transform_checked(t.data_ptr(), 26, 1, fr.INV, s, algo)
            torch.cuda.synchronize()
            assert np.array_equal(to_host(t), x)
            del t
    finally:
        torch.cuda.synchronize()
        c.close()


# ------------------------------------------------------------------ server

def _fetch(srv, ticket, log_n):
    out = np.zeros(((1 << log_n), 4), dtype=np.uint64)
    srv.result(ticket, out.ctypes.data_as(ctypes.c_void_p).value)
    return out


def test_server_large_sizes_mix_and_alone():
    """Requests of 2^19..2^22 (the upper half of the serving mix), every kind,
    submitted together: each result equals the oracle and the same transform
    run alone."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=22)
    srv = fr.Server(c, 16 << 30, slots=4)
    try:
        reqs = [(19, 0), (22, 1), (20, 2), (21, 3), (19, 3), (22, 2), (21, 0), (20, 1)]
        tickets = [srv.submit(kind, l, 9) for l, kind in reqs]
        srv.drain(300)
        st = srv.stats()
        _say(f"server stats {st}")
        for (l, kind), tk in zip(reqs, tickets):
            got = _fetch(srv, tk, l)
            x = si.polynomial(9, l, stream=tk)
            assert np.array_equal(got, cref.transform(x, l, kind)), (l, kind)
            assert np.array_equal(run(c, x, l, kind), got), (l, kind)
    finally:
        srv.close()
        torch.cuda.synchronize()
        c.close()


def test_server_two_pass_plan_at_2e12():
    """A two-pass plan for a size of one tile: the request buffer carries the
    scratch the plan needs, fixed when the request is submitted."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=14)
    try:
        for algo in ALGOS:
            c.set_plan(algo, 12, [6, 6])
        srv = fr.Server(c, 1 << 30, slots=2)
        try:
            tks = [srv.submit(kind, 12, 77) for kind in range(4)] + [srv.submit(0, 10, 77)]
            srv.drain(60)
            for kind, tk in enumerate(tks[:4]):
                x = si.polynomial(77, 12, stream=tk)
                assert np.array_equal(_fetch(srv, tk, 12), cref.transform(x, 12, kind)), kind
            x = si.polynomial(77, 10, stream=tks[4])
            assert np.array_equal(_fetch(srv, tks[4], 10), cref.transform(x, 10, 0))
        finally:
            srv.close()
    finally:
        torch.cuda.synchronize()
        c.close()


# --------------------------------------------------------------- capture

def test_transform_under_stream_capture():
    """Inside a hipGraph capture a transform that would have to build its
    twiddle table or allocate scratch refuses (FRNTT_ESTATE, nothing
    enqueued); after frntt_prepare and one transform on the stream the same
    call captures, and every replay of the graph is exact."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=16)
    try:
        x = si.polynomial(55, 16)
        t = to_dev(x)
        s = torch.cuda.Stream()
        L = fr.lib()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                rc = L.ntt_fwd(c.handle, t.data_ptr(), 16, 1, s.cuda_stream)
        assert rc == fr.frntt.ESTATE
        torch.cuda.synchronize()
        assert np.array_equal(to_host(t), x)            # nothing ran
        c.prepare(16, fr.FWD)
        with torch.cuda.stream(s):
            c.transform_checked(t.data_ptr(), 16, 1, fr.FWD, s.cuda_stream)     # allocates the scratch
        torch.cuda.synchronize()
        want = cref.transform(x, 16, 0)
        assert np.array_equal(to_host(t), want)
        g2 = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g2, stream=s):
                rc = L.ntt_fwd(c.handle, t.data_ptr(), 16, 1, s.cuda_stream)
        assert rc == 0
        for _ in range(3):
            t.copy_(to_dev(x))
            torch.cuda.synchronize()
            g2.replay()
            torch.cuda.synchronize()
            assert np.array_equal(to_host(t), want)
    finally:
        torch.cuda.synchronize()
        c.close()


# ------------------------------------------------ HBM-level 5-step (3 passes)

@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
def test_three_pass_2e22_every_kind(algo):
    """The recursive 5-step form (Eq. 1) as three HBM passes at 2^22, every kind."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=22)
    try:
        c.set_plan(algo, 22, [8, 7, 7])
        x = si.polynomial(22, 22)
        for kind in range(4):
            _say(f"3-pass 2^22 algo={algo} kind={kind}")
            assert np.array_equal(run(c, x, 22, kind, algo), cref.transform(x, 22, kind)), kind
    finally:
        torch.cuda.synchronize()
        c.close()


def test_three_pass_2e24_every_kind(ctx24):
    """Three HBM passes of 2^8 at 2^24, every kind, both forms, every output."""
    x = si.polynomial(1024, 24)
    for kind in range(4):
        want = cref.transform(x, 24, kind)
        for algo in ALGOS:
            _say(f"3-pass 2^24 algo={algo} kind={kind}")
            ctx24.set_plan(algo, 24, [8, 8, 8])
            try:
                assert np.array_equal(run(ctx24, x, 24, kind, algo), want), (algo, kind)
            finally:
                ctx24.set_plan(algo, 24, [])
