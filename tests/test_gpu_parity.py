"""Parity of the HIP transforms with the CPU oracle, bit-exact (error 0).

Every call goes through the C ABI (ctypes binding); device memory comes from
torch. Inputs are the seeded uniform elements of [0, r). Expected values come
from the C oracle (oracle/ntt_ref.c), itself pinned in test_oracle_pins.py.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import cref

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402

pytestmark = pytest.mark.gpu

R = si.modulus()
ALGOS = [fr.ALGO_BUTTERFLY, fr.ALGO_FOURSTEP_MFMA]
ALGO_IDS = ["butterfly", "mfma"]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = fr.Context(0, max_log_n=24)
    yield c
    torch.cuda.synchronize()
    c.close()


def to_dev(x: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(x).view(np.int64).copy()).to("cuda:0")


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64).reshape(-1, 4)


def run(ctx, x: np.ndarray, log_n: int, kind: int, algo=None, batch=None):
    batch = batch if batch is not None else x.shape[0] >> log_n
    t = to_dev(x)
    stream = torch.cuda.current_stream().cuda_stream
    ctx.transform_checked(t.data_ptr(), log_n, batch, kind, stream, algo)
    torch.cuda.synchronize()
    return to_host(t)


def inputs(seed, log_n, batch):
    return np.concatenate([si.polynomial(seed, log_n, stream=s) for s in range(batch)])


# ------------------------------------------------------------ small sizes

@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
def test_c1_n1024_fwd_inv_roundtrip(ctx, algo):
    """N = 2^10 forward then inverse (seed 1), bit-exact and round trip."""
    _say(f"c1 algo={algo}")
    x = si.polynomial(1, 10)
    X = run(ctx, x, 10, fr.FWD, algo)
    assert np.array_equal(X, cref.transform(x, 10, 0))
    back = run(ctx, X, 10, fr.INV, algo)
    assert np.array_equal(back, x)


@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("log_n", [1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12, 13, 14, 15, 16])
def test_sizes_and_kinds(ctx, algo, kind, log_n):
    batch = 3 if log_n <= 12 else 2
    _say(f"sizes algo={algo} kind={kind} log_n={log_n} batch={batch}")
    x = inputs(100 + log_n, log_n, batch)
    got = run(ctx, x, log_n, kind, algo)
    want = cref.transform(x, log_n, kind)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
@pytest.mark.parametrize("batch", [1, 2, 4, 5, 8, 16])
def test_batch_counts(ctx, algo, batch):
    _say(f"batch algo={algo} batch={batch}")
    x = inputs(7, 10, batch)
    assert np.array_equal(run(ctx, x, 10, fr.FWD, algo), cref.transform(x, 10, 0))


@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
@pytest.mark.parametrize("plan", [[8, 8], [10, 6], [6, 10], [4, 12], [12, 4], [4, 6, 6], [6, 5, 5],
                                  [2, 2, 12], [11, 5], [5, 11], [9, 7], [7, 9]])
def test_plans_bit_identical(ctx, algo, plan):
    """Every pass split of 2^16 gives the same bytes as the oracle."""
    _say(f"plan algo={algo} plan={plan}")
    ctx.set_plan(algo, 16, plan)
    try:
        x = inputs(11, 16, 2)
        for kind in range(4):
            assert np.array_equal(run(ctx, x, 16, kind, algo), cref.transform(x, 16, kind))
    finally:
        ctx.set_plan(algo, 16, [])


def test_first_pass_tables_per_kind():
    """The first pass's twiddle table differs per kind: an inverse kind's
    entries carry N^-1; a forward coset kind's carry the line's g^rest and it
    ends with 2^l0 pre-scale entries; a two-pass coset INTT's carry N^-1 g^-k
    and it ends with 2^l1 epilogue entries. A single-pass transform builds
    none. Every kind stays exact."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _say("pass tables per kind")
    c = fr.Context(0, max_log_n=20)
    try:
        plan = c.get_plan(fr.ALGO_AUTO, 16)
        assert len(plan) == 2                    # one table of 2^16 entries
        t, tail, tail_inv = 32 << 16, 32 << plan[0], 32 << plan[1]
        sizes = []
        for kind in (fr.FWD, fr.COSET, fr.INV, fr.COSET_INV):
            c.prepare(16, kind)
            sizes.append(c.table_bytes())
        base = sizes[0] - t
        assert sizes == [base + t, base + 2 * t + tail, base + 3 * t + tail, base + 4 * t + tail + tail_inv]
        c.prepare(12, fr.INV)
        assert c.table_bytes() == sizes[-1]
        x = inputs(12, 16, 1)
        for kind in range(4):
            assert np.array_equal(run(c, x, 16, kind), cref.transform(x, 16, kind))
        assert c.table_bytes() == sizes[-1]      # the transforms used the prepared tables
    finally:
        torch.cuda.synchronize()
        c.close()


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
@pytest.mark.parametrize("log_n,batch", [(12, 1), (11, 2), (10, 4), (9, 8), (8, 16), (7, 32), (6, 64), (5, 128),
                                         (11, 4), (10, 2)])
def test_full_tile_level_shapes(ctx, log_n, batch, kind):
    """Single-pass transforms whose lines fill a 4096-element tile: every
    level split of the matrix form (radix 2^5 .. 2^12) and every epilogue."""
    _say(f"tile shapes log_n={log_n} batch={batch} kind={kind}")
    x = inputs(200 + log_n, log_n, batch)
    got = run(ctx, x, log_n, kind, fr.ALGO_FOURSTEP_MFMA)
    assert np.array_equal(got, cref.transform(x, log_n, kind))


@pytest.mark.parametrize("pattern", ["zeros", "rminus1", "onehot", "alternating"])
def test_adversarial_inputs(ctx, pattern):
    n = 1 << 14
    if pattern == "zeros":
        v = np.zeros((n, 4), dtype=np.uint64)
    elif pattern == "rminus1":
        v = np.repeat(si.from_ints([R - 1]), n, axis=0)
    elif pattern == "onehot":
        v = np.zeros((n, 4), dtype=np.uint64)
        v[12345] = si.from_ints([R - 1])[0]
    else:
        v = np.repeat(si.from_ints([1, R - 1]), n // 2, axis=0)
    _say(f"adversarial {pattern}")
    for algo in ALGOS:
        for kind in range(4):
            assert np.array_equal(run(ctx, v, 14, kind, algo), cref.transform(v, 14, kind))


# ---------------------------------------------------------- full sizes

@pytest.mark.parametrize("algo", ALGOS, ids=ALGO_IDS)
def test_c2_n2pow20_forward(ctx, algo):
    """N = 2^20 forward (seed 2): butterfly and four-step MFMA, bit-exact."""
    _say(f"c2 algo={algo}")
    x = si.polynomial(2, 20)
    got = run(ctx, x, 20, fr.FWD, algo)
    assert np.array_equal(got, cref.transform(x, 20, 0))


def test_c3_n2pow24_coset_roundtrip(ctx):
    """N = 2^24 coset NTT (g = 5) then its inverse (seed 3), MFMA form."""
    _say("c3 2^24 coset -> coset_inv (mfma)")
    x = si.polynomial(3, 24)
    t = to_dev(x)
    stream = torch.cuda.current_stream().cuda_stream
    ctx.transform_checked(t.data_ptr(), 24, 1, fr.COSET, stream, fr.ALGO_FOURSTEP_MFMA)
    torch.cuda.synchronize()
    Y = to_host(t)
    want = cref.transform(x, 24, 2, threads=0)
    assert np.array_equal(Y, want)
    ctx.transform_checked(t.data_ptr(), 24, 1, fr.COSET_INV, stream, fr.ALGO_FOURSTEP_MFMA)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), x)


def test_c3_butterfly_sampled(ctx):
    """2^24 butterfly coset: outputs sampled against the definition (O(N) each)."""
    _say("c3 2^24 coset butterfly sampled")
    x = si.polynomial(3, 24)
    Y = run(ctx, x, 24, fr.COSET, fr.ALGO_BUTTERFLY)
    rng = np.random.default_rng(3)
    for k in [0, 1, (1 << 24) - 1] + list(rng.integers(0, 1 << 24, 5)):
        assert np.array_equal(Y[k], cref.eval_output(x, 24, int(k), 2))


# ------------------------------------------------------------ edge cases

def test_edge_cases(ctx):
    x = si.polynomial(5, 6)
    t = to_dev(x)
    L = fr.lib()
    s = torch.cuda.current_stream().cuda_stream
    assert L.ntt_fwd(ctx.handle, t.data_ptr(), 6, 0, s) == 0           # batch 0: no-op
    assert L.ntt_fwd(ctx.handle, t.data_ptr(), 0, 4, s) == 0           # log_n 0: identity
    assert L.ntt_fwd(ctx.handle, t.data_ptr() + 8, 6, 1, s) == fr.frntt.EALIGN
    assert L.ntt_fwd(ctx.handle, t.data_ptr(), 25, 1, s) == fr.frntt.ERANGE
    assert L.ntt_fwd(ctx.handle, t.data_ptr(), -1, 1, s) == fr.frntt.ERANGE
    assert L.ntt_fwd(ctx.handle, t.data_ptr(), 6, -1, s) == fr.frntt.EINVAL
    assert L.ntt_transform(ctx.handle, t.data_ptr(), 6, 1, 9, s) == fr.frntt.EINVAL
    assert L.ntt_transform_algo(ctx.handle, t.data_ptr(), 6, 1, 0, 7, s) == fr.frntt.EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), x)                                 # nothing was changed


def test_log_n_one_and_zero(ctx):
    x = si.field_elements(9, 8)
    assert np.array_equal(run(ctx, x, 0, fr.FWD, batch=8), x)
    assert np.array_equal(run(ctx, x, 1, fr.COSET_INV), cref.transform(x, 1, 3))


def test_validate_flag():
    c = fr.Context(0, max_log_n=12, flags=fr.frntt.VALIDATE)
    try:
        x = si.polynomial(4, 8)
        t = to_dev(x)
        c.transform_checked(t.data_ptr(), 8, 1, fr.FWD)
        assert c.check_inputs() == 0
        bad = x.copy()
        bad[17] = si.from_ints([R])[0]
        t2 = to_dev(bad)
        c.transform_checked(t2.data_ptr(), 8, 1, fr.FWD)
        assert c.check_inputs() == fr.frntt.EINVAL
        assert c.check_inputs() == 0                                      # flag cleared
    finally:
        torch.cuda.synchronize()
        c.close()


def test_device_generator_matches_host(ctx):
    n = 5000
    t = torch.empty((n, 4), dtype=torch.int64, device="cuda:0")
    ctx.generate(t.data_ptr(), 1001, 7, 123, n)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(t), si.field_elements(1001, n, stream=7, start=123))


def test_determinism(ctx):
    x = si.polynomial(6, 18)
    outs = [run(ctx, x, 18, fr.FWD, fr.ALGO_FOURSTEP_MFMA) for _ in range(5)]
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    assert np.array_equal(run(ctx, x, 18, fr.FWD, fr.ALGO_BUTTERFLY), outs[0])
