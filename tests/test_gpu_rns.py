"""Parity of the RNS lazy modular product (Alg. 1) and the radix Montgomery
baseline with the oracle, bit-exact: every residue and every canonical
output is unique, so the HIP results must equal the oracle's word for word.

Inputs are the seeded uniform elements of [0, r) plus the extreme values
(0, 1, r - 1); the oracle (oracle/rns_lazy.py) is pinned in
test_rns_oracle.py. Sizes span several 32-element column groups, ragged
tails, and one 2^22-element run checked on a sample."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import seeded_inputs as si
from oracle import rns_lazy as R

torch = pytest.importorskip("torch")
import paper_2604_17808_amd as fr  # noqa: E402

pytestmark = pytest.mark.gpu

M = R.R_MOD
QW, PW = fr.RNS_Q_WORDS, fr.RNS_P_WORDS


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


@pytest.fixture(scope="module")
def pre():
    qs, ps = R.moduli()
    return qs, ps, R.Precomputation(qs, ps)


def ints_to_words(vals) -> np.ndarray:
    out = np.zeros((len(vals), 4), dtype=np.uint64)
    for i, v in enumerate(vals):
        for w in range(4):
            out[i, w] = (v >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return out


def words_to_ints(a: np.ndarray):
    a = np.asarray(a, dtype=np.uint64).reshape(-1, 4)
    return [int(r[0]) | (int(r[1]) << 64) | (int(r[2]) << 128) | (int(r[3]) << 192) for r in a]


def dev(arr: np.ndarray):
    a = np.ascontiguousarray(arr)
    return torch.from_numpy(a.view(np.int64).reshape(-1).copy() if a.dtype.itemsize == 8
                            else a.view(np.int32).reshape(-1).copy()).to("cuda:0")


def residues_to_dev(res: np.ndarray, words: int):
    n = res.shape[0]
    full = np.zeros((n, words), dtype=np.uint32)
    full[:, :res.shape[1]] = res.astype(np.uint32)
    return torch.from_numpy(full.view(np.int32).reshape(-1).copy()).to("cuda:0")


def host_u32(t, words):
    return t.cpu().numpy().view(np.uint32).reshape(-1, words)


def operands(n, seed):
    a = words_to_ints(si.field_elements(seed, n, stream=0))
    b = words_to_ints(si.field_elements(seed, n, stream=1))
    edges = [(0, 0), (1, M - 1), (M - 1, M - 1), (M - 1, 1), (2, (M + 1) // 2)]
    for i, (x, y) in enumerate(edges[:n]):
        a[i], b[i] = x, y
    return a, b


SIZES = [1, 31, 32, 33, 100, 1000, 4097]


@pytest.mark.parametrize("n", SIZES)
def test_encode_matches_oracle(ctx, pre, n):
    qs, _, _ = pre
    _say(f"rns encode n={n}")
    a, _ = operands(n, 101 + n)
    ta = dev(ints_to_words(a))
    xq = torch.full((n * QW,), -1, dtype=torch.int32, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    ctx.rns_encode(ta.data_ptr(), xq.data_ptr(), n, s)
    torch.cuda.synchronize()
    got = host_u32(xq, QW)
    want = np.zeros((n, QW), dtype=np.uint32)
    want[:, :17] = R.encode(a, qs).astype(np.uint32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", SIZES)
def test_mul_matches_alg1_main(ctx, pre, n):
    qs, ps, P = pre
    _say(f"rns mul n={n}")
    a, b = operands(n, 202 + n)
    xa, xb = R.encode(a, qs), R.encode(b, qs)
    want = R.main(P, R.vec_mul(xa, xb, qs))
    ta, tb = residues_to_dev(xa, QW), residues_to_dev(xb, QW)
    xp = torch.full((n * PW,), -1, dtype=torch.int32, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    ctx.rns_mul(ta.data_ptr(), tb.data_ptr(), xp.data_ptr(), n, s)
    torch.cuda.synchronize()
    got = host_u32(xp, PW)
    assert np.array_equal(got[:, :9], want.astype(np.uint32))
    assert not got[:, 9:].any()


@pytest.mark.parametrize("n", SIZES)
def test_decode_matches_crt(ctx, pre, n):
    qs, ps, P = pre
    _say(f"rns decode n={n}")
    a, b = operands(n, 303 + n)
    xp = R.main(P, R.vec_mul(R.encode(a, qs), R.encode(b, qs), qs))
    want = R.decode(xp, ps)
    tx = residues_to_dev(xp, PW)
    out = torch.zeros((n * 4,), dtype=torch.int64, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    ctx.rns_decode(tx.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert words_to_ints(out.cpu().numpy().view(np.uint64)) == want


def _pipeline(ctx, a_dev, b_dev, n):
    s = torch.cuda.current_stream().cuda_stream
    xa = torch.empty((n * QW,), dtype=torch.int32, device="cuda:0")
    xb = torch.empty_like(xa)
    xp = torch.empty((n * PW,), dtype=torch.int32, device="cuda:0")
    out = torch.empty((n * 4,), dtype=torch.int64, device="cuda:0")
    ctx.rns_encode(a_dev.data_ptr(), xa.data_ptr(), n, s)
    ctx.rns_encode(b_dev.data_ptr(), xb.data_ptr(), n, s)
    ctx.rns_mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, s)
    ctx.rns_decode(xp.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("n", [1, 33, 4097])
def test_pipeline_is_the_field_product(ctx, n):
    _say(f"rns pipeline n={n}")
    a, b = operands(n, 404 + n)
    out = _pipeline(ctx, dev(ints_to_words(a)), dev(ints_to_words(b)), n)
    assert words_to_ints(out.cpu().numpy().view(np.uint64)) == [x * y % M for x, y in zip(a, b)]


def test_pipeline_2e22_sampled(ctx):
    n = 1 << 22
    _say(f"rns pipeline n={n} sampled")
    wa, wb = si.field_elements(7, n, stream=0), si.field_elements(7, n, stream=1)
    wa[0], wb[0] = ints_to_words([M - 1])[0], ints_to_words([M - 1])[0]
    out = _pipeline(ctx, dev(wa), dev(wb), n).cpu().numpy().view(np.uint64).reshape(-1, 4)
    rng = np.random.default_rng(1)
    idx = np.concatenate([[0, 1, n - 1], rng.integers(0, n, 3000)])
    a, b = words_to_ints(wa[idx]), words_to_ints(wb[idx])
    assert words_to_ints(out[idx]) == [x * y % M for x, y in zip(a, b)]


@pytest.mark.parametrize("n", [1, 255, 4096, 100003])
def test_mont_mul_baseline(ctx, n):
    _say(f"mont mul n={n}")
    a, b = operands(n, 505 + n)
    ta, tb = dev(ints_to_words(a)), dev(ints_to_words(b))
    out = torch.empty((n * 4,), dtype=torch.int64, device="cuda:0")
    s = torch.cuda.current_stream().cuda_stream
    ctx.mont_mul(ta.data_ptr(), tb.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert words_to_ints(out.cpu().numpy().view(np.uint64)) == R.mont_product(a, b)


def test_rns_errors(ctx):
    L = fr.lib()
    t = torch.zeros(64, dtype=torch.int64, device="cuda:0")
    p = t.data_ptr()
    assert L.frntt_rns_encode(ctx.handle, p, p, 0, None) == 0
    assert L.frntt_rns_mul(ctx.handle, p, p, p, -1, None) == fr.frntt.EINVAL
    assert L.frntt_rns_encode(ctx.handle, p + 4, p, 1, None) == fr.frntt.EALIGN
    assert L.frntt_rns_decode(ctx.handle, p, p + 8, 1, None) == fr.frntt.EALIGN
    assert L.frntt_mont_mul(ctx.handle, p, None, p, 1, None) == fr.frntt.EINVAL
