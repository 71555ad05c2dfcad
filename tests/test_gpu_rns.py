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


# ---- the field objects: BN254 r through the generic path, and 377/753 bits ---

WIDTHS = [254, 377, 753]


@pytest.fixture(scope="module")
def fields(ctx):
    out = {254: fr.RnsField(ctx, M), 377: fr.RnsField(ctx, fr.FIELD_377), 753: fr.RnsField(ctx, fr.FIELD_753)}
    yield out
    for f in out.values():
        f.close()


def ints_to_u32(vals, words) -> np.ndarray:
    out = np.zeros((len(vals), words), dtype=np.uint32)
    for i, v in enumerate(vals):
        for w in range(words):
            out[i, w] = (v >> (32 * w)) & 0xFFFFFFFF
    return out


def u32_to_ints(a: np.ndarray):
    a = np.asarray(a, dtype=np.uint64)
    return [sum(int(x) << (32 * w) for w, x in enumerate(row)) for row in a]


def u32_dev(arr: np.ndarray):
    return torch.from_numpy(np.ascontiguousarray(arr, dtype=np.uint32).view(np.int32).reshape(-1).copy()).to("cuda:0")


def wide_operands(m, n, seed):
    import random
    rnd = random.Random(seed)
    a = [rnd.randrange(m) for _ in range(n)]
    b = [rnd.randrange(m) for _ in range(n)]
    edges = [(0, 0), (1, m - 1), (m - 1, m - 1), (m - 1, 1)]
    for i, (x, y) in enumerate(edges[:n]):
        a[i], b[i] = x, y
    return a, b


@pytest.mark.parametrize("bits", WIDTHS)
@pytest.mark.parametrize("n", [1, 33, 1000])
def test_field_steps_match_oracle(fields, bits, n):
    f = fields[bits]
    m, n_q, n_p, u, _ = R.width_params(bits)
    qs, ps = R.moduli(n_q, n_p)
    pre = R.Precomputation(qs, ps, m=m, u=u)
    _say(f"rns field {bits} bits n={n}")
    a, b = wide_operands(m, n, 7 * bits + n)
    s = torch.cuda.current_stream().cuda_stream
    # encode
    ta = u32_dev(ints_to_u32(a, f.words))
    xq = torch.full((n * f.q_words,), -1, dtype=torch.int32, device="cuda:0")
    f.encode(ta.data_ptr(), xq.data_ptr(), n, s)
    torch.cuda.synchronize()
    want = np.zeros((n, f.q_words), dtype=np.uint32)
    ea = R.encode(a, qs)
    want[:, :n_q] = ea.astype(np.uint32)
    assert np.array_equal(host_u32(xq, f.q_words), want)
    # product (Alg. 1 Main after the residue-wise product), from oracle inputs
    eb = R.encode(b, qs)
    wp = R.main(pre, R.vec_mul(ea, eb, qs))
    xa, xb = residues_to_dev(ea, f.q_words), residues_to_dev(eb, f.q_words)
    xp = torch.full((n * f.p_words,), -1, dtype=torch.int32, device="cuda:0")
    f.mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, s)
    torch.cuda.synchronize()
    got = host_u32(xp, f.p_words)
    assert np.array_equal(got[:, :n_p], wp.astype(np.uint32)) and not got[:, n_p:].any()
    # decode, from oracle inputs
    tx = residues_to_dev(wp, f.p_words)
    out = torch.zeros((n * f.words,), dtype=torch.int32, device="cuda:0")
    f.decode(tx.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert u32_to_ints(host_u32(out, f.words)) == R.decode(wp, ps, m=m) == [x * y % m for x, y in zip(a, b)]
    # radix Montgomery baseline
    tb = u32_dev(ints_to_u32(b, f.words))
    f.mont_mul(ta.data_ptr(), tb.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert u32_to_ints(host_u32(out, f.words)) == R.mont_product(a, b, m)


@pytest.mark.parametrize("bits", [377, 753])
def test_field_pipeline_sampled(fields, bits):
    f = fields[bits]
    m = R.width_params(bits)[0]
    n = 1 << 18
    _say(f"rns field pipeline {bits} bits n={n}")
    a, b = wide_operands(m, 2048, bits)
    idx = np.arange(n) % 2048                      # repeat 2048 operands over the whole range
    ta = u32_dev(ints_to_u32(a, f.words)[idx])
    tb = u32_dev(ints_to_u32(b, f.words)[idx])
    s = torch.cuda.current_stream().cuda_stream
    xa = torch.empty((n * f.q_words,), dtype=torch.int32, device="cuda:0")
    xb = torch.empty_like(xa)
    xp = torch.empty((n * f.p_words,), dtype=torch.int32, device="cuda:0")
    out = torch.empty((n * f.words,), dtype=torch.int32, device="cuda:0")
    f.encode(ta.data_ptr(), xa.data_ptr(), n, s)
    f.encode(tb.data_ptr(), xb.data_ptr(), n, s)
    f.mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, s)
    f.decode(xp.data_ptr(), out.data_ptr(), n, s)
    torch.cuda.synchronize()
    got = host_u32(out, f.words)
    want = [x * y % m for x, y in zip(a, b)]
    rng = np.random.default_rng(bits)
    for i in np.concatenate([[0, 1, n - 1], rng.integers(0, n, 2000)]):
        assert u32_to_ints(got[i:i + 1])[0] == want[i % 2048], i


def test_bn254_field_object_equals_context_calls(ctx, fields):
    f = fields[254]
    n = 777
    a, b = operands(n, 31)
    ta, tb = dev(ints_to_words(a)), dev(ints_to_words(b))
    s = torch.cuda.current_stream().cuda_stream
    outs = []
    for enc, mul, dec in ((ctx.rns_encode, ctx.rns_mul, ctx.rns_decode), (f.encode, f.mul, f.decode)):
        xa = torch.empty((n * QW,), dtype=torch.int32, device="cuda:0")
        xb = torch.empty_like(xa)
        xp = torch.empty((n * PW,), dtype=torch.int32, device="cuda:0")
        o = torch.empty((n * 4,), dtype=torch.int64, device="cuda:0")
        enc(ta.data_ptr(), xa.data_ptr(), n, s)
        enc(tb.data_ptr(), xb.data_ptr(), n, s)
        mul(xa.data_ptr(), xb.data_ptr(), xp.data_ptr(), n, s)
        dec(xp.data_ptr(), o.data_ptr(), n, s)
        torch.cuda.synchronize()
        outs.append((xa.cpu().numpy(), xp.cpu().numpy(), o.cpu().numpy()))
    for x, y in zip(*outs):
        assert np.array_equal(x, y)
    assert (f.n_q, f.n_p, f.q_words, f.p_words) == (17, 9, QW, PW)


def test_field_errors(ctx):
    import ctypes
    L = fr.lib()
    h = ctypes.c_void_p()
    even = (ctypes.c_uint32 * 8)(*([2] + [0] * 6 + [1]))
    assert L.frntt_rns_field_create(ctypes.byref(h), ctx.handle, even, 8) == fr.frntt.ERANGE
    wide = (ctypes.c_uint32 * 8)(*([1] + [0] * 6 + [0x80000000]))   # 256 bits: too wide for 8 words
    assert L.frntt_rns_field_create(ctypes.byref(h), ctx.handle, wide, 8) == fr.frntt.ERANGE
    assert L.frntt_rns_field_create(ctypes.byref(h), ctx.handle, even, 10) == fr.frntt.EINVAL
