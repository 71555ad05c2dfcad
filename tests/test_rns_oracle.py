"""Pins of the RNS lazy modular multiplication oracle (Alg. 1, "MXU RNS
Lazy") against what the mathematics fixes: the plain product a b mod r, the
CRT identity behind I_i, the byte decomposition of the constant table, the
exactness of the overflow count k, and planted mistakes that must fail."""
from __future__ import annotations

import random

import numpy as np
import pytest
import sympy

from oracle import rns_lazy as R

M = R.R_MOD


@pytest.fixture(scope="module")
def setup():
    qs, ps = R.moduli()
    return qs, ps, R.Precomputation(qs, ps)


def _pairs(n, seed):
    rnd = random.Random(seed)
    a = [rnd.randrange(M) for _ in range(n)] + [0, 1, M - 1, M - 1, 2, (M - 1) // 2]
    b = [rnd.randrange(M) for _ in range(n)] + [M - 1, M - 1, M - 1, 1, (M + 1) // 2, M - 2]
    return a, b


def test_moduli_are_consecutive_primes_below_the_bound(setup):
    qs, ps, _ = setup
    allm = qs + ps
    assert len(qs) == 17 and len(ps) == 9
    expect = [sympy.prevprime(R.MOD_BOUND)]
    while len(expect) < len(allm):
        expect.append(sympy.prevprime(expect[-1]))
    assert allm == expect
    assert all(sympy.isprime(m) for m in allm)
    Q, P = R._prod(qs), R._prod(ps)
    # a product of two canonical values stays below Q / 2, so k is exact
    assert Q > 2 * (M - 1) ** 2
    # every lazily reduced output W' lies in (-P/2, P/2)
    bound = (17 * 4 * 255 + 1) * M
    assert P > 2 * bound


def test_modmul_is_the_field_product(setup):
    a, b = _pairs(400, 11)
    assert R.modmul(a, b) == [x * y % M for x, y in zip(a, b)]


def test_crt_coefficients_rebuild_the_integer(setup):
    qs, ps, pre = setup
    rnd = random.Random(3)
    for _ in range(50):
        X = rnd.randrange(pre.Q)
        xq = [(X * pre.z) % q for q in qs]        # Montgomery-form residues
        assert sum(x * I for x, I in zip(xq, pre.I)) % pre.Q == X
    # I_i is 0 modulo every other q and z^-1 modulo its own
    for i, Ii in enumerate(pre.I):
        for k, q in enumerate(qs):
            assert Ii % q == (pow(pre.z, -1, q) if k == i else 0)


def test_constant_table_is_the_byte_split(setup):
    qs, ps, pre = setup
    E = pre.e_bytes()
    assert E.min() >= 0 and E.max() <= 255
    for i in range(len(qs)):
        for b in range(4):
            for j, p in enumerate(ps):
                c = sum(int(E[4 * i + b, 4 * j + h]) << (8 * h) for h in range(4))
                assert c == pre.C[i][b][j] == (pre.z * (pre.Ib[i][b] % M)) % p
    # signed digits used by the int8 form rebuild the same constants
    for row in pre.C:
        for cs in row:
            for c in cs:
                assert sum(d << (8 * h) for h, d in enumerate(R.signed_digits(c, 4))) == c
    assert pre.g == [(-pre.z * (pre.Q % M)) % p for p in ps]


def test_overflow_count_is_exact_and_output_is_lazy(setup):
    qs, ps, pre = setup
    a, b = _pairs(300, 5)
    x = R.vec_mul(R.encode(a, qs), R.encode(b, qs), qs)
    out, k = R.main(pre, x, return_k=True)
    assert k.tolist() == R.main_exact_k(pre, x)
    P = R._prod(ps)
    zinv = pow(pre.z, -1, P)
    bound = (17 * 4 * 255 + 1) * M
    for row, x_, y_ in zip(out.tolist(), a, b):
        W = sum((r * pow(P // p, -1, p) % p) * (P // p) for r, p in zip(row, ps)) * zinv % P
        if W > P // 2:
            W -= P
        assert abs(W) < bound
        assert W % M == x_ * y_ % M


def test_residue_product_is_montgomery(setup):
    qs, _, _ = setup
    a, b = _pairs(100, 9)
    x = R.vec_mul(R.encode(a, qs), R.encode(b, qs), qs)
    for row, x_, y_ in zip(x.tolist(), a, b):
        assert row == [(x_ * y_ * (1 << 32)) % q for q in qs]


def test_mont_product_definition():
    a, b = _pairs(50, 2)
    for o, x, y in zip(R.mont_product(a, b), a, b):
        assert o * (1 << 261) % M == x * y % M and 0 <= o < M


# ---- planted mistakes (in the oracle, on the CPU) --------------------------

def _modmul_with(pre_patch=None, main_patch=None):
    qs, ps = R.moduli()
    pre = R.Precomputation(qs, ps)
    if pre_patch:
        pre_patch(pre)
    a, b = _pairs(200, 21)
    x = R.vec_mul(R.encode(a, qs), R.encode(b, qs), qs)
    out = R.decode((main_patch or R.main)(pre, x), ps)
    return out == [p * q % M for p, q in zip(a, b)]


def test_planted_dropped_correction_fails():
    def drop(pre):
        pre.g = [0] * len(pre.g)
    assert not _modmul_with(drop)


def test_planted_unshifted_f_fails():
    def unshift(pre):
        pre.f = [[row[0]] * 4 for row in pre.f]
    assert not _modmul_with(unshift)


def test_planted_byte_order_fails():
    def swap(pre):
        pre.C = [[[((c & 0xFF) << 24) | ((c >> 8) & 0xFFFFFF) for c in cs] for cs in row] for row in pre.C]
    assert not _modmul_with(swap)


def test_planted_missing_y_fails():
    def no_y(pre):
        Q = pre.Q
        pre.I = [pow(Q // q, -1, q) * (Q // q) % Q for q in pre.src]
        pre.Ib = [[(Ii << (8 * b)) % Q for b in range(4)] for Ii in pre.I]
        pre.C = [[[(pre.z * (pre.Ib[i][b] % M)) % p for p in pre.dst] for b in range(4)] for i in range(len(pre.src))]
        pre.f = [[-((-pre.Ib[i][b] << pre.u) // Q) for b in range(4)] for i in range(len(pre.src))]
    assert not _modmul_with(no_y)


# ---- wider fields (377 and 753 bits) ---------------------------------------

@pytest.mark.parametrize("bits", [377, 753])
def test_wide_parameters(bits):
    m, n_q, n_p, u, u_dec = R.width_params(bits)
    assert m == sympy.prevprime(1 << bits) and m.bit_length() == bits
    qs, ps = R.moduli(n_q, n_p)
    expect = [sympy.prevprime(R.MOD_BOUND)]
    while len(expect) < n_q + n_p:
        expect.append(sympy.prevprime(expect[-1]))
    assert qs + ps == expect
    Q, P = R._prod(qs), R._prod(ps)
    assert Q > 2 * (m - 1) ** 2
    assert P > 2 * (4 * n_q * 255 + 1) * m
    # exact k: the estimate's error stays below 1 - (products / Q)
    assert 4 * n_q * 255 / 2 ** u + (m - 1) ** 2 / Q < 1
    # the decode's nearest-integer k: error below 1/2 with margin
    assert 4 * n_p * 255 / 2 ** u_dec < 0.5


@pytest.mark.parametrize("bits", [377, 753])
def test_wide_modmul_is_the_field_product(bits):
    m = R.width_params(bits)[0]
    rnd = random.Random(bits)
    a = [rnd.randrange(m) for _ in range(150)] + [0, 1, m - 1, m - 1]
    b = [rnd.randrange(m) for _ in range(150)] + [m - 1, m - 1, m - 1, 1]
    assert R.modmul(a, b, bits) == [x * y % m for x, y in zip(a, b)]


@pytest.mark.parametrize("bits", [377, 753])
def test_wide_overflow_count_exact(bits):
    m, n_q, n_p, u, _ = R.width_params(bits)
    qs, ps = R.moduli(n_q, n_p)
    pre = R.Precomputation(qs, ps, m=m, u=u)
    rnd = random.Random(bits + 1)
    a = [rnd.randrange(m) for _ in range(60)] + [m - 1]
    b = [rnd.randrange(m) for _ in range(60)] + [m - 1]
    x = R.vec_mul(R.encode(a, qs), R.encode(b, qs), qs)
    _, k = R.main(pre, x, return_k=True)
    assert k.tolist() == R.main_exact_k(pre, x)


def test_wide_mont_product_definition():
    for bits in (377, 753):
        m = R.width_params(bits)[0]
        limbs = -(-bits // 29)
        a, b = [3, m - 1, m // 2], [m - 2, m - 1, 5]
        for o, x, y in zip(R.mont_product(a, b, m), a, b):
            assert o * (1 << (29 * limbs)) % m == x * y % m
