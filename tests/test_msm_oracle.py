"""Pins of the multi-scalar multiplication oracle (Background, "Multi-Scalar
Multiplication"; Alg. 2, LS-PPG) against what the mathematics fixes: the
published order of the curve's prime subgroup and its base point, the group
axioms, brute-force repeated addition, and the plain sum of products, with
planted mistakes that must fail."""
from __future__ import annotations

import random

import pytest
import sympy

from oracle import msm as M

# Baby Jubjub (EIP-2494): prime subgroup order l, cofactor 8, and the
# published generator of the subgroup
L_ORDER = 2736030358979909402780800718157159386076813972158567259200215660948447373041
BASE8 = (5299619240641551281634865583518297030282874472190772894086521144482721001553,
         16950150798460657717958625567821834550301663161624707787222815936182638968203)


def _points(n, seed):
    rnd = random.Random(seed)
    out = []
    while len(out) < n:
        p = M.point_from_x(rnd.randrange(M.R))
        if p is not None:
            out.append(p)
    return out


def test_curve_constants():
    # a square and d a non-square mod r: the affine addition law is complete
    assert pow(M.A, (M.R - 1) // 2, M.R) == 1
    assert pow(M.D, (M.R - 1) // 2, M.R) == M.R - 1
    assert sympy.isprime(M.R) and sympy.isprime(L_ORDER)
    # Hasse bound for the whole group order 8 l
    assert abs(M.R + 1 - 8 * L_ORDER) <= 2 * sympy.sqrt(M.R) + 1


def test_published_base_point_has_prime_order():
    assert M.on_curve(BASE8)
    assert M.mul(L_ORDER, BASE8) == M.ZERO
    assert M.mul(L_ORDER - 1, BASE8) == M.neg(BASE8)
    assert M.mul(8, BASE8) != M.ZERO


def test_group_order_kills_random_points():
    for p in _points(4, 1):
        assert M.on_curve(p)
        assert M.mul(8 * L_ORDER, p) == M.ZERO


def test_group_axioms():
    p, q, s = _points(3, 2)
    assert M.add(p, M.ZERO) == p and M.add(M.ZERO, p) == p
    assert M.add(p, M.neg(p)) == M.ZERO
    assert M.add(p, q) == M.add(q, p)
    assert M.add(M.add(p, q), s) == M.add(p, M.add(q, s))
    assert M.on_curve(M.add(p, q)) and M.on_curve(M.add(p, p))


def test_mul_is_repeated_addition():
    p = _points(1, 3)[0]
    acc = M.ZERO
    for k in range(40):
        assert M.mul(k, p) == acc
        acc = M.add(acc, p)


def test_mul_is_linear_in_the_scalar():
    p = _points(1, 4)[0]
    rnd = random.Random(4)
    for _ in range(3):
        a, b = rnd.randrange(1 << 256), rnd.randrange(1 << 256)
        assert M.mul(a + b, p) == M.add(M.mul(a, p), M.mul(b, p))


def test_naive_msm_brute_force_small_scalars():
    pts = _points(5, 5)
    sc = [3, 0, 7, 1, 12]
    acc = M.ZERO
    for s, p in zip(sc, pts):
        for _ in range(s):
            acc = M.add(acc, p)
    assert M.msm_naive(sc, pts) == acc


def _edge_scalars(n, seed):
    rnd = random.Random(seed)
    s = [rnd.randrange(1 << 256) for _ in range(n)]
    return s + [0, 1, (1 << 256) - 1, M.R - 1, 1 << 255, L_ORDER]


@pytest.mark.parametrize("c", [1, 3, 5, 8, 13, 16])
def test_lsppg_equals_sum_of_products(c):
    sc = _edge_scalars(5, 10 + c)
    pts = _points(len(sc), 20 + c)
    assert M.msm_lsppg(sc, pts, c) == M.msm_naive(sc, pts)


def test_lsppg_repeated_points_and_digits():
    # equal points and equal scalars land in the same buckets
    p, q = _points(2, 30)
    sc = [5, 5, 5, 9, (1 << 256) - 1, 0]
    pts = [p, p, q, q, p, q]
    for c in (2, 4, 7):
        assert M.msm_lsppg(sc, pts, c) == M.msm_naive(sc, pts)


def test_lsppg_empty_input_is_zero():
    assert M.msm_lsppg([], [], 4) == M.ZERO
    assert M.msm_naive([], []) == M.ZERO


def test_planted_mistakes_fail():
    p, q = _points(2, 40)
    # a wrong sign in the y numerator of the addition law
    def bad_add(u, v):
        x1, y1 = u
        x2, y2 = v
        t = M.D * x1 * x2 * y1 * y2 % M.R
        x3 = (x1 * y2 + y1 * x2) * pow(1 + t, -1, M.R) % M.R
        y3 = (y1 * y2 + M.A * x1 * x2) * pow(1 - t, -1, M.R) % M.R
        return (x3, y3)
    assert not M.on_curve(bad_add(p, q))
    assert M.mul(8 * L_ORDER, bad_add(p, q)) != M.ZERO
    # the sum misses the term of one point
    sc, pts = [6, 3, 11], [p, q, p]
    assert M.msm_lsppg(sc[:2], pts[:2], 2) != M.msm_naive(sc, pts)
