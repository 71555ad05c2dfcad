"""Pins for the CPU oracle: facts fixed by the mathematics, not by the oracle.

The paper prints no worked example (its walk-through figure is an image), so
the oracle is pinned by: an independent library (sympy's primitive root,
multiplicative order and NTT routine), closed forms of the definition
(paper: Background, "Number Theory Transformation"), a hand-derived N = 4
example, invariants (inverse, linearity, the convolution theorem against
schoolbook multiplication), coset evaluation by Horner's rule, brute force on
tiny inputs, and planted mistakes that these pins must catch.
"""
from __future__ import annotations

import os
import random

import numpy as np
import pytest
import sympy
from sympy.discrete.transforms import intt as sympy_intt
from sympy.discrete.transforms import ntt as sympy_ntt

import seeded_inputs as si
from oracle import cref
from oracle import fr_ntt as F

R = F.R_MOD
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_vec(n, seed):
    rng = random.Random(seed)
    return [rng.randrange(R) for _ in range(n)]


# ---------------------------------------------------------------- field facts

def _golden_field():
    vals = {}
    with open(os.path.join(GOLDEN, "bn254_fr.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v, 0)
    return vals


def test_modulus_matches_golden_and_is_prime():
    vals = _golden_field()
    assert F.R_MOD == vals["modulus_dec"]
    assert si.modulus() == vals["modulus_dec"]
    assert sympy.isprime(R)
    assert R.bit_length() == 254
    t, s = R - 1, 0
    while t % 2 == 0:
        t //= 2
        s += 1
    assert s == vals["two_adicity"] == F.TWO_ADICITY
    assert sympy.ntheory.primitive_root(R) == vals["generator"] == F.GENERATOR


@pytest.mark.parametrize("log_n", [1, 2, 3, 10, 16, 20, 24, 27, 28])
def test_root_properties(log_n):
    n = 1 << log_n
    w = F.root_of_unity(n)
    assert pow(w, n, R) == 1
    assert pow(w, n // 2, R) == R - 1          # w^(N/2) = -1
    assert (w * F.root_of_unity(n, inverse=True)) % R == 1


@pytest.mark.parametrize("log_n", [10, 20, 24, 28])
def test_python_roots_match_golden_hex(log_n):
    """The Python oracle's w_N equals the hex value written out independently."""
    vals = _golden_field()
    assert F.root_of_unity(1 << log_n) == vals[f"omega_2e{log_n}"]


def test_python_inverses_and_radix_match_golden_hex():
    vals = _golden_field()
    assert F.inv_mod(1 << 10) == vals["inv_2e10"]
    assert F.inv_mod(F.COSET_SHIFT) == vals["inv_5"]
    assert pow(2, 256, R) == vals["two256_mod_r"]
    # and the defining properties, so that a wrong hex value cannot pass
    assert (vals["inv_2e10"] << 10) % R == 1 and (vals["inv_5"] * 5) % R == 1


@pytest.mark.parametrize("log_n", [10, 20, 24])
def test_c_oracle_roots_and_scale_match_golden(log_n):
    """The C oracle reaches the same constants through its own arithmetic:
    output 1 of the transform of delta_1 is w_N (sum_n delta_1[n] w^(kn) at
    k = 1), output 0 of the inverse transform of delta_0 is N^-1, and output 1
    of the coset transform of delta_1 is g w_N."""
    vals = _golden_field()
    n = 1 << log_n
    d1 = np.zeros((n, 4), dtype=np.uint64)
    d1[1, 0] = 1
    w = si.to_ints(cref.eval_output(d1, log_n, 1, 0))[0]
    assert w == vals[f"omega_2e{log_n}"]
    assert si.to_ints(cref.eval_output(d1, log_n, 1, 2))[0] == (5 * w) % R
    d0 = np.zeros((n, 4), dtype=np.uint64)
    d0[0, 0] = 1
    ninv = si.to_ints(cref.eval_output(d0, log_n, 0, 1))[0]
    assert (ninv * n) % R == 1
    if log_n == 10:
        assert ninv == vals["inv_2e10"]
    # the full transform of delta_1 at N = 2^10 is the power table of w_N
    if log_n == 10:
        got = si.to_ints(cref.transform(d1, log_n, 0))
        assert got == [pow(vals["omega_2e10"], k, R) for k in range(n)]


def test_c_oracle_large_sizes_against_python_definition():
    """Sampled outputs of the C radix-2 transform at 2^16 and 2^20, every
    kind, against the Python big-integer definition (Horner, O(N) each)."""
    for log_n, ks in ((16, (0, 1, 40000, (1 << 16) - 1)), (20, (0, 777777))):
        x = si.polynomial(1000 + log_n, log_n)
        xi = si.to_ints(x)
        for kind in range(4):
            full = cref.transform(x, log_n, kind)
            for k in ks:
                assert si.to_ints(full[k:k + 1])[0] == F.eval_output(xi, k, kind), (log_n, kind, k)


@pytest.mark.parametrize("log_n", [1, 4, 8, 12])
def test_root_order_by_sympy(log_n):
    n = 1 << log_n
    assert sympy.ntheory.n_order(F.root_of_unity(n), R) == n


# ---------------------------------------------------------- pin predicates
# Each takes a transform family (dict of callables with the oracle's API) so
# the planted-mistake test can run the same predicates on mutated copies.

def pin_definition(T, sizes=(1, 2, 4, 8, 16, 32)):
    for n in sizes:
        x = _rand_vec(n, 1000 + n)
        if T["ntt"](x) != F.dft(x):
            return False
        if T["intt"](x) != F.dft(x, inverse=True):
            return False
    return True


def pin_sympy(T, sizes=(2, 8, 64, 1024)):
    for n in sizes:
        x = _rand_vec(n, 2000 + n)
        if T["ntt"](x) != sympy_ntt(x, R):
            return False
        if T["intt"](x) != sympy_intt(x, R):
            return False
    return True


def pin_worked_example(T):
    w = F.root_of_unity(4)
    expect = []
    with open(os.path.join(GOLDEN, "n4_worked_example.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, c0, c1 = (int(v) for v in line.split())
                expect.append((c0 + c1 * w) % R)
    return T["ntt"]([1, 2, 3, 4]) == expect


def pin_closed_forms(T, n=64):
    w = F.root_of_unity(n)
    delta0 = [1] + [0] * (n - 1)
    if T["ntt"](delta0) != [1] * n:
        return False
    if T["ntt"]([1] * n) != [n % R] + [0] * (n - 1):
        return False
    for j in (1, 3, n - 1):
        dj = [0] * n
        dj[j] = 1
        if T["ntt"](dj) != [pow(w, j * k, R) for k in range(n)]:
            return False
    c = 7                                        # c^n != 1
    geo = [pow(c, i, R) for i in range(n)]
    want = [((pow(c, n, R) - 1) * pow((c * pow(w, k, R) - 1) % R, R - 2, R)) % R for k in range(n)]
    if T["ntt"](geo) != want:
        return False
    d1 = [0, 1] + [0] * (n - 2)
    if T["coset"](d1) != [(F.COSET_SHIFT * pow(w, k, R)) % R for k in range(n)]:
        return False
    return True


def pin_horner_coset(T, n=32):
    x = _rand_vec(n, 77)
    w = F.root_of_unity(n)
    want = []
    for k in range(n):
        z = (F.COSET_SHIFT * pow(w, k, R)) % R
        acc = 0
        for v in reversed(x):
            acc = (acc * z + v) % R
        want.append(acc)
    return T["coset"](x) == want


def pin_invariants(T, n=128):
    x = _rand_vec(n, 5)
    y = _rand_vec(n, 6)
    if T["intt"](T["ntt"](x)) != x:
        return False
    if T["coset_inv"](T["coset"](x)) != x:
        return False
    a = 123456789
    lhs = T["ntt"]([(a * u + v) % R for u, v in zip(x, y)])
    X, Y = T["ntt"](x), T["ntt"](y)
    if lhs != [(a * u + v) % R for u, v in zip(X, Y)]:
        return False
    # inverse after coset returns x_n * g^n
    if T["intt"](T["coset"](x)) != [(v * pow(F.COSET_SHIFT, i, R)) % R for i, v in enumerate(x)]:
        return False
    return True


def pin_convolution(T, n=64):
    a = _rand_vec(n, 8)
    b = _rand_vec(n, 9)
    pa = a + [0] * n
    pb = b + [0] * n
    prod = T["intt"]([(u * v) % R for u, v in zip(T["ntt"](pa), T["ntt"](pb))])
    want = F.schoolbook_mul(a, b) + [0]
    return prod == want


ALL_PINS = [pin_definition, pin_sympy, pin_worked_example, pin_closed_forms,
            pin_horner_coset, pin_invariants, pin_convolution]

ORACLE = {"ntt": F.ntt, "intt": F.intt, "coset": F.coset_ntt, "coset_inv": F.coset_intt}


@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_python_oracle_pins(pin):
    assert pin(ORACLE)


def test_definition_against_fft_many_sizes():
    for log_n in range(0, 9):
        n = 1 << log_n
        x = _rand_vec(n, 300 + n)
        assert F.dft(x) == F.ntt(x)
        assert F.dft(x, inverse=True) == F.intt(x)


def test_eval_output_is_the_definition():
    n = 256
    x = _rand_vec(n, 11)
    for kind in range(4):
        full = F.transform(x, kind)
        for k in (0, 1, 17, 255):
            assert F.eval_output(x, k, kind) == full[k]


def test_oracle_rejects_out_of_range():
    with pytest.raises(ValueError):
        F.ntt([0, R])
    bad = si.from_ints([0, R])
    with pytest.raises(ValueError):
        cref.transform(bad, 1)


# ------------------------------------------------------- planted mistakes

def _mutant(kind):
    """A copy of the radix-2 oracle with one plausible mistake planted."""
    def fft(x, inverse=False):
        a = [int(v) for v in x]
        n = len(a)
        bits = n.bit_length() - 1
        if kind != "no_bitrev":
            a = [a[F._bit_reverse(i, bits)] for i in range(n)]
        m = 2
        while m <= n:
            wm = F.root_of_unity(m, inverse if kind != "wrong_root_dir" else not inverse)
            if kind == "wrong_root" and m == n and n >= 4:
                wm = pow(wm, 3, R)
            half = m // 2
            for s in range(0, n, m):
                w = 1
                for j in range(half):
                    u = a[s + j]
                    v = (a[s + j + half] * w) % R
                    a[s + j] = (u + v) % R
                    a[s + j + half] = (u - v) % R if kind != "sign" else (v - u) % R
                    if kind != "stale_twiddle":
                        w = (w * wm) % R
            m *= 2
        if inverse and kind != "no_scale":
            ninv = F.inv_mod(n)
            a = [(v * ninv) % R for v in a]
        return a

    def coset(x):
        g = F.COSET_SHIFT if kind != "coset_g_inv" else F.inv_mod(F.COSET_SHIFT)
        return fft([(v * pow(g, i, R)) % R for i, v in enumerate(x)])

    def coset_inv(X):
        y = fft(X, inverse=True)
        gi = F.inv_mod(F.COSET_SHIFT)
        return [(v * pow(gi, i, R)) % R for i, v in enumerate(y)]

    return {"ntt": fft, "intt": lambda X: fft(X, True), "coset": coset, "coset_inv": coset_inv}


@pytest.mark.parametrize("kind", ["no_bitrev", "wrong_root_dir", "wrong_root", "sign",
                                  "stale_twiddle", "no_scale", "coset_g_inv"])
def test_pins_catch_planted_mistakes(kind):
    T = _mutant(kind)
    caught = []
    for pin in ALL_PINS:
        try:
            ok = pin(T)
        except Exception:
            ok = False
        if not ok:
            caught.append(pin.__name__)
    assert caught, f"planted mistake {kind!r} passed every pin"


# ------------------------------------------------------ C oracle vs Python

@pytest.mark.parametrize("log_n", [0, 1, 2, 5, 9, 12, 13, 14])
@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_c_oracle_matches_python(log_n, kind):
    batch = 3 if log_n <= 9 else 1
    x = np.concatenate([si.polynomial(7, log_n, stream=s) for s in range(batch)])
    got = cref.transform(x, log_n, kind)
    n = 1 << log_n
    for b in range(batch):
        want = F.transform(si.to_ints(x[b * n:(b + 1) * n]), kind)
        assert si.to_ints(got[b * n:(b + 1) * n]) == want


@pytest.mark.parametrize("pattern", ["zeros", "ones", "rminus1", "onehot", "alternating"])
def test_c_oracle_adversarial(pattern):
    n = 256
    if pattern == "zeros":
        v = [0] * n
    elif pattern == "ones":
        v = [1] * n
    elif pattern == "rminus1":
        v = [R - 1] * n
    elif pattern == "onehot":
        v = [0] * n
        v[37] = R - 1
    else:
        v = [R - 1 if i % 2 else 1 for i in range(n)]
    x = si.from_ints(v)
    for kind in range(4):
        assert si.to_ints(cref.transform(x, 8, kind)) == F.transform(v, kind)


def test_c_eval_output_and_mul():
    x = si.polynomial(3, 10)
    xi = si.to_ints(x)
    for kind in range(4):
        full = F.transform(xi, kind)
        for k in (0, 5, 1023):
            assert si.to_ints(cref.eval_output(x, 10, k, kind))[0] == full[k]
    a, b = _rand_vec(2, 4)
    assert si.to_ints(cref.mul(si.from_ints([a])[0], si.from_ints([b])[0]))[0] == (a * b) % R


def test_c_oracle_pins_via_wrapper():
    """The C oracle passes the same pins as the Python one."""
    def wrap(kind):
        def f(x):
            n = len(x)
            return si.to_ints(cref.transform(si.from_ints(x), n.bit_length() - 1, kind))
        return f
    T = {"ntt": wrap(0), "intt": wrap(1), "coset": wrap(2), "coset_inv": wrap(3)}
    for pin in ALL_PINS:
        assert pin(T), pin.__name__
