"""Python big-integer oracle for the BN254-Fr number-theoretic transform.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library.

What it computes (paper: Background, "Number Theory Transformation"): for an
input vector x of length N, ``X_k = sum_n x_n * w_N^(k*n) mod r`` for k in
[0, N), with w_N a primitive N-th root of unity and r the field's prime.

Readings of points the paper leaves open (each one is also listed in the
design notes):

* The field is BN254's scalar field Fr (the paper only says "256-bit").
* w_N = 5^((r-1)/N); 5 generates the multiplicative group of Fr.
* The inverse transform includes the factor N^-1, so inverse(forward(x)) = x.
* The coset transform evaluates at g*w_N^k with shift g = 5:
  ``coset(x)_k = sum_n x_n g^n w_N^(kn)``; ``coset_inv`` is its exact inverse.
* Elements are canonical integers in [0, r); inputs >= r are rejected.
* Input and output are in natural order.

Functions here are the plain definition (``dft``: O(N^2)), a textbook
iterative radix-2 Cooley-Tukey FFT used as a fast step (``ntt``), and the
variants built from them. The FFT is checked against the definition in
``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

# BN254 scalar field modulus r (254 bits).
R_MOD = 21888242871839275222246405745257275088548364400416034343698204186575808495617
TWO_ADICITY = 28          # r - 1 = 2^28 * odd
GENERATOR = 5             # generator of Fr^*, also the coset shift g
COSET_SHIFT = GENERATOR

FWD, INV, COSET, COSET_INV = 0, 1, 2, 3


def _check(x):
    for v in x:
        if not (0 <= v < R_MOD):
            raise ValueError("input element outside [0, r)")


def root_of_unity(n: int, inverse: bool = False) -> int:
    """Primitive n-th root of unity w_n = 5^((r-1)/n), or its inverse."""
    if n <= 0 or n & (n - 1) or n > (1 << TWO_ADICITY):
        raise ValueError("n must be a power of two <= 2^28")
    w = pow(GENERATOR, (R_MOD - 1) // n, R_MOD)
    return pow(w, R_MOD - 2, R_MOD) if inverse else w


def inv_mod(a: int) -> int:
    return pow(a, R_MOD - 2, R_MOD)


def dft(x, inverse: bool = False):
    """The definition, term by term: X_k = sum_n x_n w^(kn) (O(N^2)).

    With ``inverse`` the root is w^-1 and the result is scaled by N^-1.
    """
    x = [int(v) for v in x]
    _check(x)
    n = len(x)
    if n == 0:
        return []
    w = root_of_unity(n, inverse)
    out = []
    for k in range(n):
        wk = pow(w, k, R_MOD)
        acc = 0
        p = 1
        for j in range(n):
            acc = (acc + x[j] * p) % R_MOD
            p = (p * wk) % R_MOD
        out.append(acc)
    if inverse:
        ninv = inv_mod(n)
        out = [(v * ninv) % R_MOD for v in out]
    return out


def _bit_reverse(i: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def ntt(x, inverse: bool = False):
    """Textbook iterative radix-2 decimation-in-time FFT over Fr.

    Bit-reverse the input, then for each span m = 2, 4, ..., N combine the
    halves with the twiddle w_m^j. Same result as ``dft``.
    """
    a = [int(v) for v in x]
    _check(a)
    n = len(a)
    if n == 0:
        return []
    bits = n.bit_length() - 1
    if 1 << bits != n:
        raise ValueError("length must be a power of two")
    a = [a[_bit_reverse(i, bits)] for i in range(n)]
    m = 2
    while m <= n:
        wm = root_of_unity(m, inverse)
        half = m // 2
        for start in range(0, n, m):
            w = 1
            for j in range(half):
                u = a[start + j]
                v = (a[start + j + half] * w) % R_MOD
                a[start + j] = (u + v) % R_MOD
                a[start + j + half] = (u - v) % R_MOD
                w = (w * wm) % R_MOD
        m *= 2
    if inverse:
        ninv = inv_mod(n)
        a = [(v * ninv) % R_MOD for v in a]
    return a


def intt(X):
    """Inverse transform: x_n = N^-1 sum_k X_k w^(-kn)."""
    return ntt(X, inverse=True)


def coset_ntt(x, g: int = COSET_SHIFT):
    """Evaluate at g*w^k: NTT of (x_n * g^n)."""
    x = [int(v) for v in x]
    _check(x)
    scaled = [(v * pow(g, i, R_MOD)) % R_MOD for i, v in enumerate(x)]
    return ntt(scaled)


def coset_intt(X, g: int = COSET_SHIFT):
    """Exact inverse of ``coset_ntt``: g^-n * INTT(X)_n."""
    y = intt(X)
    ginv = inv_mod(g)
    return [(v * pow(ginv, i, R_MOD)) % R_MOD for i, v in enumerate(y)]


def transform(x, kind: int):
    """Dispatch on kind: 0 forward, 1 inverse, 2 coset, 3 coset inverse."""
    if kind == FWD:
        return ntt(x)
    if kind == INV:
        return intt(x)
    if kind == COSET:
        return coset_ntt(x)
    if kind == COSET_INV:
        return coset_intt(x)
    raise ValueError("unknown transform kind")


def eval_output(x, k: int, kind: int = FWD) -> int:
    """One output of the transform, straight from the definition (O(N)).

    Used to check single outputs of transforms too large for the full oracle.
    """
    x = [int(v) for v in x]
    n = len(x)
    if kind in (FWD, COSET):
        base = root_of_unity(n)
        z = pow(base, k, R_MOD)
        if kind == COSET:
            z = (z * COSET_SHIFT) % R_MOD
        acc = 0
        for v in reversed(x):           # Horner: sum_n x_n z^n
            acc = (acc * z + v) % R_MOD
        return acc
    base = root_of_unity(n, inverse=True)
    z = pow(base, k, R_MOD)
    acc = 0
    for v in reversed(x):
        acc = (acc * z + v) % R_MOD
    acc = (acc * inv_mod(n)) % R_MOD
    if kind == COSET_INV:
        acc = (acc * pow(inv_mod(COSET_SHIFT), k, R_MOD)) % R_MOD
    return acc


def schoolbook_mul(a, b):
    """Polynomial product by the schoolbook rule (coefficients mod r)."""
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            out[i + j] = (out[i + j] + ai * bj) % R_MOD
    return out
