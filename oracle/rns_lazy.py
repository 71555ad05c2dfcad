"""Oracle for the MXU-centric RNS lazy modular multiplication (paper:
Arithmetic Optimizations, "Solution: Reducing O(D^2) Reduction via MXU-Centric
RNS Lazy Reduction", and Alg. 1, "MXU RNS Lazy"), written from Alg. 1's
Precomputation and Main steps in their order, plus the plain definitions of
what surrounds it: the RNS encode (residues of x z), the residue-wise
Montgomery product (the "RNS-level 32-bit VecMul with Montgomery reduction"
of the walk-through) and the RNS decode (CRT reconstruction).

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library.

Parameters (the paper leaves them open; these are this implementation's),
for the three field widths the paper evaluates (256/377/753 bits):
  M   = r, the BN254 scalar-field prime (254 bits), or the largest prime
        below 2^377 or 2^753 (the paper names no curves for those widths);
  Q   = product of I primes q_i (I = 17, 25, 49), the largest below
        2^31 - 2^24, so that Q > 2 M^2 (a product of two canonical values
        never wraps Q);
  P   = product of J primes p_j (J = 9, 13, 25), the next ones below the
        q_i, so that P exceeds twice any lazily reduced output;
  w   = 32: residues are kept in Montgomery form x z mod q (z = 2^w),
        y = z^-1 (mod Q for the Q side, mod P for the P side);
  B   = H = 4 bytes per residue; u = 15, 16, 17 fraction bits for the
        overflow count k of Main (15, 16, 16 for the decode).
Readings of the printed algorithm:
  * I_i uses ((Q/q_i)^-1 mod q_i), the CRT coefficient of residue i (the
    text prints "mod p_i");
  * the dot product v = x . f is fused into the byte einsum, so f is taken
    per byte position: f_(i,b) = ceil(I_(i,b) 2^u / Q), matching the
    BAT-shifted I_(i,b) the einsum uses;
  * the returned x_P[j] + k g_j is reduced to its canonical residue mod p_j.
"""
from __future__ import annotations

import numpy as np

R_MOD = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
I_RES = 17
J_RES = 9
W_BITS = 32
U_BITS = 15
BYTES = 4
MOD_BOUND = (1 << 31) - (1 << 24)


def _is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (bases 2..41)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def moduli(n_q: int = I_RES, n_p: int = J_RES) -> tuple[list[int], list[int]]:
    """q_0 > ... > q_(n_q-1) > p_0 > ... > p_(n_p-1): consecutive primes below 2^31 - 2^24."""
    out = []
    n = MOD_BOUND - 1
    while len(out) < n_q + n_p:
        if _is_prime(n):
            out.append(n)
        n -= 2 if n % 2 else 1
    return out[:n_q], out[n_q:]


def _prev_prime(n: int) -> int:
    """Largest probable prime below n (Miller-Rabin with the 40 bases
    2..41; a one-off parameter choice, pinned against sympy in the tests)."""
    def probable_prime(x):
        if x % 2 == 0:
            return x == 2
        d, s = x - 1, 0
        while d % 2 == 0:
            d //= 2
            s += 1
        for a in range(2, 42):
            y = pow(a, d, x)
            if y in (1, x - 1):
                continue
            for _ in range(s - 1):
                y = y * y % x
                if y == x - 1:
                    break
            else:
                return False
        return True
    x = n - 1
    while not probable_prime(x):
        x -= 1
    return x


# field width -> (modulus, I, J, u of Main, u of the decode)
WIDTHS = {254: (R_MOD, 17, 9, 15, 15)}


def width_params(bits: int):
    """(M, I, J, u_mul, u_dec) of a field width (254: BN254 r; 377, 753: the
    largest prime below 2^bits)."""
    if bits not in WIDTHS:
        u = {377: (25, 13, 16, 16), 753: (49, 25, 17, 16)}[bits]
        WIDTHS[bits] = (_prev_prime(1 << bits),) + u
    return WIDTHS[bits]


def _prod(xs):
    p = 1
    for x in xs:
        p *= x
    return p


def signed_digits(c: int, n: int) -> list[int]:
    """Digits e_h in [-128, 127] with sum_h e_h 256^h = c (c below 2^(8n-1))."""
    e, carry = [], 0
    for h in range(n):
        d = ((c >> (8 * h)) & 255) + carry
        if d >= 128:
            e.append(d - 256)
            carry = 1
        else:
            e.append(d)
            carry = 0
    assert carry == 0, "value needs another digit"
    return e


class Precomputation:
    """Alg. 1 Precomputation(Q, P, w) for source base `src` and target base `dst`.

    I_i = ((Q/q_i)^-1 mod q_i) (Q/q_i) y mod Q; I_(i,b) = I_i 2^(8b) mod Q
    (the BAT shift); E[i,b,j,h] = byte h of (z (I_(i,b) mod M)) mod p_j;
    f_(i,b) = ceil(I_(i,b) 2^u / Q); g_j = (-z (Q mod M)) mod p_j.
    """

    def __init__(self, src: list[int], dst: list[int], m: int = R_MOD, w: int = W_BITS, u: int = U_BITS):
        self.src, self.dst, self.m, self.w, self.u = src, dst, m, w, u
        Q = _prod(src)
        self.Q = Q
        z = 1 << w
        self.z = z
        y = pow(z, -1, Q)
        self.I = []
        for q in src:
            Qi = Q // q
            self.I.append(pow(Qi, -1, q) * Qi * y % Q)
        self.Ib = [[(Ii << (8 * b)) % Q for b in range(BYTES)] for Ii in self.I]
        # E[i,b,j,h] as unsigned bytes and as signed digits
        self.C = [[[(z * (self.Ib[i][b] % m)) % p for p in dst] for b in range(BYTES)] for i in range(len(src))]
        self.f = [[-((-self.Ib[i][b] << u) // Q) for b in range(BYTES)] for i in range(len(src))]
        self.g = [(-z * (Q % m)) % p for p in dst]

    def e_bytes(self) -> np.ndarray:
        """E[(i,b), (j,h)] as unsigned bytes (int64 array, I*4 x J*4)."""
        I, J = len(self.src), len(self.dst)
        E = np.zeros((I * BYTES, J * BYTES), dtype=np.int64)
        for i in range(I):
            for b in range(BYTES):
                for j in range(J):
                    c = self.C[i][b][j]
                    for h in range(BYTES):
                        E[i * BYTES + b, j * BYTES + h] = (c >> (8 * h)) & 255
        return E

    def f_vec(self) -> np.ndarray:
        return np.array([self.f[i][b] for i in range(len(self.src)) for b in range(BYTES)], dtype=np.int64)


def byte_decompose(x: np.ndarray) -> np.ndarray:
    """ByteDecompose: [n, K] residues below 2^32 -> [n, K*4] bytes, byte b of residue i at 4i + b."""
    x = np.asarray(x, dtype=np.uint64)
    out = np.empty(x.shape[:-1] + (x.shape[-1] * BYTES,), dtype=np.int64)
    for b in range(BYTES):
        out[..., b::BYTES] = ((x >> np.uint64(8 * b)) & np.uint64(255)).astype(np.int64)
    return out


def byte_merge(xb: np.ndarray) -> np.ndarray:
    """ByteMerge: [n, J*4] byte-plane sums -> [n, J] integers sum_h x_h 2^(8h) (int64)."""
    out = np.zeros(xb.shape[:-1] + (xb.shape[-1] // BYTES,), dtype=np.int64)
    for h in range(BYTES):
        out += xb[..., h::BYTES] << (8 * h)
    return out


def main(pre: Precomputation, xq: np.ndarray, return_k: bool = False):
    """Alg. 1 Main: x_Q ([n, I] residues, Montgomery form) -> x_P ([n, J])."""
    xb = byte_decompose(xq)                      # [x_Q]_(i,b)
    v = xb @ pre.f_vec()                         # dot product with f (fused into the einsum)
    k = v >> pre.u                               # 32-bit vectorised shift
    xp_h = xb @ pre.e_bytes()                    # uint8 einsum over (i, b)
    xp = byte_merge(xp_h)                        # ByteMerge per residue j
    g = np.array(pre.g, dtype=np.int64)
    out = xp + k[:, None] * g[None, :]           # x_P[j] + k g_j
    p = np.array(pre.dst, dtype=np.int64)
    out = out % p[None, :]
    return (out, k) if return_k else out


# ---- plain definitions around Main ----------------------------------------

def encode(a: list[int], base: list[int], w: int = W_BITS) -> np.ndarray:
    """Residues of a z mod q (Montgomery form) of canonical values a."""
    z = 1 << w
    return np.array([[(x * z) % q for q in base] for x in a], dtype=np.int64)


def vec_mul(xa: np.ndarray, xb: np.ndarray, base: list[int], w: int = W_BITS) -> np.ndarray:
    """Residue-wise Montgomery product: a_i b_i z^-1 mod q_i."""
    q = np.array(base, dtype=np.uint64)
    zinv = np.array([pow(1 << w, -1, x) for x in base], dtype=np.uint64)
    t = (np.asarray(xa, dtype=np.uint64) * np.asarray(xb, dtype=np.uint64)) % q
    return ((t * zinv) % q).astype(np.int64)


def decode(xp: np.ndarray, base: list[int], m: int = R_MOD, w: int = W_BITS) -> list[int]:
    """The value W' with residues W' z mod p_j (signed representative, |W'| < P/2), reduced mod m."""
    P = _prod(base)
    zinv = pow(1 << w, -1, P)
    out = []
    for row in np.asarray(xp):
        x = 0
        for r_j, p in zip(row.tolist(), base):
            Pj = P // p
            x += (int(r_j) * pow(Pj, -1, p) % p) * Pj
        x = x * zinv % P
        if x > P // 2:
            x -= P
        out.append(x % m)
    return out


def modmul(a: list[int], b: list[int], bits: int = 254) -> list[int]:
    """a b mod M through encode, residue-wise product, Alg. 1 Main and decode."""
    m, n_q, n_p, u, _ = width_params(bits)
    qs, ps = moduli(n_q, n_p)
    pre = Precomputation(qs, ps, m=m, u=u)
    x = vec_mul(encode(a, qs), encode(b, qs), qs)
    return decode(main(pre, x), ps, m=m)


def mont_product(a: list[int], b: list[int], m: int = R_MOD) -> list[int]:
    """The radix Montgomery product the VALU baseline computes: a b 2^(-29 L)
    mod m with L = ceil(bits(m) / 29) 29-bit limbs (2^-261 for BN254 r)."""
    limbs = -(-m.bit_length() // 29)
    rinv = pow(1 << (29 * limbs), -1, m)
    return [x * y % m * rinv % m for x, y in zip(a, b)]


def main_exact_k(pre: Precomputation, xq: np.ndarray) -> list[int]:
    """floor(S' / Q) with S' = sum_(i,b) x_(i,b) I_(i,b), in exact integers."""
    out = []
    for row in np.asarray(xq).tolist():
        s = 0
        for i, x in enumerate(row):
            for b in range(BYTES):
                s += ((int(x) >> (8 * b)) & 255) * pre.Ib[i][b]
        out.append(s // pre.Q)
    return out
