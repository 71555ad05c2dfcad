"""Oracle for multi-scalar multiplication (paper: Background, "Multi-Scalar
Multiplication", and Alg. 2, Layout Stationary Pippenger "LS-PPG").

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this module;
only ``tests/`` and the ``cpu_baseline`` leg of ``bench.py`` may use it. It
shares no code with the HIP library.

MSM(S, P) = sum_n S_n * P_n over the points P_n of a twisted Edwards curve
(the paper's Alg. 2 works on twisted Edwards curves, zero point (0, 1, 1, 0)
in extended coordinates). Reading: the curve is Baby Jubjub,
a x^2 + y^2 = 1 + d x^2 y^2 over BN254's scalar field r with a = 168700,
d = 168696 (a twisted Edwards curve over the 256-bit field the rest of this
project uses; the paper names no curve). a is a square and d is not, so the
affine addition law below is complete.

* ``add``/``mul``/``msm_naive``: the plain definitions (affine addition law,
  double-and-add, the sum of products);
* ``msm_lsppg``: Alg. 2's steps in order with window width c: Bucketize
  (argsort of each window's digits, points gathered into their buckets),
  Bucket Accumulation, the tree-form Bucket Reduction
  (W <- W_L + W_R + B_R, B <- 2 (B_L + B_R) per level), Window Merging
  (MSM <- 2^c MSM + W_k from the top window down).
Scalars are non-negative integers below 2^256 (K = ceil(256 / c) windows).
"""
from __future__ import annotations

R = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
A = 168700
D = 168696
ZERO = (0, 1)


def on_curve(p) -> bool:
    x, y = p
    x2, y2 = x * x % R, y * y % R
    return (A * x2 + y2 - 1 - D * x2 * y2) % R == 0


def add(p, q):
    """Affine twisted Edwards addition (complete: a square, d non-square)."""
    x1, y1 = p
    x2, y2 = q
    t = D * x1 * x2 * y1 * y2 % R
    x3 = (x1 * y2 + y1 * x2) * pow(1 + t, -1, R) % R
    y3 = (y1 * y2 - A * x1 * x2) * pow(1 - t, -1, R) % R
    return (x3, y3)


def neg(p):
    return ((-p[0]) % R, p[1])


def mul(k: int, p):
    """k p by double-and-add (k >= 0)."""
    acc = ZERO
    base = p
    while k:
        if k & 1:
            acc = add(acc, base)
        base = add(base, base)
        k >>= 1
    return acc


def msm_naive(scalars, points):
    acc = ZERO
    for s, p in zip(scalars, points):
        acc = add(acc, mul(s, p))
    return acc


def msm_lsppg(scalars, points, c: int):
    """Alg. 2 (LS-PPG) with c-bit windows over 256-bit scalars."""
    K = -(-256 // c)
    n = len(points)
    # Bucketize: per window, sort point indices by digit and place each point
    # into bucket I_k[n]
    buckets = []
    for k in range(K):
        digits = [(s >> (c * k)) & ((1 << c) - 1) for s in scalars]
        order = sorted(range(n), key=lambda i: digits[i])
        bk = [[] for _ in range(1 << c)]
        for i in order:
            bk[digits[i]].append(points[i])
        buckets.append(bk)
    # Bucket Accumulation: B_(k,j) = sum of its points
    B = [[ZERO] * (1 << c) for _ in range(K)]
    for k in range(K):
        for j in range(1, 1 << c):
            acc = ZERO
            for p in buckets[k][j]:
                acc = add(acc, p)
            B[k][j] = acc
    # Bucket Reduction, tree form: level s combines pairs (2b, 2b + 1)
    W = [[ZERO] * (1 << c) for _ in range(K)]
    for s in range(c - 1, -1, -1):
        for k in range(K):
            nb, nw = [], []
            for b in range(1 << s):
                bl, br = B[k][2 * b], B[k][2 * b + 1]
                wl, wr = W[k][2 * b], W[k][2 * b + 1]
                nw.append(add(add(wl, wr), br))
                t = add(bl, br)
                nb.append(add(t, t))
            B[k], W[k] = nb, nw
    # Window Merging from the top window down
    acc = ZERO
    for k in range(K - 1, -1, -1):
        for _ in range(c):
            acc = add(acc, acc)
        acc = add(acc, W[k][0])
    return acc


def sqrt_mod(a: int):
    """A square root of a mod R (Tonelli-Shanks; R - 1 = 2^28 q), or None."""
    a %= R
    if a == 0:
        return 0
    if pow(a, (R - 1) // 2, R) != 1:
        return None
    q, s = R - 1, 0
    while q % 2 == 0:
        q //= 2
        s += 1
    z = 5  # a non-residue mod R
    m, c, t, x = s, pow(z, q, R), pow(a, q, R), pow(a, (q + 1) // 2, R)
    while t != 1:
        i, t2 = 0, t
        while t2 != 1:
            t2 = t2 * t2 % R
            i += 1
        b = pow(c, 1 << (m - i - 1), R)
        m, c, t, x = i, b * b % R, t * b * b % R, x * b % R
    return x


def point_from_x(x: int):
    """(x, y) on the curve with the smaller root y, or None if x has no point."""
    x2 = x * x % R
    num = (1 - A * x2) % R
    den = (1 - D * x2) % R
    if den == 0:
        return None
    y = sqrt_mod(num * pow(den, -1, R) % R)
    if y is None:
        return None
    return (x, min(y, R - y))
