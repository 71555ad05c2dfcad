"""Seeded synthetic inputs for BN254-Fr transforms.

This module is the only code shared by the CPU oracle and the GPU path's
tests and benchmarks. It draws random field elements and workload shapes; it
holds none of the transform's arithmetic.

The paper gives no value distribution for its NTT workloads (zk-SNARK
polynomials of degree 2^14..2^26, Experiment Setup); uniform elements of
[0, r) stand in for them.

Generator (counter based, so any element can be produced on its own):

* ``mix64(z)`` is the SplitMix64 output finaliser of Steele, Lea and Flood
  (OOPSLA 2014): ``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
  z *= 0x94D049BB133111EB; z ^= z >> 31`` (all mod 2^64).
* Word ``j`` (0..3) of attempt ``t`` (0..63) of element ``i`` of stream ``s``
  is ``mix64(seed*0x9E3779B97F4A7C15 + (s << 40) + (i << 8) + (t << 2) + j)``.
* The candidate is ``w0 + w1*2^64 + w2*2^128 + (w3 & (2^62-1))*2^192``
  (< 2^254). The first candidate below r is taken; if all 64 attempts fail
  the element is ``candidate_63 - r``.
* Shape and arrival draws use streams ``s >= 2^23`` (see ``draw_u64``).

Elements are returned as numpy ``uint64`` arrays of shape ``(..., 4)``:
four little-endian 64-bit limbs, canonical in [0, r).
"""
from __future__ import annotations

import math

import numpy as np

# BN254 scalar-field modulus, as four little-endian 64-bit limbs (only used
# for the rejection test of the sampler).
_R_LIMBS = (
    0x43E1F593F0000001,
    0x2833E84879B97091,
    0xB85045B68181585D,
    0x30644E72E131A029,
)
_R_INT = sum(limb << (64 * k) for k, limb in enumerate(_R_LIMBS))

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MIX_C1 = 0xBF58476D1CE4E5B9
MIX_C2 = 0x94D049BB133111EB
MAX_ATTEMPTS = 64
SHAPE_STREAM_BASE = 1 << 23
_M64 = (1 << 64) - 1


def mix64_int(z: int) -> int:
    """SplitMix64 finaliser on one Python integer (mod 2^64)."""
    z &= _M64
    z ^= z >> 30
    z = (z * MIX_C1) & _M64
    z ^= z >> 27
    z = (z * MIX_C2) & _M64
    z ^= z >> 31
    return z


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(MIX_C1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(MIX_C2)
        z ^= z >> np.uint64(31)
    return z


def _counter_base(seed: int, stream: int) -> np.uint64:
    return np.uint64(((seed * GOLDEN_GAMMA) + (stream << 40)) & _M64)


def _below_r(w: np.ndarray) -> np.ndarray:
    """Lexicographic (most significant limb first) test w < r on (..., 4)."""
    lt = np.zeros(w.shape[:-1], dtype=bool)
    eq = np.ones(w.shape[:-1], dtype=bool)
    for k in (3, 2, 1, 0):
        rk = np.uint64(_R_LIMBS[k])
        lt |= eq & (w[..., k] < rk)
        eq &= w[..., k] == rk
    return lt


def _sub_r(w: np.ndarray) -> np.ndarray:
    out = np.empty_like(w)
    borrow = np.zeros(w.shape[:-1], dtype=np.uint64)
    for k in range(4):
        rk = np.uint64(_R_LIMBS[k])
        with np.errstate(over="ignore"):
            d = w[..., k] - rk - borrow
        nb = (w[..., k] < rk) | ((w[..., k] == rk) & (borrow == 1))
        out[..., k] = d
        borrow = nb.astype(np.uint64)
    return out


def field_elements(seed: int, count: int, stream: int = 0, start: int = 0) -> np.ndarray:
    """Elements ``start .. start+count-1`` of ``stream`` as a (count, 4) uint64 array."""
    if count < 0 or start < 0:
        raise ValueError("count and start must be non-negative")
    if start + count > (1 << 32):
        raise ValueError("element index exceeds the generator's 2^32 counter range")
    out = np.zeros((count, 4), dtype=np.uint64)
    if count == 0:
        return out
    base = _counter_base(seed, stream)
    idx = np.arange(start, start + count, dtype=np.uint64) << np.uint64(8)
    pending = np.arange(count)
    mask62 = np.uint64((1 << 62) - 1)
    last = None
    for t in range(MAX_ATTEMPTS):
        if pending.size == 0:
            break
        cand = np.empty((pending.size, 4), dtype=np.uint64)
        with np.errstate(over="ignore"):
            ctr = base + idx[pending] + np.uint64(t << 2)
            for j in range(4):
                cand[:, j] = _mix64_np(ctr + np.uint64(j))
        cand[:, 3] &= mask62
        ok = _below_r(cand)
        out[pending[ok]] = cand[ok]
        last = cand[~ok]
        pending = pending[~ok]
    if pending.size:
        out[pending] = _sub_r(last)
    return out


def polynomial(seed: int, log_n: int, stream: int = 0) -> np.ndarray:
    """One polynomial of 2^log_n coefficients (stream = polynomial index)."""
    return field_elements(seed, 1 << log_n, stream=stream)


def batch(seed: int, log_n: int, count: int) -> np.ndarray:
    """``count`` polynomials of 2^log_n coefficients, (count, 2^log_n, 4)."""
    return np.stack([polynomial(seed, log_n, stream=s) for s in range(count)]) if count else \
        np.zeros((0, 1 << log_n, 4), dtype=np.uint64)


def draw_u64(seed: int, stream: int, index: int) -> int:
    """One raw 64-bit draw from a reserved shape/arrival stream (s >= 2^23)."""
    if stream < SHAPE_STREAM_BASE:
        raise ValueError("shape streams start at 2^23")
    ctr = (seed * GOLDEN_GAMMA + (stream << 40) + (index << 8)) & _M64
    return mix64_int(ctr)


def draw_log_n(seed: int, stream: int, index: int, lo: int, hi: int) -> int:
    """Uniform integer in [lo, hi] (log2 of a transform size)."""
    return lo + draw_u64(seed, stream, index) % (hi - lo + 1)


def draw_unit(seed: int, stream: int, index: int) -> float:
    """Uniform double in [0, 1) with 53 random bits."""
    return (draw_u64(seed, stream, index) >> 11) * (2.0 ** -53)


SIZE_STREAM = SHAPE_STREAM_BASE + 0
KIND_STREAM = SHAPE_STREAM_BASE + 1
ARRIVAL_STREAM = SHAPE_STREAM_BASE + 2


def uneven_batch_sizes(seed: int, count: int, lo: int, hi: int) -> list[int]:
    """log2 sizes of ``count`` jobs, uniform over [lo, hi]."""
    return [draw_log_n(seed, SIZE_STREAM, i, lo, hi) for i in range(count)]


def request_stream(seed: int, count: int, lo: int, hi: int, rate_per_s: float,
                   mix=(0.4, 0.4, 0.2)) -> list[dict]:
    """Poisson arrivals of NTT / INTT / coset-NTT requests.

    Each request is ``{"id", "log_n", "kind", "t_arrive_s"}`` with kind 0 =
    forward, 1 = inverse, 2 = coset forward, drawn with probabilities ``mix``.
    Inter-arrival gaps are exponential with the given rate.
    """
    out = []
    t = 0.0
    c0, c1 = mix[0], mix[0] + mix[1]
    for i in range(count):
        u = draw_unit(seed, KIND_STREAM, i)
        kind = 0 if u < c0 else (1 if u < c1 else 2)
        gap = -math.log(1.0 - draw_unit(seed, ARRIVAL_STREAM, i)) / rate_per_s
        t += gap
        out.append({"id": i, "log_n": draw_log_n(seed, SIZE_STREAM, i, lo, hi),
                    "kind": kind, "t_arrive_s": t})
    return out


def to_ints(a: np.ndarray) -> list[int]:
    """(N, 4) uint64 limbs -> list of Python integers."""
    a = np.asarray(a, dtype=np.uint64).reshape(-1, 4)
    return [int(w[0]) | (int(w[1]) << 64) | (int(w[2]) << 128) | (int(w[3]) << 192) for w in a]


def from_ints(vals) -> np.ndarray:
    """Python integers in [0, 2^256) -> (N, 4) uint64 limbs."""
    vals = list(vals)
    out = np.zeros((len(vals), 4), dtype=np.uint64)
    m = (1 << 64) - 1
    for i, v in enumerate(vals):
        for k in range(4):
            out[i, k] = (v >> (64 * k)) & m
    return out


def modulus() -> int:
    """The modulus the sampler rejects against (for callers that check it)."""
    return _R_INT
