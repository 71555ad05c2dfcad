// Host-side Fr arithmetic used only to build the context's constant tables
// (twiddles, coset powers, byte-limb blocks). Cold path: run once per context.
//
// Four 64-bit limbs; products by Montgomery multiplication in separated
// operand scanning form (full 512-bit product, then word-by-word reduction),
// R = 2^256. Constants R mod r and R^2 mod r are derived from r at start-up.
#pragma once
#include <stdint.h>
#include <string.h>

namespace frntt {
namespace host {

typedef unsigned __int128 u128;

struct Fe {
  uint64_t v[4];
};

static const Fe kR = {{0x43E1F593F0000001ULL, 0x2833E84879B97091ULL, 0xB85045B68181585DULL,
                       0x30644E72E131A029ULL}};

inline bool geq(const Fe& a, const Fe& b) {
  for (int i = 3; i >= 0; --i) {
    if (a.v[i] != b.v[i]) return a.v[i] > b.v[i];
  }
  return true;
}

inline uint64_t sub_in(Fe& a, const Fe& b) {  // a -= b, returns borrow
  uint64_t br = 0;
  for (int i = 0; i < 4; ++i) {
    u128 d = (u128)a.v[i] - b.v[i] - br;
    a.v[i] = (uint64_t)d;
    br = (uint64_t)(d >> 127);
  }
  return br;
}

inline uint64_t add_in(Fe& a, const Fe& b) {
  uint64_t c = 0;
  for (int i = 0; i < 4; ++i) {
    u128 s = (u128)a.v[i] + b.v[i] + c;
    a.v[i] = (uint64_t)s;
    c = (uint64_t)(s >> 64);
  }
  return c;
}

inline Fe add(Fe a, const Fe& b) {
  add_in(a, b);
  if (geq(a, kR)) sub_in(a, kR);
  return a;
}

inline Fe sub(Fe a, const Fe& b) {
  if (sub_in(a, b)) add_in(a, kR);
  return a;
}

inline Fe from_u64(uint64_t x) {
  Fe a = {{x, 0, 0, 0}};
  return a;
}

struct Field {
  uint64_t ninv;  // -r^-1 mod 2^64
  Fe one_m;       // R mod r
  Fe r2;          // R^2 mod r

  Field() {
    // inverse of r mod 2^64 by Hensel lifting
    uint64_t x = 1;
    for (int i = 0; i < 64; ++i) {
      // x <- x * (2 - r*x), doubling precision; 7 rounds suffice, 64 is harmless
      x = x * (2 - kR.v[0] * x);
    }
    ninv = 0 - x;
    Fe a = from_u64(1);
    for (int i = 0; i < 512; ++i) {
      a = add(a, a);
      if (i == 255) one_m = a;
    }
    r2 = a;
  }

  // SOS Montgomery product
  Fe mul_m(const Fe& a, const Fe& b) const {
    uint64_t t[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) {
      uint64_t c = 0;
      for (int j = 0; j < 4; ++j) {
        u128 s = (u128)a.v[i] * b.v[j] + t[i + j] + c;
        t[i + j] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
      }
      t[i + 4] = c;
    }
    for (int i = 0; i < 4; ++i) {
      uint64_t m = t[i] * ninv;
      uint64_t c = 0;
      for (int j = 0; j < 4; ++j) {
        u128 s = (u128)m * kR.v[j] + t[i + j] + c;
        t[i + j] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
      }
      for (int k = i + 4; k < 9 && c; ++k) {
        u128 s = (u128)t[k] + c;
        t[k] = (uint64_t)s;
        c = (uint64_t)(s >> 64);
      }
    }
    Fe o = {{t[4], t[5], t[6], t[7]}};
    if (t[8] || geq(o, kR)) sub_in(o, kR);
    return o;
  }

  Fe to_m(const Fe& a) const { return mul_m(a, r2); }
  Fe from_m(const Fe& a) const { return mul_m(a, from_u64(1)); }
  // canonical product
  Fe mul(const Fe& a, const Fe& b) const { return from_m(mul_m(to_m(a), to_m(b))); }

  Fe pow(const Fe& base, const Fe& e) const {
    Fe acc = one_m, b = to_m(base);
    for (int i = 255; i >= 0; --i) {
      acc = mul_m(acc, acc);
      if ((e.v[i >> 6] >> (i & 63)) & 1) acc = mul_m(acc, b);
    }
    return from_m(acc);
  }
  Fe pow_u64(const Fe& base, uint64_t e) const { return pow(base, from_u64(e)); }

  Fe inv(const Fe& a) const {
    Fe e = kR;
    e.v[0] -= 2;
    return pow(a, e);
  }

  // primitive 2^log_n-th root of unity 5^((r-1)/2^log_n)
  Fe root(int log_n) const {
    Fe e = kR;
    e.v[0] -= 1;
    for (int s = 0; s < log_n; ++s) {  // shift right by one bit, log_n times
      for (int i = 0; i < 4; ++i) e.v[i] = (e.v[i] >> 1) | (i < 3 ? (e.v[i + 1] << 63) : 0);
    }
    return pow(from_u64(5), e);
  }
};

}  // namespace host
}  // namespace frntt
