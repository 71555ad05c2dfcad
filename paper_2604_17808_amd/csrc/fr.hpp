// Fr arithmetic on 32-bit lanes for gfx950.
//
// An element of the BN254 scalar field is held as eight 32-bit little-endian
// words (the paper's "D 32-bit digits", Related Work: Arithmetic
// Implementations). Products use Montgomery multiplication with R = 2^256
// (the paper's "radix Mont" baseline), in the coarsely integrated operand
// scanning form with the carry-free inner step of Botrel and El Housni
// ("Faster big-integer modular multiplication for most moduli", 2020), which
// applies because the top word of r is below 2^31 - 1. Twiddle constants are
// kept in Montgomery form w*R mod r, so mont_mul(x, w*R) = x*w mod r maps
// canonical inputs to canonical outputs without domain conversions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FRNTT_INLINE __attribute__((always_inline)) inline

namespace frntt {

struct fr_t {
  uint32_t w[8];
};

// r = 0x30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001
#define FR_R0 0xf0000001u
#define FR_R1 0x43e1f593u
#define FR_R2 0x79b97091u
#define FR_R3 0x2833e848u
#define FR_R4 0x8181585du
#define FR_R5 0xb85045b6u
#define FR_R6 0xe131a029u
#define FR_R7 0x30644e72u
#define FR_NPRIME 0xefffffffu  // -r^-1 mod 2^32

__host__ __device__ constexpr uint32_t fr_mod_word(int i) {
  return i == 0 ? FR_R0 : i == 1 ? FR_R1 : i == 2 ? FR_R2 : i == 3 ? FR_R3
       : i == 4 ? FR_R4 : i == 5 ? FR_R5 : i == 6 ? FR_R6 : FR_R7;
}

__device__ FRNTT_INLINE uint32_t addc(uint32_t a, uint32_t b, uint32_t cin, uint32_t* cout) {
  uint32_t c;
  uint32_t s = __builtin_addc(a, b, cin, &c);
  *cout = c;
  return s;
}

__device__ FRNTT_INLINE uint32_t subb(uint32_t a, uint32_t b, uint32_t bin, uint32_t* bout) {
  uint32_t c;
  uint32_t s = __builtin_subc(a, b, bin, &c);
  *bout = c;
  return s;
}

// If x >= r then x - r else x, for x < 2^256 with x < 2r.
__device__ FRNTT_INLINE fr_t fr_reduce_once(const fr_t& x) {
  fr_t d;
  uint32_t b = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d.w[i] = subb(x.w[i], fr_mod_word(i), b, &b);
  // borrow set -> x < r -> keep x
  fr_t o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = b ? x.w[i] : d.w[i];
  return o;
}

__device__ FRNTT_INLINE fr_t fr_add(const fr_t& a, const fr_t& b) {
  fr_t s;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s.w[i] = addc(a.w[i], b.w[i], c, &c);
  return fr_reduce_once(s);  // a + b < 2r < 2^255: no carry out
}

__device__ FRNTT_INLINE fr_t fr_sub(const fr_t& a, const fr_t& b) {
  fr_t d;
  uint32_t br = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d.w[i] = subb(a.w[i], b.w[i], br, &br);
  // on borrow add r back
  uint32_t mask = 0u - br;
  fr_t o;
  uint32_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = addc(d.w[i], fr_mod_word(i) & mask, c, &c);
  return o;
}

// x + y as a 64-bit value (carry in the high word). Written with an explicit
// add-with-carry so the pair feeds v_mad_u64_u32 directly, without
// zero-extension moves.
__device__ FRNTT_INLINE uint64_t add_2x32(uint32_t x, uint32_t y) {
  uint32_t carry;
  const uint32_t lo = __builtin_addc(x, y, 0u, &carry);
  return ((uint64_t)carry << 32) | lo;
}

// Montgomery product a*b*2^-256 mod r for a, b < r; result canonical.
// Row i adds a*b_i and m*r with m chosen to clear the low word, then shifts
// one word; the two carry chains of a row are interleaved (A for a*b_i, C
// for m*r), each step one 32x32+64 multiply-add.
__device__ FRNTT_INLINE fr_t mont_mul(const fr_t& a, const fr_t& b) {
  uint32_t t[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) t[j] = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t p = (uint64_t)a.w[0] * b.w[i] + t[0];
    uint32_t A = (uint32_t)(p >> 32);
    const uint32_t t0 = (uint32_t)p;
    const uint32_t m = t0 * FR_NPRIME;
    uint64_t q = (uint64_t)m * FR_R0 + t0;
    uint32_t C = (uint32_t)(q >> 32);
#pragma unroll
    for (int j = 1; j < 8; ++j) {
      p = (uint64_t)a.w[j] * b.w[i] + add_2x32(t[j], A);
      A = (uint32_t)(p >> 32);
      q = (uint64_t)m * fr_mod_word(j) + add_2x32((uint32_t)p, C);
      C = (uint32_t)(q >> 32);
      t[j - 1] = (uint32_t)q;
    }
    t[7] = C + A;
  }
  fr_t o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o.w[j] = t[j];
  return fr_reduce_once(o);
}

// 2r as eight 32-bit words.
__host__ __device__ constexpr uint32_t two_r_word(int i) {
  uint64_t c = 0;
  uint32_t w = 0;
  for (int j = 0; j <= i; ++j) {
    uint64_t s = (uint64_t)fr_mod_word(j) * 2 + c;
    w = (uint32_t)s;
    c = s >> 32;
  }
  return w;
}

// y < 3r (eight words) -> y mod r: subtract 2r, then r, where no borrow
__device__ FRNTT_INLINE void cond_sub_words(uint32_t* y, bool twice) {
  uint32_t d[8], b = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d[i] = subb(y[i], twice ? two_r_word(i) : fr_mod_word(i), b, &b);
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = b ? y[i] : d[i];
}

// y < 3r -> y mod r
__device__ FRNTT_INLINE fr_t fr_reduce_3r(const fr_t& x) {
  uint32_t y[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = x.w[i];
  cond_sub_words(y, true);
  cond_sub_words(y, false);
  fr_t o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = y[i];
  return o;
}

__device__ FRNTT_INLINE fr_t fr_zero() {
  fr_t z;
#pragma unroll
  for (int i = 0; i < 8; ++i) z.w[i] = 0;
  return z;
}

}  // namespace frntt
