// Fr arithmetic on 32-bit lanes for gfx950.
//
// An element of the BN254 scalar field is held as eight 32-bit little-endian
// words (the paper's "D 32-bit digits", Related Work: Arithmetic
// Implementations). Products use Montgomery multiplication (the paper's
// "radix Mont" baseline) in a reduced-radix form: nine 29-bit limbs with
// lazy carries, R = 2^261 (see mont_mul). Twiddle constants are kept in
// Montgomery form w*R mod r, so mont_mul(x, w*R) = x*w mod r maps canonical
// inputs to canonical outputs without domain conversions.
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

// ---- Montgomery product on 29-bit limbs -----------------------------------
//
// The product runs on nine 29-bit limbs (261 bits) with 64-bit column
// accumulators: every partial product is below 2^58 and a column collects at
// most 18 of them (a*b and m*r, each limb position once per row of the
// operand scan) plus a carry below 2^36, so it stays below 2^63 and every
// multiply-add is a single 32x32+64-bit instruction with no carry handling
// inside the rows. The Montgomery radix is R = 2^261; -r^-1 mod 2^29 is
// 2^28 - 1 because r = 1 + 2^28 (mod 2^29).
constexpr uint32_t kLimbMask = (1u << 29) - 1;
constexpr uint32_t kNprime29 = 0x0fffffffu;

__host__ __device__ constexpr uint32_t fr_limb29(int k) {
  return k == 0 ? 0x10000001u : k == 1 ? 0x1f0fac9fu : k == 2 ? 0x0e5c2450u : k == 3 ? 0x07d090f3u
       : k == 4 ? 0x1585d283u : k == 5 ? 0x02db40c0u : k == 6 ? 0x00a6e141u : k == 7 ? 0x0e5c2634u
       : 0x0030644eu;
}

// eight 32-bit words -> nine 29-bit limbs (funnel shifts on registers)
__device__ FRNTT_INLINE void to_limbs29(const fr_t& x, uint32_t* l) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const int bit = 29 * k, wi = bit >> 5, sh = bit & 31;
    uint32_t v;
    if (sh + 29 <= 32 || wi + 1 >= 8) v = x.w[wi] >> sh;
    else v = __builtin_amdgcn_alignbit(x.w[wi + 1], x.w[wi], (uint32_t)sh);
    l[k] = v & kLimbMask;
  }
}

// Montgomery product a*b*2^-261 mod r for any a, b < 2^256; canonical
// result. Row i adds a*b_i and m*r (m clears the low limb), then drops one
// limb; the result is below 2r before the final subtraction. The work is
// split into load(), nine row()s and finish(), so that it can also be spread
// over the MFMA issue slots of the matrix form.
struct MontMul {
  uint32_t al[9], bl[9];
  uint64_t t[9];

  __device__ FRNTT_INLINE void load(const fr_t& a, const fr_t& b) {
    to_limbs29(a, al);
    to_limbs29(b, bl);
  }
  __device__ FRNTT_INLINE void row(int i) {
    if (i == 0) {
#pragma unroll
      for (int j = 0; j < 9; ++j) t[j] = (uint64_t)al[j] * bl[0];
    } else {
#pragma unroll
      for (int j = 0; j < 9; ++j) t[j] += (uint64_t)al[j] * bl[i];
    }
    const uint32_t m = ((uint32_t)t[0] * kNprime29) & kLimbMask;
#pragma unroll
    for (int j = 0; j < 9; ++j) t[j] += (uint64_t)m * fr_limb29(j);
    const uint64_t c = t[0] >> 29;
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = t[j + 1];
    t[8] = 0;
    t[0] += c;
  }
  __device__ FRNTT_INLINE fr_t finish() const { return fr_reduce_once(finish_lazy()); }
  // The product before the final subtraction: a value below 2r (< 2^255),
  // congruent to a * b * 2^-261. Enough where the next consumer only needs
  // 32 bytes of a value below 2^256 (the byte digits of the matrix form).
  __device__ FRNTT_INLINE fr_t finish_lazy() const {
    // carry-propagate the columns into 29-bit limbs, then pack 32-bit words
    uint32_t l[9];
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint64_t v = t[j] + c;
      l[j] = (uint32_t)v & kLimbMask;
      c = v >> 29;
    }
    l[8] = (uint32_t)(t[8] + c);
    // word i = bits [32 i, 32 i + 32): limb k from bit sh on, then the next
    // one or two limbs (32-bit shifts; the limbs are below 2^29)
    fr_t o;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int bit = 32 * i, k = bit / 29, sh = bit % 29;
      uint32_t v = l[k] >> sh;
      const int have = 29 - sh;
      if (k + 1 < 9) v |= l[k + 1] << have;
      if (have + 29 < 32 && k + 2 < 9) v |= l[k + 2] << (have + 29);
      o.w[i] = v;
    }
    return o;
  }
};

// Product y w mod r of an unreduced y < 2^290 and a constant w < r by
// Shoup's method (multiplication by a constant with a precomputed quotient
// factor: w' = floor(w 2^290 / r), q = floor(y w' / 2^290), then
// y w - q r lies in [0, 2r)). Here q comes from the columns 8..18 of the
// 29-bit-limb product y w' only (the dropped columns add less than 2^265,
// so the estimate is q or q - 1), and y w - q r is formed modulo 2^261 from
// the low columns of y w and q r (it is below 3r < 2^261): 64 + 45 + 45
// multiply-adds, no reduction of y beforehand and none afterwards. The
// result is below 3r, enough for a consumer that reads only 32 bytes of a
// value below 2^256. The work is cut into kSteps steps (see step()).
struct ShoupMul {
  static constexpr int kSteps = 12;
  uint32_t a[10];  // y as ten 29-bit limbs
  uint64_t h[11];  // columns 8..18 of y w'
  uint32_t q[9];   // the quotient estimate mod 2^261, nine limbs
  int64_t lo[9];   // columns 0..8 of y w - q r
  fr_t out;

  // rows i in [I0, I1) of the high columns
  template <int I0, int I1>
  __device__ FRNTT_INLINE void hi_rows(const uint32_t* wp) {
#pragma unroll
    for (int i = I0; i < I1; ++i)
#pragma unroll
      for (int j = (8 - i > 0 ? 8 - i : 0); j < 10; ++j) {
        const int c = i + j - 8;
        const uint64_t p = (uint64_t)a[i] * wp[j];
        // first product of column c comes from row max(0, c - 1)
        if (i == (c - 1 > 0 ? c - 1 : 0)) h[c] = p;
        else h[c] += p;
      }
  }
  // rows i in [I0, I1) of the low columns: + a_i w_j - q_i r_j
  template <int I0, int I1>
  __device__ FRNTT_INLINE void lo_rows(const uint32_t* w) {
#pragma unroll
    for (int i = I0; i < I1; ++i)
#pragma unroll
      for (int j = 0; i + j < 9; ++j) {
        const int c = i + j;
        const uint64_t p = (uint64_t)a[i] * w[j];
        int64_t acc = i == 0 ? (int64_t)p : lo[c] + (int64_t)p;
        acc += (int64_t)(int32_t)q[i] * (int64_t)(-(int32_t)fr_limb29(j));
        lo[c] = acc;
      }
  }
  // step Q of kSteps; wp, w: the Shoup operand form of the constant; y: nine
  // words of the input (y < 2^290)
  template <int Q>
  __device__ FRNTT_INLINE void step(const uint32_t* wp, const uint32_t* w, const uint32_t* y) {
    if constexpr (Q == 0) {
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        const int bit = 29 * k, wi = bit >> 5, sh = bit & 31;
        uint32_t v;
        if (sh + 29 <= 32 || wi + 1 >= 9) v = y[wi] >> sh;
        else v = __builtin_amdgcn_alignbit(y[wi + 1], y[wi], (uint32_t)sh);
        a[k] = v & kLimbMask;
      }
    } else if constexpr (Q == 1) {
      hi_rows<0, 4>(wp);
    } else if constexpr (Q == 2) {
      hi_rows<4, 6>(wp);
    } else if constexpr (Q == 3) {
      hi_rows<6, 8>(wp);
    } else if constexpr (Q == 4) {
      hi_rows<8, 9>(wp);
    } else if constexpr (Q == 5) {
      hi_rows<9, 10>(wp);
    } else if constexpr (Q == 6) {
      // q = floor(sum_(c >= 8) h_c 2^(29 c) / 2^290): carry through columns
      // 8 and 9, then columns 10..18 give the limbs of q
      uint64_t c = h[0] >> 29;
      c = (h[1] + c) >> 29;
#pragma unroll
      for (int m = 0; m < 9; ++m) {
        const uint64_t v = h[2 + m] + c;
        q[m] = (uint32_t)v & kLimbMask;
        c = v >> 29;
      }
    } else if constexpr (Q == 7) {
      lo_rows<0, 1>(w);
    } else if constexpr (Q == 8) {
      lo_rows<1, 3>(w);
    } else if constexpr (Q == 9) {
      lo_rows<3, 6>(w);
    } else if constexpr (Q == 10) {
      lo_rows<6, 9>(w);
    } else {
      // signed carries give the nine limbs of y w - q r mod 2^261 (the value
      // itself: it lies in [0, 3r)); then eight 32-bit words
      uint32_t l[9];
      int64_t c = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int64_t v = lo[k] + c;
        l[k] = (uint32_t)v & kLimbMask;
        c = v >> 29;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int bit = 32 * i, k = bit / 29, sh = bit % 29;
        uint32_t v = l[k] >> sh;
        const int have = 29 - sh;
        if (k + 1 < 9) v |= l[k + 1] << have;
        if (have + 29 < 32 && k + 2 < 9) v |= l[k + 2] << (have + 29);
        out.w[i] = v;
      }
    }
  }
};

__device__ FRNTT_INLINE fr_t mont_mul(const fr_t& a, const fr_t& b) {
  MontMul mm;
  mm.load(a, b);
#pragma unroll
  for (int i = 0; i < 9; ++i) mm.row(i);
  return mm.finish();
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
