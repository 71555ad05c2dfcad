// Constant tables of a context, built on the host once and copied to HBM.
//
// * twiddles: the paper generates its twiddle matrices offline (Fig. 4
//   caption) and notes that tables growing with N run out of memory (3-step
//   NTT, Introduction); here the pass twiddles w_M^e for any M <= 2^28 come
//   from two 2^14-entry tables of w_{2^28} powers and one extra product;
//   in-pass twiddles come from one 4096-entry table, kept a second time for
//   the matrix form's inter-level twiddles in the operand form of its Shoup
//   product: w as nine 29-bit limbs and w' = floor(w 2^290 / r) as ten.
// * byte-limb constant blocks for the matrix form (Alg. 1, Precomputation:
//   the BAT-shifted constants I_{i,b} = ... << 8b mod Q and their byte split
//   E[i,b,j,h]): for a radix rho, block j holds the signed base-256 digits
//   e_h of w_rho^j * 2^(8a) mod r for a, h in [0, 32).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "frntt_internal.hpp"
#include "host_field.hpp"

namespace frntt {

namespace {

using host::Fe;
using host::Field;

void put_elem(uint8_t* dst, const Fe& a) { std::memcpy(dst, a.v, 32); }

uint8_t byte_of(const Fe& a, int h) { return (uint8_t)(a.v[h >> 3] >> (8 * (h & 7))); }

// 29-bit limbs of a little-endian word array (limb k = bits [29k, 29k + 29))
void limbs29(const uint32_t* w, int nwords, uint32_t* l, int nlimbs) {
  for (int k = 0; k < nlimbs; ++k) {
    uint32_t v = 0;
    for (int b = 0; b < 29; ++b) {
      const int bit = 29 * k + b;
      if (bit < 32 * nwords && ((w[bit >> 5] >> (bit & 31)) & 1)) v |= 1u << b;
    }
    l[k] = v;
  }
}

// x * y mod 2^(32 n) on n-word little-endian integers
void mul_lo(const uint32_t* x, const uint32_t* y, uint32_t* out, int n) {
  std::vector<uint32_t> o(n, 0);
  for (int i = 0; i < n; ++i) {
    uint64_t c = 0;
    for (int j = 0; i + j < n; ++j) {
      const uint64_t t = (uint64_t)x[i] * y[j] + o[i + j] + c;
      o[i + j] = (uint32_t)t;
      c = t >> 32;
    }
  }
  for (int i = 0; i < n; ++i) out[i] = o[i];
}

constexpr int kShoupK = 290;   // w' = floor(w 2^290 / r): products of inputs below 2^290
constexpr int kDivWords = 10;  // w' < 2^290 < 2^320

// The Shoup operand form of a canonical w: words 0..9 the ten 29-bit limbs of
// w' = floor(w 2^290 / r), words 10..18 the nine limbs of w, word 19 zero.
// w 2^290 - (w 2^290 mod r) is a multiple of r, and w' below 2^320, so w' is
// that difference times r^-1 mod 2^320 (exact division by an odd divisor).
struct ShoupForm {
  Field F;
  Fe two_k;                     // 2^290 mod r
  uint32_t rinv[kDivWords];     // r^-1 mod 2^320
  ShoupForm() {
    two_k = host::from_u64(1);
    for (int i = 0; i < kShoupK; ++i) two_k = host::add(two_k, two_k);
    uint32_t r[kDivWords] = {};
    for (int i = 0; i < 8; ++i) r[i] = fr_mod_word(i);
    // Newton iteration x <- x (2 - r x) doubles the correct low bits: 1 -> 512
    uint32_t x[kDivWords] = {1};
    for (int it = 0; it < 9; ++it) {
      uint32_t rx[kDivWords], two_minus[kDivWords], nx[kDivWords];
      mul_lo(r, x, rx, kDivWords);
      uint64_t br = 0;
      for (int i = 0; i < kDivWords; ++i) {  // 2 - r x mod 2^320
        const uint64_t d = (uint64_t)(i == 0 ? 2u : 0u) - rx[i] - br;
        two_minus[i] = (uint32_t)d;
        br = (d >> 32) & 1;
      }
      mul_lo(x, two_minus, nx, kDivWords);
      std::memcpy(x, nx, sizeof x);
    }
    std::memcpy(rinv, x, sizeof rinv);
  }
  void put(uint8_t* dst, const Fe& w) const {
    const Fe rem = F.mul(w, two_k);  // w 2^290 mod r
    // D = w 2^290 - rem, low 320 bits (w 2^290 has zero low 290 bits)
    uint32_t D[kDivWords] = {};
    for (int bit = 0; bit < 320; ++bit) {
      const int src = bit - kShoupK;
      if (src >= 0 && src < 256 && ((w.v[src >> 6] >> (src & 63)) & 1)) D[bit >> 5] |= 1u << (bit & 31);
    }
    uint64_t br = 0;
    for (int i = 0; i < kDivWords; ++i) {
      const uint32_t rw = i < 8 ? (uint32_t)(rem.v[i >> 1] >> (32 * (i & 1))) : 0u;
      const uint64_t d = (uint64_t)D[i] - rw - br;
      D[i] = (uint32_t)d;
      br = (d >> 32) & 1;
    }
    uint32_t wp[kDivWords];
    mul_lo(D, rinv, wp, kDivWords);
    uint32_t words[20] = {};
    limbs29(wp, kDivWords, words, 10);
    uint32_t ww[8];
    for (int i = 0; i < 8; ++i) ww[i] = (uint32_t)(w.v[i >> 1] >> (32 * (i & 1)));
    limbs29(ww, 8, words + 10, 9);
    std::memcpy(dst, words, 80);
  }
};

// Signed base-256 digits of a canonical value: sum_h e_h 256^h = a, e_h in [-128, 127].
void signed_digits(const Fe& a, int8_t e[32]) {
  int carry = 0;
  for (int h = 0; h < 32; ++h) {
    int d = byte_of(a, h) + carry;
    if (d >= 128) {
      e[h] = (int8_t)(d - 256);
      carry = 1;
    } else {
      e[h] = (int8_t)d;
      carry = 0;
    }
  }
  // top byte of a value < r is at most 0x30, so the last carry is zero
}

struct Layout {
  size_t tw_lo[2], tw_hi[2], w4096[2], w4096_s[2], g_lo[2], g_hi[2], ninv;
  size_t bat[2][6], bat_init[2][6];
  size_t total;
};

Layout make_layout() {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  for (int d = 0; d < 2; ++d) {
    L.tw_lo[d] = take((size_t)32 << kSplit);
    L.tw_hi[d] = take((size_t)32 << kSplit);
    L.w4096[d] = take(32 * 4096);
    L.w4096_s[d] = take(80 * 4096);
    L.g_lo[d] = take((size_t)32 << kSplit);
    L.g_hi[d] = take((size_t)32 << kSplit);
  }
  L.ninv = take(32 * 29);
  for (int d = 0; d < 2; ++d)
    for (int m = 1; m <= 5; ++m) {
      L.bat[d][m] = take((size_t)1024 << m);
      L.bat_init[d][m] = take((size_t)128 << m);
    }
  L.total = off;
  return L;
}

}  // namespace

// Builds every table into host memory `h` (layout from make_layout).
static void fill_tables(uint8_t* h, const Layout& L) {
  Field F;
  const Fe one = host::from_u64(1);
  // the device Montgomery radix R = 2^261: a table entry for w holds w * R mod r
  Fe dev_r = one;
  for (int i = 0; i < 261; ++i) dev_r = host::add(dev_r, dev_r);
  auto dev_m = [&](const Fe& x) { return F.mul(x, dev_r); };
  const ShoupForm shoup;
  Fe w28[2];
  w28[0] = F.root(kMasterLog);
  w28[1] = F.inv(w28[0]);
  const Fe g[2] = {host::from_u64(5), F.inv(host::from_u64(5))};
  for (int d = 0; d < 2; ++d) {
    // w28^j and w28^(2^14 j)
    Fe step_hi = F.pow_u64(w28[d], 1ull << kSplit);
    Fe p = one, q = one;
    for (int j = 0; j < (1 << kSplit); ++j) {
      put_elem(h + L.tw_lo[d] + 32 * (size_t)j, dev_m(p));
      put_elem(h + L.tw_hi[d] + 32 * (size_t)j, dev_m(q));
      p = F.mul(p, w28[d]);
      q = F.mul(q, step_hi);
    }
    // w_4096^j
    Fe w4096 = F.pow_u64(w28[d], 1ull << (kMasterLog - 12));
    p = one;
    for (int j = 0; j < 4096; ++j) {
      put_elem(h + L.w4096[d] + 32 * (size_t)j, dev_m(p));
      shoup.put(h + L.w4096_s[d] + 80 * (size_t)j, p);
      p = F.mul(p, w4096);
    }
    // g^(+-j) and g^(+-(2^14 j))
    Fe g_hi_step = F.pow_u64(g[d], 1ull << kSplit);
    p = one;
    q = one;
    for (int j = 0; j < (1 << kSplit); ++j) {
      put_elem(h + L.g_lo[d] + 32 * (size_t)j, dev_m(p));
      put_elem(h + L.g_hi[d] + 32 * (size_t)j, dev_m(q));
      p = F.mul(p, g[d]);
      q = F.mul(q, g_hi_step);
    }
  }
  // 2^-L
  Fe half = F.inv(host::from_u64(2)), p = one;
  for (int l = 0; l <= 28; ++l) {
    put_elem(h + L.ninv + 32 * (size_t)l, dev_m(p));
    p = F.mul(p, half);
  }
  // Row offsets of the accumulator seeds: row h starts at 2^25 + delta_h,
  // which lifts every byte-plane partial sum_(n,a) E * u (|.| < 2^25 for
  // radices up to 32) into [0, 2^26), so the merge runs on unsigned
  // integers. The delta_h are the bytes of D = -O mod r for
  // O = 2^25 * sum_h 2^(8h), so the offsets add O + D = 0 (mod r).
  Fe o_mod = host::from_u64(0), p256 = one;
  for (int hh = 0; hh < 32; ++hh) {
    o_mod = host::add(o_mod, p256);
    for (int s8 = 0; s8 < 8; ++s8) p256 = host::add(p256, p256);
  }
  for (int s25 = 0; s25 < 25; ++s25) o_mod = host::add(o_mod, o_mod);
  const Fe dlt = host::sub(host::from_u64(0), o_mod);
  int32_t beta[32];
  for (int hh = 0; hh < 32; ++hh) beta[hh] = (1 << 25) + (int32_t)byte_of(dlt, hh);
  // byte-limb blocks per radix
  for (int d = 0; d < 2; ++d) {
    for (int m = 1; m <= 5; ++m) {
      const int rho = 1 << m;
      const Fe wr = F.pow_u64(w28[d], 1ull << (kMasterLog - m));
      std::vector<int8_t> dig((size_t)rho * 32 * 32);  // [j][a][h]
      Fe wj = one;
      for (int j = 0; j < rho; ++j) {
        Fe c = wj;
        for (int a = 0; a < 32; ++a) {
          signed_digits(c, &dig[((size_t)j * 32 + a) * 32]);
          c = host::add(c, c);  // *2 eight times = *256
          for (int s = 0; s < 7; ++s) c = host::add(c, c);
        }
        wj = F.mul(wj, wr);
      }
      int8_t* blk = (int8_t*)(h + L.bat[d][m]);
      for (int j = 0; j < rho; ++j)
        for (int lane = 0; lane < 64; ++lane)
          for (int i = 0; i < 16; ++i) {
            const int hh = lane & 31, a = 16 * (lane >> 5) + i;
            blk[(size_t)j * 1024 + lane * 16 + i] = dig[((size_t)j * 32 + a) * 32 + hh];
          }
      // Seeds of the even/odd accumulators of output pair k' < rho/2 (the
      // even-digit sum e and the odd-digit sum o of w^(k' n) x_n; outputs k'
      // and k' + rho/2 are e + o and e - o): the signed-digit correction
      // 128 * sum_(n of that parity, a) E[(k',h),(n,a)] for each row h, plus
      // the row offsets on the even accumulator only, so that both e + o and
      // e - o carry them once.
      int32_t* init = (int32_t*)(h + L.bat_init[d][m]);
      for (int k = 0; k < rho / 2; ++k)
        for (int par = 0; par < 2; ++par) {
          int32_t S[32] = {0};
          for (int n = par; n < rho; n += 2) {
            const int j = (k * n) & (rho - 1);
            for (int a = 0; a < 32; ++a)
              for (int hh = 0; hh < 32; ++hh) S[hh] += dig[((size_t)j * 32 + a) * 32 + hh];
          }
          for (int half2 = 0; half2 < 2; ++half2)
            for (int rg = 0; rg < 16; ++rg) {
              const int hh = 8 * (rg >> 2) + 4 * half2 + (rg & 3);
              init[((2 * k + par) * 2 + half2) * 16 + rg] = 128 * S[hh] + (par == 0 ? beta[hh] : 0);
            }
        }
    }
  }
}

int build_tables(frntt_ctx* ctx) {
  const Layout L = make_layout();
  std::vector<uint8_t> h(L.total, 0);
  fill_tables(h.data(), L);
  void* dmem = nullptr;
  hipError_t e = hipMalloc(&dmem, L.total);
  if (e != hipSuccess) {
    set_hip_error(ctx, e);
    return FRNTT_ENOMEM;
  }
  e = hipMemcpy(dmem, h.data(), L.total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(dmem);
    return set_hip_error(ctx, e);
  }
  ctx->table_mem = dmem;
  ctx->table_bytes = L.total;
  uint8_t* b = (uint8_t*)dmem;
  DevTables& T = ctx->tables;
  for (int d = 0; d < 2; ++d) {
    T.tw_lo[d] = (const u32x4*)(b + L.tw_lo[d]);
    T.tw_hi[d] = (const u32x4*)(b + L.tw_hi[d]);
    T.w4096[d] = (const u32x4*)(b + L.w4096[d]);
    T.w4096_s[d] = (const u32x4*)(b + L.w4096_s[d]);
    T.g_lo[d] = (const u32x4*)(b + L.g_lo[d]);
    T.g_hi[d] = (const u32x4*)(b + L.g_hi[d]);
    T.bat[d][0] = nullptr;
    T.bat_init[d][0] = nullptr;
    for (int m = 1; m <= 5; ++m) {
      T.bat[d][m] = (const i32x4*)(b + L.bat[d][m]);
      T.bat_init[d][m] = (const i32x4*)(b + L.bat_init[d][m]);
    }
  }
  T.ninv = (const u32x4*)(b + L.ninv);
  T.byte_w[0] = 1u << 8;
  T.byte_w[1] = 1u << 16;
  T.byte_w[2] = 1u << 24;
  T.byte_w[3] = 1u;
  return FRNTT_OK;
}

}  // namespace frntt
