// The MXU-centric RNS lazy modular product (paper: Arithmetic Optimizations,
// "Solution: Reducing O(D^2) Reduction via MXU-Centric RNS Lazy Reduction",
// the walk-through example, and Alg. 1 "MXU RNS Lazy") on gfx950.
//
// A field element x in [0, r) is carried in an extended non-prime ring Z_Q,
// Q = q_0 ... q_16 > 2 r^2, as its residues x z mod q_i (z = 2^32: the
// residue-wise Montgomery form). A product of two elements is then
//   1. residue-wise: x_i = a_i b_i z^-1 mod q_i (one 32x32-bit Montgomery
//      product per residue, no carries across residues; VALU);
//   2. Alg. 1 Main: one int8 matrix product of the residues' bytes
//      [x]_(i,b) with the constant table E[i,b,j,h] (the bytes of
//      z (I_(i,b) mod r) mod p_j, I_(i,b) the CRT coefficient of residue i
//      times z^-1, shifted by 2^(8b) mod Q), fused with the rows of
//      f_(i,b) = ceil(I_(i,b) 2^u / Q) whose sum v gives the overflow count
//      k = floor(v / 2^u); then per residue j of the base P the byte merge,
//      + k g_j and the reduction to [0, p_j).
// The result is the lazily reduced product W' (|W'| < 2^15 r, W' = a b mod r)
// in base P, residues W' z mod p_j.
//
// Around the product: the encode (canonical value -> base-Q residues) is the
// same byte matrix product with the bytes of z 2^(8b) mod q_i; the decode
// (base P -> canonical) applies Main once more with the base P as the source
// and the 32 bytes of a 256-bit word as the target (the constants are the
// bytes of I^P_(j,b) mod r), rounds k to the nearest integer so that a
// negative W' comes out right, adds k ((-P) mod r), and reduces below r.
//
// MFMA use: v_mfma_i32_32x32x32_i8 with the constant table as the A operand
// (rows = output bytes) and 32 elements as the columns of B (each lane loads
// 16 bytes of one element straight from HBM: the B fragment layout). Bytes
// u in [0, 255] enter as u - 128 and the constants as signed base-256
// digits; the accumulator seeds add back 128 x the digit sums of each row.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "fr.hpp"
#include "frntt_internal.hpp"
#include "rns_lazy.hpp"

namespace frntt {

namespace {

// ------------------------------------------------------------------ host

// Unsigned integers of a few hundred bits (table construction only).
struct Big {
  std::vector<uint32_t> w;  // little-endian words, no leading zero words

  Big() = default;
  explicit Big(uint64_t v) {
    while (v) {
      w.push_back((uint32_t)v);
      v >>= 32;
    }
  }
  void trim() {
    while (!w.empty() && w.back() == 0) w.pop_back();
  }
  int bits() const {
    if (w.empty()) return 0;
    return 32 * ((int)w.size() - 1) + (32 - __builtin_clz(w.back()));
  }
  bool bit(int i) const { return (size_t)(i >> 5) < w.size() && ((w[i >> 5] >> (i & 31)) & 1); }
  uint32_t word(int i) const { return (size_t)i < w.size() ? w[i] : 0u; }
};

int cmp(const Big& a, const Big& b) {
  if (a.w.size() != b.w.size()) return a.w.size() < b.w.size() ? -1 : 1;
  for (int i = (int)a.w.size() - 1; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
  return 0;
}

Big add(const Big& a, const Big& b) {
  Big r;
  uint64_t c = 0;
  const size_t n = std::max(a.w.size(), b.w.size());
  for (size_t i = 0; i < n; ++i) {
    c += (uint64_t)a.word((int)i) + b.word((int)i);
    r.w.push_back((uint32_t)c);
    c >>= 32;
  }
  if (c) r.w.push_back((uint32_t)c);
  r.trim();
  return r;
}

Big sub(const Big& a, const Big& b) {  // a >= b
  Big r;
  int64_t br = 0;
  for (size_t i = 0; i < a.w.size(); ++i) {
    int64_t d = (int64_t)a.w[i] - b.word((int)i) - br;
    br = d < 0;
    r.w.push_back((uint32_t)(d + (br << 32)));
  }
  r.trim();
  return r;
}

Big mul_small(const Big& a, uint32_t m) {
  Big r;
  uint64_t c = 0;
  for (uint32_t x : a.w) {
    c += (uint64_t)x * m;
    r.w.push_back((uint32_t)c);
    c >>= 32;
  }
  if (c) r.w.push_back((uint32_t)c);
  r.trim();
  return r;
}

Big shl(const Big& a, int s) {
  Big r;
  r.w.assign(a.w.size() + s / 32 + 1, 0);
  for (size_t i = 0; i < a.w.size(); ++i) {
    const uint64_t v = (uint64_t)a.w[i] << (s % 32);
    r.w[i + s / 32] |= (uint32_t)v;
    r.w[i + s / 32 + 1] |= (uint32_t)(v >> 32);
  }
  r.trim();
  return r;
}

// a = qt * m + rem (m small)
uint32_t divmod_small(const Big& a, uint32_t m, Big* qt) {
  uint64_t rem = 0;
  Big q;
  q.w.assign(a.w.size(), 0);
  for (int i = (int)a.w.size() - 1; i >= 0; --i) {
    const uint64_t cur = (rem << 32) | a.w[i];
    q.w[i] = (uint32_t)(cur / m);
    rem = cur % m;
  }
  q.trim();
  if (qt) *qt = q;
  return (uint32_t)rem;
}

// a = qt * m + rem, schoolbook binary long division
Big divmod(const Big& a, const Big& m, Big* qt) {
  Big r, q;
  q.w.assign(a.w.size() + 1, 0);
  for (int i = a.bits() - 1; i >= 0; --i) {
    r = shl(r, 1);
    if (a.bit(i)) {
      if (r.w.empty()) r.w.push_back(0);
      r.w[0] |= 1;
    }
    if (cmp(r, m) >= 0) {
      r = sub(r, m);
      q.w[i >> 5] |= 1u << (i & 31);
    }
  }
  q.trim();
  if (qt) *qt = q;
  return r;
}

uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = r * b % m;
    b = b * b % m;
    e >>= 1;
  }
  return r;
}

// Deterministic Miller-Rabin for n < 2^32 (bases 2, 7, 61).
bool is_prime32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
    if (n % p == 0) return n == p;
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int t = 1; t < s; ++t) {
      x = x * x % n;
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

// q_0 > ... > q_16 > p_0 > ... > p_8: consecutive primes below kRnsBound.
void rns_moduli(uint32_t* q, uint32_t* p) {
  uint32_t n = kRnsBound - 1;
  int got = 0;
  while (got < kRnsI + kRnsJ) {
    if (is_prime32(n)) {
      if (got < kRnsI) q[got] = n;
      else p[got - kRnsI] = n;
      ++got;
    }
    n -= 1;
  }
}

// Signed base-256 digits: sum_h e_h 256^h = c.
void signed_digits(const Big& c, int n, int8_t* e) {
  int carry = 0;
  for (int h = 0; h < n; ++h) {
    const int d = (int)((c.word(h / 4) >> (8 * (h % 4))) & 255) + carry;
    if (d >= 128) {
      e[h] = (int8_t)(d - 256);
      carry = 1;
    } else {
      e[h] = (int8_t)d;
      carry = 0;
    }
  }
}

// A-fragment table and seeds of a signed-digit matrix A[row][k] (RB x 32 rows,
// KS x 32 columns).
void pack_table(const std::vector<int8_t>& A, int RB, int KS, uint8_t* frag, int32_t* seeds) {
  const int K = 32 * KS;
  for (int rb = 0; rb < RB; ++rb)
    for (int s = 0; s < KS; ++s)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 16; ++t) {
          const int row = 32 * rb + (lane & 31), k = 32 * s + 16 * (lane >> 5) + t;
          frag[((size_t)(rb * KS + s) * 64 + lane) * 16 + t] = (uint8_t)A[(size_t)row * K + k];
        }
  for (int rb = 0; rb < RB; ++rb)
    for (int half = 0; half < 2; ++half)
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + 8 * (r / 4) + 4 * half + r % 4;
        int32_t sum = 0;
        for (int k = 0; k < K; ++k) sum += A[(size_t)row * K + k];
        seeds[(rb * 2 + half) * 16 + r] = 128 * sum;
      }
}

Big field_modulus() {
  Big m;
  for (int i = 0; i < 8; ++i) m.w.push_back(fr_mod_word(i));
  m.trim();
  return m;
}

// Precomputation of Alg. 1 for source base `src` (n_src moduli): the CRT
// coefficients I_s = (Q/q_s) ((Q/q_s)^-1 z^-1 mod q_s) (so that
// sum_s x_s I_s = X mod Q for Montgomery-form residues x_s = X z mod q_s),
// shifted by 2^(8b) mod Q, and f_(s,b) = ceil(I_(s,b) 2^u / Q).
struct SourceBase {
  Big Q;
  std::vector<Big> Ib;          // [s * 4 + b]
  std::vector<uint32_t> f;      // [s * 4 + b]
};

SourceBase source_base(const uint32_t* m, int n) {
  SourceBase S;
  S.Q = Big(1);
  for (int s = 0; s < n; ++s) S.Q = mul_small(S.Q, m[s]);
  for (int s = 0; s < n; ++s) {
    Big Qs;
    divmod_small(S.Q, m[s], &Qs);
    const uint64_t qs_mod = divmod_small(Qs, m[s], nullptr);
    const uint64_t c = powmod(qs_mod, m[s] - 2, m[s]);                   // (Q/q_s)^-1 mod q_s
    const uint64_t zinv = powmod(powmod(2, 32, m[s]), m[s] - 2, m[s]);  // z^-1 mod q_s
    const Big I = mul_small(Qs, (uint32_t)(c * zinv % m[s]));
    for (int b = 0; b < 4; ++b) {
      const Big Ib = divmod(shl(I, 8 * b), S.Q, nullptr);
      S.Ib.push_back(Ib);
      Big fq;
      // ceil(Ib 2^u / Q) = floor((Ib 2^u + Q - 1) / Q)
      divmod(sub(add(shl(Ib, kRnsU), S.Q), Big(1)), S.Q, &fq);
      S.f.push_back(fq.word(0));
    }
  }
  return S;
}

}  // namespace

int build_rns_tables(frntt_ctx* ctx) {
  RnsConsts C{};
  uint32_t q[kRnsI], p[kRnsJ];
  rns_moduli(q, p);
  for (int i = 0; i < 24; ++i) {
    C.q[i] = i < kRnsI ? q[i] : 1u;
    // -q^-1 mod 2^32 by Newton iteration (q odd)
    uint32_t inv = C.q[i];
    for (int it = 0; it < 5; ++it) inv *= 2u - C.q[i] * inv;
    C.qneg[i] = 0u - inv;
    C.qinv[i] = 1.0 / (double)C.q[i];
  }
  for (int j = 0; j < 12; ++j) {
    C.p[j] = j < kRnsJ ? p[j] : 1u;
    C.pinv[j] = 1.0 / (double)C.p[j];
  }
  const Big M = field_modulus();

  // ---- Alg. 1 Main: source base Q, target base P
  const SourceBase SQ = source_base(q, kRnsI);
  const Big QmodM = divmod(SQ.Q, M, nullptr);
  for (int j = 0; j < kRnsJ; ++j) {
    const uint64_t zj = powmod(2, 32, p[j]);
    const uint64_t qm = divmod_small(QmodM, p[j], nullptr);
    C.g[j] = (uint32_t)((p[j] - zj * qm % p[j]) % p[j]);
  }
  std::vector<int8_t> Amul((size_t)64 * 96, 0);
  for (int i = 0; i < kRnsI; ++i)
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * i + b;
      const Big IbM = divmod(SQ.Ib[k], M, nullptr);
      for (int j = 0; j < kRnsJ; ++j) {
        const uint64_t zj = powmod(2, 32, p[j]);
        const uint64_t c = zj * divmod_small(IbM, p[j], nullptr) % p[j];
        int8_t e[4];
        signed_digits(Big(c), 4, e);
        for (int h = 0; h < 4; ++h) Amul[(size_t)(4 * j + h) * 96 + k] = e[h];
      }
      int8_t e[3];
      signed_digits(Big(SQ.f[k]), 3, e);
      for (int t = 0; t < 3; ++t) Amul[(size_t)(36 + t) * 96 + k] = e[t];
    }

  // ---- encode: bytes of a 256-bit word -> residues z 2^(8b) mod q_i
  std::vector<int8_t> Aenc((size_t)96 * 32, 0);
  for (int i = 0; i < kRnsI; ++i)
    for (int b = 0; b < 32; ++b) {
      const uint64_t c = powmod(2, 32 + 8 * b, q[i]);
      int8_t e[4];
      signed_digits(Big(c), 4, e);
      for (int h = 0; h < 4; ++h) Aenc[(size_t)(4 * i + h) * 32 + b] = e[h];
    }

  // ---- decode: source base P, target the 32 bytes of a 256-bit word
  const SourceBase SP = source_base(p, kRnsJ);
  std::vector<int8_t> Adec((size_t)64 * 64, 0);
  for (int j = 0; j < kRnsJ; ++j)
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * j + b;
      const Big D = divmod(SP.Ib[k], M, nullptr);
      int8_t e[32];
      signed_digits(D, 32, e);
      for (int h = 0; h < 32; ++h) Adec[(size_t)h * 64 + k] = e[h];
      int8_t ef[3];
      signed_digits(Big(SP.f[k]), 3, ef);
      for (int t = 0; t < 3; ++t) Adec[(size_t)(32 + t) * 64 + k] = ef[t];
    }
  const Big PmodM = divmod(SP.Q, M, nullptr);
  const Big gdec = cmp(PmodM, Big(0)) == 0 ? Big(0) : sub(M, PmodM);
  for (int w = 0; w < 8; ++w) C.gdec[w] = gdec.word(w);

  // ---- device copy: fragments then seeds of each table
  const size_t enc_b = (kRnsEncFrag + kRnsEncSeed) * 16, mul_b = (kRnsMulFrag + kRnsMulSeed) * 16,
               dec_b = (kRnsDecFrag + kRnsDecSeed) * 16;
  std::vector<uint8_t> h(enc_b + mul_b + dec_b, 0);
  pack_table(Aenc, 3, 1, h.data(), (int32_t*)(h.data() + kRnsEncFrag * 16));
  pack_table(Amul, 2, 3, h.data() + enc_b, (int32_t*)(h.data() + enc_b + kRnsMulFrag * 16));
  pack_table(Adec, 2, 2, h.data() + enc_b + mul_b, (int32_t*)(h.data() + enc_b + mul_b + kRnsDecFrag * 16));
  void* d = nullptr;
  hipError_t err = hipMalloc(&d, h.size());
  if (err != hipSuccess) {
    set_hip_error(ctx, err);
    return FRNTT_ENOMEM;
  }
  err = hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return set_hip_error(ctx, err);
  }
  ctx->rns_mem = d;
  ctx->table_bytes += h.size();
  ctx->rns.enc = (const i32x4*)d;
  ctx->rns.mul = (const i32x4*)((uint8_t*)d + enc_b);
  ctx->rns.dec = (const i32x4*)((uint8_t*)d + enc_b + mul_b);
  ctx->rns.c = C;
  return FRNTT_OK;
}

// ---------------------------------------------------------------- device

namespace {

constexpr int kRnsThreads = 256;

__device__ FRNTT_INLINE i32x16 load_seed(const i32x4* s) {
  const i32x4 a = s[0], b = s[1], c = s[2], d = s[3];
  i32x16 r;
  r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; r[3] = a[3];
  r[4] = b[0]; r[5] = b[1]; r[6] = b[2]; r[7] = b[3];
  r[8] = c[0]; r[9] = c[1]; r[10] = c[2]; r[11] = c[3];
  r[12] = d[0]; r[13] = d[1]; r[14] = d[2]; r[15] = d[3];
  return r;
}

// Residue-wise Montgomery product a b 2^-32 mod q (q < 2^31: t + m q < 2^64).
__device__ FRNTT_INLINE uint32_t redc32(uint32_t a, uint32_t b, uint32_t q, uint32_t qneg) {
  const uint64_t t = (uint64_t)a * b;
  const uint32_t m = (uint32_t)t * qneg;
  const uint32_t u = (uint32_t)((t + (uint64_t)m * q) >> 32);  // < 2q
  return u >= q ? u - q : u;
}

// t mod m for 0 <= t < 2^50 and m < 2^31 (quotient from fp64, corrected once
// either way).
__device__ FRNTT_INLINE uint32_t mod_small(int64_t t, uint32_t m, double minv) {
  const int64_t quo = (int64_t)((double)t * minv);
  int64_t r = t - quo * (int64_t)m;
  r = r < 0 ? r + m : r;
  r = r >= (int64_t)m ? r - m : r;
  return (uint32_t)r;
}

// sum_h acc[4 g + h] 2^(8h): the merged value of one 4-row group
__device__ FRNTT_INLINE int64_t row_group(const i32x16& a, int g) {
  return (int64_t)a[4 * g] + ((int64_t)a[4 * g + 1] << 8) + ((int64_t)a[4 * g + 2] << 16) +
         ((int64_t)a[4 * g + 3] << 24);
}

__device__ FRNTT_INLINE uint32_t sel(int half, uint32_t a0, uint32_t a1) { return half ? a1 : a0; }

// Lane halves hold residues 8m + 2 gi + half (gi < 4) of one element in r[gi].
// Two exchanges with the partner lane give half 0 the residues 8m .. 8m + 3
// and half 1 the residues 8m + 4 .. 8m + 7, each stored as one 16-byte word
// group at dst (= the element's word 8m). All lanes take part in the
// exchanges; `store` masks the write.
__device__ FRNTT_INLINE void store_block(uint32_t* dst, const uint32_t (&r)[4], int half, bool store) {
  const uint32_t x1 = __shfl_xor(half ? r[0] : r[2], 32, 64);  // half 0 gets 8m+1, half 1 gets 8m+4
  const uint32_t x2 = __shfl_xor(half ? r[1] : r[3], 32, 64);  // half 0 gets 8m+3, half 1 gets 8m+6
  if (store) {
    if (half == 0) *(u32x4*)dst = u32x4{r[0], x1, r[1], x2};
    else *(u32x4*)(dst + 4) = u32x4{x1, r[2], x2, r[3]};
  }
}
__device__ FRNTT_INLINE double seld(int half, double a0, double a1) { return half ? a1 : a0; }

}  // namespace

// Canonical values (32 B each) -> base-Q residues x z mod q_i (20 words each).
__global__ __launch_bounds__(kRnsThreads) void rns_encode_kernel(const u32x4* a, uint32_t* xq, int64_t n,
                                                                  RnsTables T) {
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  i32x4 A[3];
  i32x16 S[3];
#pragma unroll
  for (int rb = 0; rb < 3; ++rb) {
    A[rb] = T.enc[rb * 64 + lane];
    S[rb] = load_seed(T.enc + kRnsEncFrag + (rb * 2 + half) * 4);
  }
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    u32x4 raw = {0u, 0u, 0u, 0u};
    if (e < n) raw = a[2 * e + half];
    const i32x4 B = (i32x4)(raw ^ 0x80808080u);
    i32x16 acc[3];
#pragma unroll
    for (int rb = 0; rb < 3; ++rb) acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb], B, S[rb], 0, 0, 0);
    // residues 8 rb + 2 gi + half of this lane's element; the two halves swap
    // two of them per block so that each stores four consecutive words
    uint32_t* out = xq + e * kRnsQWords;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      uint32_t r[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        const int j0 = 8 * rb + 2 * gi;
        r[gi] = mod_small(row_group(acc[rb], gi), sel(half, T.c.q[j0], T.c.q[j0 + 1]),
                          seld(half, T.c.qinv[j0], T.c.qinv[j0 + 1]));
      }
      store_block(out + 8 * rb, r, half, e < n);
    }
    if (e < n && half == 0) {
      const uint32_t r16 = mod_small(row_group(acc[2], 0), T.c.q[16], T.c.qinv[16]);
      *(u32x4*)(out + 16) = u32x4{r16, 0u, 0u, 0u};
    }
  }
}

// Alg. 1 with the residue-wise product in front: base-Q residues of a and b
// -> base-P residues of the lazily reduced product (12 words each).
__global__ __launch_bounds__(kRnsThreads) void rns_mul_kernel(const uint32_t* xa, const uint32_t* xb,
                                                               uint32_t* xp, int64_t n, RnsTables T) {
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  i32x4 A[2][3];
  i32x16 S[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int s = 0; s < 3; ++s) A[rb][s] = T.mul[(rb * 3 + s) * 64 + lane];
    S[rb] = load_seed(T.mul + kRnsMulFrag + (rb * 2 + half) * 4);
  }
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    // x_i = a_i b_i z^-1 mod q_i for this lane's residues: K step s holds
    // residues 8 s + 4 half .. + 3 (residue 16 and the padding in step 2)
    i32x4 B[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      u32x4 x = {0u, 0u, 0u, 0u};
      const bool has = e < n && (s < 2 || half == 0);
      if (has) {
        const int w0 = 8 * s + 4 * half;
        const u32x4 ua = *(const u32x4*)(xa + e * kRnsQWords + w0);
        const u32x4 ub = *(const u32x4*)(xb + e * kRnsQWords + w0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i0 = 8 * s + t;  // residue in the half-0 lanes (i0 + 4 in half 1)
          if (i0 >= kRnsI) continue;
          const uint32_t qi = sel(half, T.c.q[i0], T.c.q[i0 + 4]);
          const uint32_t qn = sel(half, T.c.qneg[i0], T.c.qneg[i0 + 4]);
          x[t] = redc32(ua[t], ub[t], qi, qn);
        }
      }
      B[s] = (i32x4)(x ^ 0x80808080u);
    }
    i32x16 acc[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      acc[rb] = S[rb];
#pragma unroll
      for (int s = 0; s < 3; ++s) acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb][s], B[s], acc[rb], 0, 0, 0);
    }
    // v = sum x_(i,b) f_(i,b): rows 36..38 sit in block 1, registers 0..2 of
    // the half-1 lanes; k = floor(v / 2^u) goes to both halves
    const int64_t v = (int64_t)acc[1][0] + ((int64_t)acc[1][1] << 8) + ((int64_t)acc[1][2] << 16);
    const int32_t k_own = (int32_t)(v >> kRnsU);
    const int32_t k_other = __shfl_xor(k_own, 32, 64);
    const int64_t k = half ? k_own : k_other;
    uint32_t* out = xp + e * kRnsPWords;
    uint32_t r[4];
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
      const int j0 = 2 * gi;
      const uint32_t pj = sel(half, T.c.p[j0], T.c.p[j0 + 1]);
      const uint32_t gj = sel(half, T.c.g[j0], T.c.g[j0 + 1]);
      r[gi] = mod_small(row_group(acc[0], gi) + k * gj, pj, seld(half, T.c.pinv[j0], T.c.pinv[j0 + 1]));
    }
    store_block(out, r, half, e < n);
    if (e < n) {
      if (half == 0) {
        const uint32_t r8 = mod_small(row_group(acc[1], 0) + k * T.c.g[8], T.c.p[8], T.c.pinv[8]);
        *(u32x4*)(out + 8) = u32x4{r8, 0u, 0u, 0u};
      }
    }
  }
}

// Base-P residues (W' z mod p_j) -> canonical W' mod r.
__global__ __launch_bounds__(kRnsThreads) void rns_decode_kernel(const uint32_t* xp, u32x4* out, int64_t n,
                                                                  RnsTables T) {
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  i32x4 A[2][2];
  i32x16 S[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
    for (int s = 0; s < 2; ++s) A[rb][s] = T.dec[(rb * 2 + s) * 64 + lane];
    S[rb] = load_seed(T.dec + kRnsDecFrag + (rb * 2 + half) * 4);
  }
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    u32x4 r0 = {0u, 0u, 0u, 0u}, r1 = {0u, 0u, 0u, 0u};
    if (e < n) {
      r0 = *(const u32x4*)(xp + e * kRnsPWords + 4 * half);
      if (half == 0) r1 = *(const u32x4*)(xp + e * kRnsPWords + 8);
    }
    const i32x4 B0 = (i32x4)(r0 ^ 0x80808080u), B1 = (i32x4)(r1 ^ 0x80808080u);
    i32x16 acc[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb][0], B0, S[rb], 0, 0, 0);
      acc[rb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[rb][1], B1, acc[rb], 0, 0, 0);
    }
    // k = round(v / 2^u) from rows 32..34 (block 1, registers 0..2 of the
    // half-0 lanes): the nearest integer, so that S'' - k P = W' also when
    // W' < 0
    const int64_t v = (int64_t)acc[1][0] + ((int64_t)acc[1][1] << 8) + ((int64_t)acc[1][2] << 16);
    const int32_t k_own = (int32_t)((v + (1 << (kRnsU - 1))) >> kRnsU);
    const int32_t k_other = __shfl_xor(k_own, 32, 64);
    const uint32_t k = (uint32_t)(half ? k_other : k_own);
    // word groups: this lane holds words 2 gi + half, the partner the others
    int64_t G[8];
#pragma unroll
    for (int gi = 0; gi < 4; ++gi) {
      const int64_t mine = row_group(acc[0], gi);
      const uint32_t lo = __shfl_xor((uint32_t)mine, 32, 64);
      const uint32_t hi = __shfl_xor((uint32_t)((uint64_t)mine >> 32), 32, 64);
      const int64_t other = (int64_t)(((uint64_t)hi << 32) | lo);
      G[2 * gi] = half ? other : mine;
      G[2 * gi + 1] = half ? mine : other;
    }
    // V = sum_w G_w 2^(32 w) + k ((-P) mod r) >= 0, below 2^269
    uint32_t y[9];
    int64_t c = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const int64_t s = G[w] + c;
      y[w] = (uint32_t)s;
      c = s >> 32;
    }
    y[8] = (uint32_t)c;
    uint64_t cu = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint64_t s = (uint64_t)T.c.gdec[w] * k + y[w] + cu;
      y[w] = (uint32_t)s;
      cu = s >> 32;
    }
    y[8] += (uint32_t)cu;
    // quotient estimate from the top 45 bits (at most 2 below floor(V / r)),
    // then V - q r < 3r and two conditional subtractions
    const double t = __builtin_fma((double)y[8], 4294967296.0, (double)y[7]);
    int32_t q = (int32_t)(t * (1.0 / 811880051.0)) - 1;
    q = q < 0 ? 0 : q;
    uint32_t carry = 0, br = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint64_t pr = (uint64_t)(uint32_t)q * fr_mod_word(w) + carry;
      carry = (uint32_t)(pr >> 32);
      y[w] = subb(y[w], (uint32_t)pr, br, &br);
    }
    fr_t o;
#pragma unroll
    for (int w = 0; w < 8; ++w) o.w[w] = y[w];
    o = fr_reduce_3r(o);
    if (e < n) {
      if (half == 0) out[2 * e] = u32x4{o.w[0], o.w[1], o.w[2], o.w[3]};
      else out[2 * e + 1] = u32x4{o.w[4], o.w[5], o.w[6], o.w[7]};
    }
  }
}

// The radix Montgomery product on the VALUs (nine 29-bit limbs, R = 2^261):
// the baseline the paper's ablation compares the RNS lazy product with.
__global__ __launch_bounds__(kRnsThreads) void mont_mul_kernel(const u32x4* a, const u32x4* b, u32x4* out,
                                                                int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * kRnsThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRnsThreads)
    st_elem(out, e, mont_mul(ld_elem(a, e), ld_elem(b, e)));
}

}  // namespace frntt

// ---------------------------------------------------------------- C ABI

using namespace frntt;

namespace {

struct RnsDeviceGuard {
  int prev = -1;
  explicit RnsDeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~RnsDeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int grid_for(const frntt_ctx* ctx, int64_t n, int per_block) {
  const int64_t need = (n + per_block - 1) / per_block;
  const int64_t cap = (int64_t)ctx->cu_count * 8;
  return (int)(need < cap ? (need < 1 ? 1 : need) : cap);
}

int launch_status(frntt_ctx* ctx) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? FRNTT_OK : set_hip_error(ctx, e);
}

}  // namespace

extern "C" {

int frntt_rns_moduli(uint32_t* q, uint32_t* p) {
  if (!q || !p) return FRNTT_EINVAL;
  rns_moduli(q, p);
  return FRNTT_OK;
}

int frntt_rns_encode(frntt_ctx* ctx, const void* a, void* xq, int64_t n, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!a || !xq))) return FRNTT_EINVAL;
  if (!aligned16(a) || !aligned16(xq)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(ctx->device);
  rns_encode_kernel<<<grid_for(ctx, n, 128), kRnsThreads, 0, (hipStream_t)stream>>>((const u32x4*)a, (uint32_t*)xq,
                                                                                   n, ctx->rns);
  return launch_status(ctx);
}

int frntt_rns_mul(frntt_ctx* ctx, const void* xa, const void* xb, void* xp, int64_t n, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!xa || !xb || !xp))) return FRNTT_EINVAL;
  if (!aligned16(xa) || !aligned16(xb) || !aligned16(xp)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(ctx->device);
  rns_mul_kernel<<<grid_for(ctx, n, 128), kRnsThreads, 0, (hipStream_t)stream>>>(
      (const uint32_t*)xa, (const uint32_t*)xb, (uint32_t*)xp, n, ctx->rns);
  return launch_status(ctx);
}

int frntt_rns_decode(frntt_ctx* ctx, const void* xp, void* out, int64_t n, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!xp || !out))) return FRNTT_EINVAL;
  if (!aligned16(xp) || !aligned16(out)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(ctx->device);
  rns_decode_kernel<<<grid_for(ctx, n, 128), kRnsThreads, 0, (hipStream_t)stream>>>((const uint32_t*)xp,
                                                                                   (u32x4*)out, n, ctx->rns);
  return launch_status(ctx);
}

int frntt_mont_mul(frntt_ctx* ctx, const void* a, const void* b, void* out, int64_t n, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!a || !b || !out))) return FRNTT_EINVAL;
  if (!aligned16(a) || !aligned16(b) || !aligned16(out)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(ctx->device);
  mont_mul_kernel<<<grid_for(ctx, n, kRnsThreads), kRnsThreads, 0, (hipStream_t)stream>>>(
      (const u32x4*)a, (const u32x4*)b, (u32x4*)out, n);
  return launch_status(ctx);
}

}  // extern "C"
