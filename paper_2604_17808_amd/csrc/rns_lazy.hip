// The MXU-centric RNS lazy modular product (paper: Arithmetic Optimizations,
// "Solution: Reducing O(D^2) Reduction via MXU-Centric RNS Lazy Reduction",
// the walk-through example, and Alg. 1 "MXU RNS Lazy") on gfx950, for the
// three field widths the paper evaluates (BN254's 254-bit r, and 377- and
// 753-bit moduli).
//
// A field element x in [0, M) is carried in an extended non-prime ring Z_Q,
// Q = q_0 ... q_(I-1) > 2 M^2, as its residues x z mod q_i (z = 2^32: the
// residue-wise Montgomery form). A product of two elements is then
//   1. residue-wise: x_i = a_i b_i z^-1 mod q_i (one 32x32-bit Montgomery
//      product per residue, no carries across residues; VALU);
//   2. Alg. 1 Main: one int8 matrix product of the residues' bytes
//      [x]_(i,b) with the constant table E[i,b,j,h] (the bytes of
//      z (I_(i,b) mod M) mod p_j, I_(i,b) the CRT coefficient of residue i
//      times z^-1, shifted by 2^(8b) mod Q), fused with the rows of
//      f_(i,b) = ceil(I_(i,b) 2^u / Q) whose sum v gives the overflow count
//      k = floor(v / 2^u); then per residue j of the base P the byte merge,
//      + k g_j and the reduction to [0, p_j).
// The result is the lazily reduced product W' (W' = a b mod M, |W'| below
// (4 I 255 + 1) M) in base P, residues W' z mod p_j.
//
// Around the product: the encode (canonical value -> base-Q residues) is the
// same byte matrix product with the bytes of z 2^(8b) mod q_i; the decode
// (base P -> canonical) applies Main once more with the base P as the source
// and the bytes of a binary word as the target (the constants are the bytes
// of I^P_(j,b) mod M), rounds k to the nearest integer so that a negative W'
// comes out right, adds k ((-P) mod M), and reduces below M.
//
// MFMA use: v_mfma_i32_32x32x32_i8 with the constant table (staged in LDS)
// as the A operand (rows = output bytes) and 32 elements as the columns of B
// (each lane loads 16 bytes of one element straight from HBM: the B fragment
// layout). Bytes u in [0, 255] enter as u - 128 and the constants as signed
// base-256 digits; the accumulator seeds add back 128 x the digit sums of
// each row.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "fr.hpp"
#include "frntt_internal.hpp"
#include "rns_lazy.hpp"

// One field: its modulus, shape and device tables.
struct frntt_rns_field {
  frntt_ctx* ctx = nullptr;
  int mw = 0;                 // words of the modulus: 8, 12 or 24 (selects the shape)
  void* mem = nullptr;        // encode, Main and decode tables, one allocation
  size_t bytes = 0;
  const frntt::i32x4* enc = nullptr;
  const frntt::i32x4* mul = nullptr;
  const frntt::i32x4* dec = nullptr;
  frntt::RnsConsts c{};
};

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

// The first n consecutive primes below kRnsBound, largest first.
void rns_primes(uint32_t* out, int n) {
  uint32_t x = kRnsBound - 1;
  int got = 0;
  while (got < n) {
    if (is_prime32(x)) out[got++] = x;
    x -= 1;
  }
}

// x mod m for x < 2^s m: conditional subtractions of m 2^t, t = s .. 0
// (quotient bits written to *qt if given)
Big mod_shifted(const Big& x, const Big& m, int s, Big* qt) {
  Big r = x, q;
  q.w.assign(s / 32 + 1, 0);
  for (int t = s; t >= 0; --t) {
    const Big mt = shl(m, t);
    if (cmp(r, mt) >= 0) {
      r = sub(r, mt);
      q.w[t >> 5] |= 1u << (t & 31);
    }
  }
  q.trim();
  if (qt) *qt = q;
  return r;
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

// Precomputation of Alg. 1 for a source base of n moduli: the CRT
// coefficients I_s = (Q/q_s) ((Q/q_s)^-1 z^-1 mod q_s) (so that
// sum_s x_s I_s = X mod Q for Montgomery-form residues x_s = X z mod q_s),
// shifted by 2^(8b) mod Q, and f_(s,b) = ceil(I_(s,b) 2^u / Q).
struct SourceBase {
  Big Q;
  std::vector<Big> Ib;          // [s * 4 + b]
  std::vector<uint32_t> f;      // [s * 4 + b]
};

SourceBase source_base(const uint32_t* m, int n, int u) {
  SourceBase S;
  S.Q = Big(1);
  for (int s = 0; s < n; ++s) S.Q = mul_small(S.Q, m[s]);
  for (int s = 0; s < n; ++s) {
    Big Qs;
    divmod_small(S.Q, m[s], &Qs);
    const uint64_t qs_mod = divmod_small(Qs, m[s], nullptr);
    const uint64_t c = powmod(qs_mod, m[s] - 2, m[s]);                   // (Q/q_s)^-1 mod q_s
    const uint64_t zinv = powmod(powmod(2, 32, m[s]), m[s] - 2, m[s]);  // z^-1 mod q_s
    Big Ib = mul_small(Qs, (uint32_t)(c * zinv % m[s]));                 // < Q
    for (int b = 0; b < 4; ++b) {
      if (b) Ib = mod_shifted(shl(Ib, 8), S.Q, 8, nullptr);
      S.Ib.push_back(Ib);
      // ceil(Ib 2^u / Q) = floor((Ib 2^u + Q - 1) / Q), a quotient below 2^u + 1
      Big fq;
      mod_shifted(sub(add(shl(Ib, u), S.Q), Big(1)), S.Q, u + 1, &fq);
      S.f.push_back(fq.word(0));
    }
  }
  return S;
}

// Residues of the field's two bases and every table of one width.
int build_field(frntt_rns_field* F, const uint32_t* m_words, int mw, int I, int J, int L, int RBE, int KSC,
                int RBM, int KSQ, int RBD, int KSP) {
  RnsConsts& C = F->c;
  C = RnsConsts{};
  C.u_mul = mw == 8 ? 15 : mw == 12 ? 16 : 17;
  C.u_dec = mw == 8 ? 15 : 16;
  std::vector<uint32_t> primes(I + J);
  rns_primes(primes.data(), I + J);
  const uint32_t* q = primes.data();
  const uint32_t* p = primes.data() + I;
  for (int i = 0; i < kRnsMaxI + 7; ++i) {
    C.q[i] = i < I ? q[i] : 1u;
    uint32_t inv = C.q[i];  // -q^-1 mod 2^32 by Newton iteration (q odd)
    for (int it = 0; it < 5; ++it) inv *= 2u - C.q[i] * inv;
    C.qneg[i] = 0u - inv;
    C.qinv[i] = 1.0 / (double)C.q[i];
  }
  for (int j = 0; j < kRnsMaxJ + 7; ++j) {
    C.p[j] = j < J ? p[j] : 1u;
    C.pinv[j] = 1.0 / (double)C.p[j];
  }
  Big M;
  for (int w = 0; w < mw; ++w) M.w.push_back(m_words[w]);
  M.trim();
  for (int w = 0; w < mw; ++w) C.m[w] = m_words[w];
  C.inv_mtop1 = 1.0 / ((double)m_words[mw - 1] + 1.0);
  // Montgomery baseline: 29-bit limbs of M and -M^-1 mod 2^29
  for (int k = 0; k < L; ++k) {
    uint32_t v = 0;
    for (int b = 0; b < 29; ++b) {
      const int bit = 29 * k + b;
      if (bit < 32 * mw && ((m_words[bit >> 5] >> (bit & 31)) & 1)) v |= 1u << b;
    }
    C.m29[k] = v;
  }
  uint32_t inv = m_words[0];
  for (int it = 0; it < 5; ++it) inv *= 2u - m_words[0] * inv;
  C.mneg29 = (0u - inv) & ((1u << 29) - 1);

  // ---- Alg. 1 Main: source base Q, target base P
  const SourceBase SQ = source_base(q, I, C.u_mul);
  Big QmodM;
  QmodM = divmod(SQ.Q, M, nullptr);
  for (int j = 0; j < J; ++j) {
    const uint64_t zj = powmod(2, 32, p[j]);
    const uint64_t qm = divmod_small(QmodM, p[j], nullptr);
    C.g[j] = (uint32_t)((p[j] - zj * qm % p[j]) % p[j]);
  }
  const int KM = 32 * KSQ;
  std::vector<int8_t> Amul((size_t)32 * RBM * KM, 0);
  for (int i = 0; i < I; ++i)
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * i + b;
      const Big IbM = divmod(SQ.Ib[k], M, nullptr);
      for (int j = 0; j < J; ++j) {
        const uint64_t zj = powmod(2, 32, p[j]);
        const uint64_t c = zj * divmod_small(IbM, p[j], nullptr) % p[j];
        int8_t e[4];
        signed_digits(Big(c), 4, e);
        for (int h = 0; h < 4; ++h) Amul[(size_t)(4 * j + h) * KM + k] = e[h];
      }
      int8_t e[3];
      signed_digits(Big(SQ.f[k]), 3, e);
      for (int t = 0; t < 3; ++t) Amul[(size_t)(4 * J + t) * KM + k] = e[t];
    }

  // ---- encode: bytes of a canonical value -> residues z 2^(8b) mod q_i
  const int KE = 32 * KSC;
  std::vector<int8_t> Aenc((size_t)32 * RBE * KE, 0);
  for (int i = 0; i < I; ++i)
    for (int b = 0; b < 4 * mw; ++b) {
      const uint64_t c = powmod(2, 32 + 8 * b, q[i]);
      int8_t e[4];
      signed_digits(Big(c), 4, e);
      for (int h = 0; h < 4; ++h) Aenc[(size_t)(4 * i + h) * KE + b] = e[h];
    }

  // ---- decode: source base P, target the bytes of an mw-word value
  const SourceBase SP = source_base(p, J, C.u_dec);
  const int KD = 32 * KSP;
  std::vector<int8_t> Adec((size_t)32 * RBD * KD, 0);
  for (int j = 0; j < J; ++j)
    for (int b = 0; b < 4; ++b) {
      const int k = 4 * j + b;
      const Big D = divmod(SP.Ib[k], M, nullptr);
      std::vector<int8_t> e(4 * mw);
      signed_digits(D, 4 * mw, e.data());
      for (int h = 0; h < 4 * mw; ++h) Adec[(size_t)h * KD + k] = e[h];
      int8_t ef[3];
      signed_digits(Big(SP.f[k]), 3, ef);
      for (int t = 0; t < 3; ++t) Adec[(size_t)(4 * mw + t) * KD + k] = ef[t];
    }
  const Big PmodM = divmod(SP.Q, M, nullptr);
  const Big gdec = PmodM.w.empty() ? Big(0) : sub(M, PmodM);
  for (int w = 0; w < mw; ++w) C.gdec[w] = gdec.word(w);

  // ---- device copy: fragments then seeds of each table
  const size_t enc_b = ((size_t)RBE * KSC * 64 + RBE * 8) * 16, mul_b = ((size_t)RBM * KSQ * 64 + RBM * 8) * 16,
               dec_b = ((size_t)RBD * KSP * 64 + RBD * 8) * 16;
  std::vector<uint8_t> h(enc_b + mul_b + dec_b, 0);
  pack_table(Aenc, RBE, KSC, h.data(), (int32_t*)(h.data() + (size_t)RBE * KSC * 64 * 16));
  pack_table(Amul, RBM, KSQ, h.data() + enc_b, (int32_t*)(h.data() + enc_b + (size_t)RBM * KSQ * 64 * 16));
  pack_table(Adec, RBD, KSP, h.data() + enc_b + mul_b,
             (int32_t*)(h.data() + enc_b + mul_b + (size_t)RBD * KSP * 64 * 16));
  void* d = nullptr;
  hipError_t err = hipMalloc(&d, h.size());
  if (err != hipSuccess) {
    set_hip_error(F->ctx, err);
    return FRNTT_ENOMEM;
  }
  err = hipMemcpy(d, h.data(), h.size(), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return set_hip_error(F->ctx, err);
  }
  F->mem = d;
  F->bytes = h.size();
  F->enc = (const i32x4*)d;
  F->mul = (const i32x4*)((uint8_t*)d + enc_b);
  F->dec = (const i32x4*)((uint8_t*)d + enc_b + mul_b);
  F->mw = mw;
  return FRNTT_OK;
}

template <class S>
int build_shape(frntt_rns_field* F, const uint32_t* m) {
  return build_field(F, m, S::MW, S::I, S::J, S::L, S::RBE, S::KSC, S::RBM, S::KSQ, S::RBD, S::KSP);
}

// Largest bit length of a modulus each shape is sized for.
int shape_max_bits(int mw) { return mw == 8 ? 254 : mw == 12 ? 377 : mw == 24 ? 753 : 0; }

}  // namespace

int create_rns_field(frntt_ctx* ctx, const uint32_t* m, int mw, frntt_rns_field** out) {
  *out = nullptr;
  frntt_rns_field* F = new (std::nothrow) frntt_rns_field();
  if (!F) return FRNTT_ENOMEM;
  F->ctx = ctx;
  const int rc = mw == 8 ? build_shape<Rns254>(F, m) : mw == 12 ? build_shape<Rns377>(F, m) : build_shape<Rns753>(F, m);
  if (rc != FRNTT_OK) {
    delete F;
    return rc;
  }
  *out = F;
  return FRNTT_OK;
}

int build_rns_tables(frntt_ctx* ctx) {
  uint32_t r[8];
  for (int i = 0; i < 8; ++i) r[i] = fr_mod_word(i);
  frntt_rns_field* F = nullptr;
  const int rc = create_rns_field(ctx, r, 8, &F);
  if (rc != FRNTT_OK) return rc;
  ctx->rns_default = F;
  ctx->table_bytes += F->bytes;
  return FRNTT_OK;
}

void destroy_rns_field(frntt_rns_field* F) {
  if (!F) return;
  if (F->mem) (void)hipFree(F->mem);
  delete F;
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
__device__ FRNTT_INLINE double seld(int half, double a0, double a1) { return half ? a1 : a0; }

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

// Copy `n` 16-byte table entries to LDS (the whole workgroup), then wait.
__device__ FRNTT_INLINE void stage_table(i32x4* lds, const i32x4* tab, int n) {
  for (int i = threadIdx.x; i < n; i += kRnsThreads) lds[i] = tab[i];
  __syncthreads();
}

// Accumulators of row block rb over KS K steps: seeds, then one MFMA per step.
template <int KS>
__device__ FRNTT_INLINE i32x16 block_product(const i32x4* lds, int frag_count, int rb, const i32x4 (&B)[KS],
                                             int lane, int half) {
  i32x16 acc = load_seed(lds + frag_count + (rb * 2 + half) * 4);
#pragma unroll
  for (int s = 0; s < KS; ++s) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(lds[(rb * KS + s) * 64 + lane], B[s], acc, 0, 0, 0);
  return acc;
}

}  // namespace

// Canonical values (S::MW words each) -> base-Q residues x z mod q_i
// (S::QW words each).
template <class S>
__global__ __launch_bounds__(kRnsThreads) void rns_encode_kernel(const uint32_t* a, uint32_t* xq, int64_t n,
                                                                  const i32x4* tab, RnsConsts C) {
  __shared__ i32x4 lds[S::ENC];
  stage_table(lds, tab, S::ENC);
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    i32x4 B[S::KSC];
#pragma unroll
    for (int s = 0; s < S::KSC; ++s) {
      u32x4 raw = {0u, 0u, 0u, 0u};
      const int w0 = 8 * s + 4 * half;
      if (e < n && w0 < S::MW) raw = *(const u32x4*)(a + e * S::MW + w0);
      B[s] = (i32x4)(raw ^ 0x80808080u);
    }
    uint32_t* out = xq + e * S::QW;
#pragma unroll
    for (int rb = 0; rb < S::RBE; ++rb) {
      const i32x16 acc = block_product<S::KSC>(lds, S::ENC_FRAG, rb, B, lane, half);
      uint32_t r[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        const int j0 = 8 * rb + 2 * gi;  // residue of the half-0 lanes (j0 + 1 in half 1)
        const uint32_t qj = sel(half, C.q[j0], C.q[j0 + 1]);
        const uint32_t v = mod_small(row_group(acc, gi), qj, seld(half, C.qinv[j0], C.qinv[j0 + 1]));
        r[gi] = j0 + half < S::I ? v : 0u;
      }
      store_block(out + 8 * rb, r, half, e < n && 8 * rb + 4 * half < S::QW);
    }
  }
}

// Alg. 1 with the residue-wise product in front: base-Q residues of a and b
// -> base-P residues of the lazily reduced product (S::PW words each).
template <class S>
__global__ __launch_bounds__(kRnsThreads) void rns_mul_kernel(const uint32_t* xa, const uint32_t* xb, uint32_t* xp,
                                                               int64_t n, const i32x4* tab, RnsConsts C) {
  __shared__ i32x4 lds[S::MUL];
  stage_table(lds, tab, S::MUL);
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  // rows 4 J .. 4 J + 2 hold the digits of f: block, register group and lane half
  constexpr int kFRow = 4 * S::J, kFB = kFRow / 32, kFG = (kFRow % 32) / 8, kFH = (kFRow / 4) & 1;
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    // x_i = a_i b_i z^-1 mod q_i for this lane's residues: K step s holds
    // residues 8 s + 4 half .. + 3
    i32x4 B[S::KSQ];
#pragma unroll
    for (int s = 0; s < S::KSQ; ++s) {
      u32x4 x = {0u, 0u, 0u, 0u};
      const int w0 = 8 * s + 4 * half;
      if (e < n && w0 < S::QW) {
        const u32x4 ua = *(const u32x4*)(xa + e * S::QW + w0);
        const u32x4 ub = *(const u32x4*)(xb + e * S::QW + w0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i0 = 8 * s + t;  // residue in the half-0 lanes (i0 + 4 in half 1)
          const uint32_t qi = sel(half, C.q[i0], C.q[i0 + 4]);
          const uint32_t qn = sel(half, C.qneg[i0], C.qneg[i0 + 4]);
          const uint32_t v = redc32(ua[t], ub[t], qi, qn);
          x[t] = i0 + 4 * half < S::I ? v : 0u;
        }
      }
      B[s] = (i32x4)(x ^ 0x80808080u);
    }
    // v = sum x_(i,b) f_(i,b) from the f rows; k = floor(v / 2^u) to both halves
    const i32x16 accf = block_product<S::KSQ>(lds, S::MUL_FRAG, kFB, B, lane, half);
    const int64_t v = (int64_t)accf[4 * kFG] + ((int64_t)accf[4 * kFG + 1] << 8) + ((int64_t)accf[4 * kFG + 2] << 16);
    const int32_t k_own = (int32_t)(v >> C.u_mul);
    const int32_t k_other = __shfl_xor(k_own, 32, 64);
    const int64_t k = half == kFH ? k_own : k_other;
    uint32_t* out = xp + e * S::PW;
#pragma unroll
    for (int rb = 0; rb < S::RBM; ++rb) {
      const i32x16 acc = rb == kFB ? accf : block_product<S::KSQ>(lds, S::MUL_FRAG, rb, B, lane, half);
      uint32_t r[4];
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        const int j0 = 8 * rb + 2 * gi;
        const uint32_t pj = sel(half, C.p[j0], C.p[j0 + 1]);
        const uint32_t gj = sel(half, C.g[j0], C.g[j0 + 1]);
        const uint32_t rv = mod_small(row_group(acc, gi) + k * gj, pj, seld(half, C.pinv[j0], C.pinv[j0 + 1]));
        r[gi] = j0 + half < S::J ? rv : 0u;
      }
      store_block(out + 8 * rb, r, half, e < n && 8 * rb + 4 * half < S::PW);
    }
  }
}

// Base-P residues (W' z mod p_j) -> canonical W' mod M (S::MW words).
template <class S>
__global__ __launch_bounds__(kRnsThreads) void rns_decode_kernel(const uint32_t* xp, uint32_t* out, int64_t n,
                                                                  const i32x4* tab, RnsConsts C) {
  __shared__ i32x4 lds[S::DEC];
  stage_table(lds, tab, S::DEC);
  const int lane = threadIdx.x & 63, half = lane >> 5, col = lane & 31;
  constexpr int MW = S::MW;
  constexpr int kFRow = 4 * MW, kFB = kFRow / 32, kFG = (kFRow % 32) / 8, kFH = (kFRow / 4) & 1;
  constexpr int kWB = (MW + 7) / 8;  // row blocks holding output words
  const int64_t groups = (n + 31) >> 5;
  const int waves = kRnsThreads / 64;
  for (int64_t g = (int64_t)blockIdx.x * waves + (threadIdx.x >> 6); g < groups; g += (int64_t)gridDim.x * waves) {
    const int64_t e = g * 32 + col;
    i32x4 B[S::KSP];
#pragma unroll
    for (int s = 0; s < S::KSP; ++s) {
      u32x4 raw = {0u, 0u, 0u, 0u};
      const int w0 = 8 * s + 4 * half;
      if (e < n && w0 < S::PW) raw = *(const u32x4*)(xp + e * S::PW + w0);
      B[s] = (i32x4)(raw ^ 0x80808080u);
    }
    // k = round(v / 2^u) from the f rows: the nearest integer, so that
    // S'' - k P = W' also when W' < 0
    const i32x16 accf = block_product<S::KSP>(lds, S::DEC_FRAG, kFB, B, lane, half);
    const int64_t v = (int64_t)accf[4 * kFG] + ((int64_t)accf[4 * kFG + 1] << 8) + ((int64_t)accf[4 * kFG + 2] << 16);
    const int32_t k_own = (int32_t)((v + (1ll << (C.u_dec - 1))) >> C.u_dec);
    const int32_t k_other = __shfl_xor(k_own, 32, 64);
    const uint32_t k = (uint32_t)(half == kFH ? k_own : k_other);
    // word groups: this lane holds words 8 rb + 2 gi + half, the partner the others
    int64_t G[8 * kWB];
#pragma unroll
    for (int rb = 0; rb < kWB; ++rb) {
      const i32x16 acc = rb == kFB ? accf : block_product<S::KSP>(lds, S::DEC_FRAG, rb, B, lane, half);
#pragma unroll
      for (int gi = 0; gi < 4; ++gi) {
        const int64_t mine = row_group(acc, gi);
        const uint32_t lo = __shfl_xor((uint32_t)mine, 32, 64);
        const uint32_t hi = __shfl_xor((uint32_t)((uint64_t)mine >> 32), 32, 64);
        const int64_t other = (int64_t)(((uint64_t)hi << 32) | lo);
        G[8 * rb + 2 * gi] = half ? other : mine;
        G[8 * rb + 2 * gi + 1] = half ? mine : other;
      }
    }
    // V = sum_w G_w 2^(32 w) + k ((-P) mod M) >= 0
    uint32_t y[MW + 1];
    int64_t c = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      const int64_t s = G[w] + c;
      y[w] = (uint32_t)s;
      c = s >> 32;
    }
    y[MW] = (uint32_t)c;
    uint64_t cu = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      const uint64_t s = (uint64_t)C.gdec[w] * k + y[w] + cu;
      y[w] = (uint32_t)s;
      cu = s >> 32;
    }
    y[MW] += (uint32_t)cu;
    // quotient estimate from the top two words (at most 2 below floor(V / M)),
    // then V - q M < 3M and two conditional subtractions of M
    const double t = __builtin_fma((double)y[MW], 4294967296.0, (double)y[MW - 1]);
    int32_t q = (int32_t)(t * C.inv_mtop1) - 1;
    q = q < 0 ? 0 : q;
    uint32_t carry = 0, br = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) {
      const uint64_t pr = (uint64_t)(uint32_t)q * C.m[w] + carry;
      carry = (uint32_t)(pr >> 32);
      y[w] = subb(y[w], (uint32_t)pr, br, &br);
    }
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      uint32_t d[MW], b2 = 0;
#pragma unroll
      for (int w = 0; w < MW; ++w) d[w] = subb(y[w], C.m[w], b2, &b2);
#pragma unroll
      for (int w = 0; w < MW; ++w) y[w] = b2 ? y[w] : d[w];
    }
    // 16-byte word groups: group m (words 4m .. 4m + 3) from lane half m % 2
#pragma unroll
    for (int m = 0; m < MW / 4; ++m)
      if (e < n && (m & 1) == half) *(u32x4*)(out + e * MW + 4 * m) = u32x4{y[4 * m], y[4 * m + 1], y[4 * m + 2], y[4 * m + 3]};
  }
}

// The radix Montgomery product on the vector ALUs with L 29-bit limbs
// (R = 2^(29 L)): out = a b R^-1 mod M for canonical a, b (MW words each).
// Row i adds a b_i and m M (m clears the low limb), then drops one limb; the
// columns stay below 2^64 for L <= 26 (at most 2 L products below 2^58 each).
template <class S>
__global__ __launch_bounds__(kRnsThreads) void mont_mul_kernel(const uint32_t* a, const uint32_t* b, uint32_t* out,
                                                                int64_t n, RnsConsts C) {
  constexpr int L = S::L, MW = S::MW;
  constexpr uint32_t mask = (1u << 29) - 1;
  for (int64_t e = (int64_t)blockIdx.x * kRnsThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kRnsThreads) {
    uint32_t aw[MW], bw[MW], al[L], bl[L];
#pragma unroll
    for (int m = 0; m < MW / 4; ++m) {
      const u32x4 x = *(const u32x4*)(a + e * MW + 4 * m), y = *(const u32x4*)(b + e * MW + 4 * m);
      aw[4 * m] = x.x; aw[4 * m + 1] = x.y; aw[4 * m + 2] = x.z; aw[4 * m + 3] = x.w;
      bw[4 * m] = y.x; bw[4 * m + 1] = y.y; bw[4 * m + 2] = y.z; bw[4 * m + 3] = y.w;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
      const int bit = 29 * k, wi = bit >> 5, sh = bit & 31;
      uint32_t va, vb;
      if (sh + 29 <= 32 || wi + 1 >= MW) {
        va = aw[wi] >> sh;
        vb = bw[wi] >> sh;
      } else {
        va = __builtin_amdgcn_alignbit(aw[wi + 1], aw[wi], (uint32_t)sh);
        vb = __builtin_amdgcn_alignbit(bw[wi + 1], bw[wi], (uint32_t)sh);
      }
      al[k] = va & mask;
      bl[k] = vb & mask;
    }
    uint64_t t[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
#pragma unroll
      for (int j = 0; j < L; ++j) t[j] = (i == 0 ? 0ull : t[j]) + (uint64_t)al[j] * bl[i];
      const uint32_t m = ((uint32_t)t[0] * C.mneg29) & mask;
#pragma unroll
      for (int j = 0; j < L; ++j) t[j] += (uint64_t)m * C.m29[j];
      const uint64_t cy = t[0] >> 29;
#pragma unroll
      for (int j = 0; j < L - 1; ++j) t[j] = t[j + 1];
      t[L - 1] = 0;
      t[0] += cy;
    }
    // carry into 29-bit limbs plus the carry out (the value is below 2M,
    // which can exceed 2^(29 L) by one bit, as for 377-bit M with L = 13),
    // pack to words, subtract M once
    uint32_t l[L + 1];
    uint64_t cy = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const uint64_t v = t[j] + cy;
      l[j] = (uint32_t)v & mask;
      cy = v >> 29;
    }
    l[L] = (uint32_t)cy;
    uint32_t y[MW];
#pragma unroll
    for (int i = 0; i < MW; ++i) {
      const int bit = 32 * i, k = bit / 29, sh = bit % 29;
      uint32_t v = k <= L ? l[k] >> sh : 0u;
      const int have = 29 - sh;
      if (k + 1 <= L) v |= l[k + 1] << have;
      if (have + 29 < 32 && k + 2 <= L) v |= l[k + 2] << (have + 29);
      y[i] = v;
    }
    uint32_t d[MW], b2 = 0;
#pragma unroll
    for (int w = 0; w < MW; ++w) d[w] = subb(y[w], C.m[w], b2, &b2);
#pragma unroll
    for (int m = 0; m < MW / 4; ++m) {
      u32x4 o;
      o.x = b2 ? y[4 * m] : d[4 * m];
      o.y = b2 ? y[4 * m + 1] : d[4 * m + 1];
      o.z = b2 ? y[4 * m + 2] : d[4 * m + 2];
      o.w = b2 ? y[4 * m + 3] : d[4 * m + 3];
      *(u32x4*)(out + e * MW + 4 * m) = o;
    }
  }
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

template <class S>
void launch_encode(const frntt_rns_field* F, const void* a, void* xq, int64_t n, hipStream_t st) {
  rns_encode_kernel<S><<<grid_for(F->ctx, n, 128), kRnsThreads, 0, st>>>((const uint32_t*)a, (uint32_t*)xq, n,
                                                                        F->enc, F->c);
}
template <class S>
void launch_mul(const frntt_rns_field* F, const void* xa, const void* xb, void* xp, int64_t n, hipStream_t st) {
  rns_mul_kernel<S><<<grid_for(F->ctx, n, 128), kRnsThreads, 0, st>>>((const uint32_t*)xa, (const uint32_t*)xb,
                                                                     (uint32_t*)xp, n, F->mul, F->c);
}
template <class S>
void launch_decode(const frntt_rns_field* F, const void* xp, void* out, int64_t n, hipStream_t st) {
  rns_decode_kernel<S><<<grid_for(F->ctx, n, 128), kRnsThreads, 0, st>>>((const uint32_t*)xp, (uint32_t*)out, n,
                                                                        F->dec, F->c);
}
template <class S>
void launch_mont(const frntt_rns_field* F, const void* a, const void* b, void* out, int64_t n, hipStream_t st) {
  mont_mul_kernel<S><<<grid_for(F->ctx, n, kRnsThreads), kRnsThreads, 0, st>>>(
      (const uint32_t*)a, (const uint32_t*)b, (uint32_t*)out, n, F->c);
}

// Dispatch on the field's shape: OP<S>(args...)
#define FRNTT_RNS_DISPATCH(F, OP, ...)              \
  do {                                              \
    if ((F)->mw == 8) OP<Rns254>(F, __VA_ARGS__);   \
    else if ((F)->mw == 12) OP<Rns377>(F, __VA_ARGS__); \
    else OP<Rns753>(F, __VA_ARGS__);                \
  } while (0)

int field_encode(frntt_rns_field* F, const void* a, void* xq, int64_t n, void* stream) {
  if (!F || n < 0 || (n > 0 && (!a || !xq))) return FRNTT_EINVAL;
  if (!aligned16(a) || !aligned16(xq)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(F->ctx->device);
  FRNTT_RNS_DISPATCH(F, launch_encode, a, xq, n, (hipStream_t)stream);
  return launch_status(F->ctx);
}

int field_mul(frntt_rns_field* F, const void* xa, const void* xb, void* xp, int64_t n, void* stream) {
  if (!F || n < 0 || (n > 0 && (!xa || !xb || !xp))) return FRNTT_EINVAL;
  if (!aligned16(xa) || !aligned16(xb) || !aligned16(xp)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(F->ctx->device);
  FRNTT_RNS_DISPATCH(F, launch_mul, xa, xb, xp, n, (hipStream_t)stream);
  return launch_status(F->ctx);
}

int field_decode(frntt_rns_field* F, const void* xp, void* out, int64_t n, void* stream) {
  if (!F || n < 0 || (n > 0 && (!xp || !out))) return FRNTT_EINVAL;
  if (!aligned16(xp) || !aligned16(out)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(F->ctx->device);
  FRNTT_RNS_DISPATCH(F, launch_decode, xp, out, n, (hipStream_t)stream);
  return launch_status(F->ctx);
}

int field_mont(frntt_rns_field* F, const void* a, const void* b, void* out, int64_t n, void* stream) {
  if (!F || n < 0 || (n > 0 && (!a || !b || !out))) return FRNTT_EINVAL;
  if (!aligned16(a) || !aligned16(b) || !aligned16(out)) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  RnsDeviceGuard guard(F->ctx->device);
  FRNTT_RNS_DISPATCH(F, launch_mont, a, b, out, n, (hipStream_t)stream);
  return launch_status(F->ctx);
}

}  // namespace

extern "C" {

int frntt_rns_moduli(uint32_t* q, uint32_t* p) {
  if (!q || !p) return FRNTT_EINVAL;
  uint32_t all[Rns254::I + Rns254::J];
  rns_primes(all, Rns254::I + Rns254::J);
  std::memcpy(q, all, sizeof(uint32_t) * Rns254::I);
  std::memcpy(p, all + Rns254::I, sizeof(uint32_t) * Rns254::J);
  return FRNTT_OK;
}

int frntt_rns_encode(frntt_ctx* ctx, const void* a, void* xq, int64_t n, void* stream) {
  return ctx ? field_encode(ctx->rns_default, a, xq, n, stream) : FRNTT_EINVAL;
}
int frntt_rns_mul(frntt_ctx* ctx, const void* xa, const void* xb, void* xp, int64_t n, void* stream) {
  return ctx ? field_mul(ctx->rns_default, xa, xb, xp, n, stream) : FRNTT_EINVAL;
}
int frntt_rns_decode(frntt_ctx* ctx, const void* xp, void* out, int64_t n, void* stream) {
  return ctx ? field_decode(ctx->rns_default, xp, out, n, stream) : FRNTT_EINVAL;
}
int frntt_mont_mul(frntt_ctx* ctx, const void* a, const void* b, void* out, int64_t n, void* stream) {
  return ctx ? field_mont(ctx->rns_default, a, b, out, n, stream) : FRNTT_EINVAL;
}

int frntt_rns_field_create(frntt_rns_field** out, frntt_ctx* ctx, const uint32_t* m, int m_words) {
  if (!out) return FRNTT_EINVAL;
  *out = nullptr;
  if (!ctx || !m || (m_words != 8 && m_words != 12 && m_words != 24)) return FRNTT_EINVAL;
  // odd, above 2^31 (coprime to every RNS modulus) and within the shape's width
  int bits = 0;
  for (int w = m_words - 1; w >= 0 && !bits; --w)
    if (m[w]) bits = 32 * w + 32 - __builtin_clz(m[w]);
  if ((m[0] & 1) == 0 || bits <= 32 || bits > shape_max_bits(m_words)) return FRNTT_ERANGE;
  RnsDeviceGuard guard(ctx->device);
  return create_rns_field(ctx, m, m_words, out);
}

int frntt_rns_field_destroy(frntt_rns_field* f) {
  if (!f) return FRNTT_OK;
  {
    RnsDeviceGuard guard(f->ctx->device);
    (void)hipDeviceSynchronize();
  }
  destroy_rns_field(f);
  return FRNTT_OK;
}

int frntt_rns_field_shape(const frntt_rns_field* f, int* n_q, int* n_p, int* q_words, int* p_words) {
  if (!f || !n_q || !n_p || !q_words || !p_words) return FRNTT_EINVAL;
  if (f->mw == 8) *n_q = Rns254::I, *n_p = Rns254::J, *q_words = Rns254::QW, *p_words = Rns254::PW;
  else if (f->mw == 12) *n_q = Rns377::I, *n_p = Rns377::J, *q_words = Rns377::QW, *p_words = Rns377::PW;
  else *n_q = Rns753::I, *n_p = Rns753::J, *q_words = Rns753::QW, *p_words = Rns753::PW;
  return FRNTT_OK;
}

int frntt_rns_field_encode(frntt_rns_field* f, const void* a, void* xq, int64_t n, void* stream) {
  return field_encode(f, a, xq, n, stream);
}
int frntt_rns_field_mul(frntt_rns_field* f, const void* xa, const void* xb, void* xp, int64_t n, void* stream) {
  return field_mul(f, xa, xb, xp, n, stream);
}
int frntt_rns_field_decode(frntt_rns_field* f, const void* xp, void* out, int64_t n, void* stream) {
  return field_decode(f, xp, out, n, stream);
}
int frntt_rns_field_mont_mul(frntt_rns_field* f, const void* a, const void* b, void* out, int64_t n, void* stream) {
  return field_mont(f, a, b, out, n, stream);
}

}  // extern "C"
