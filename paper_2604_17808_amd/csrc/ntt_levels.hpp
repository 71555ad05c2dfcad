// Transform kernels for gfx950: shared pass machinery.
//
// One launch = one HBM pass of the multi-pass decomposition N = R_1 ... R_P
// (the paper's 3-step NTT for P = 2 and its recursive 5-step refinement,
// Eq. 1, for P = 3). A workgroup stages G lines of R = 2^l <= 4096 elements
// in LDS, computes the length-R sub-DFT of every line, then applies the
// pass's twiddle (or the inverse/coset epilogue in the last pass) on the way
// back to HBM.
//
// The sub-DFT of a line runs on one of two engines:
//   * butterfly: radix-2 decimation-in-frequency stages in LDS with
//     Montgomery twiddle products on the VALUs (the paper's butterfly NTT);
//   * MFMA: nested levels of radix rho <= 16. Level l reads LDS row n_l (its
//     input digit) across V = T / rho vectors; the rho-point DFT of 32
//     vectors at a time is a GEMM of the BAT byte-limb constant blocks
//     E[(k,h),(n,a)] (signed digit h of w^(kn) * 2^(8a) mod r) with the data
//     bytes on int8 MFMA (Alg. 1's ByteDecompose and einsum), followed by the
//     carry merge sum_h P_h 2^(8h) and reduction mod r (ByteMerge and the
//     final correction), the inter-level twiddle, and a write into the row
//     order the next level reads. The vector index is always the fastest
//     LDS index.
// Both engines compute exact field values, so results are bit-identical.
#pragma once
#include "ntt_device.hpp"

namespace frntt {

constexpr int kBatMaxRho = 16;  // largest MFMA level radix; blocks staged in LDS (16 KiB)

// ---------------------------------------------------------------- LDS

__device__ FRNTT_INLINE fr_t lds_ld(const u32x4* lds, int e) {
  u32x4 a = lds[2 * e], b = lds[2 * e + 1];
  fr_t x;
  x.w[0] = a.x; x.w[1] = a.y; x.w[2] = a.z; x.w[3] = a.w;
  x.w[4] = b.x; x.w[5] = b.y; x.w[6] = b.z; x.w[7] = b.w;
  return x;
}

__device__ FRNTT_INLINE void lds_st(u32x4* lds, int e, const fr_t& x) {
  u32x4 a = {x.w[0], x.w[1], x.w[2], x.w[3]};
  u32x4 b = {x.w[4], x.w[5], x.w[6], x.w[7]};
  lds[2 * e] = a;
  lds[2 * e + 1] = b;
}

// ------------------------------------------------------ load / store phases

// Stage the workgroup's G lines in LDS at position n * G + line (with the
// coset pre-scale x_n * g^n in the first pass of a coset transform).
__device__ FRNTT_INLINE void load_lines(u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  const int T_el = 1 << P.log_t;
  const int G = 1 << P.log_g;
  const int tid = threadIdx.x;
  const int64_t nmask = (1ll << P.log_n) - 1;
  if (!P.is_last) {
    // pass axis strided: neighbouring threads take neighbouring lines
    for (int e = tid; e < T_el; e += kThreads) {
      const int n = e >> P.log_g, line = e & (G - 1);
      const LineMap mp = map_line(P, wg * G + line);
      const int64_t idx = mp.in_base + ((int64_t)n << mp.in_shift);
      fr_t x = ld_elem(P.src, idx);
      if (P.coset_pre) x = mont_mul(x, coset_pow(T, 0, (uint32_t)(idx & nmask)));
      lds_st(lds, e, x);
    }
  } else {
    // lines contiguous in memory: neighbouring threads take neighbouring n
    const int R = 1 << P.log_r;
    for (int e = tid; e < T_el; e += kThreads) {
      const int line = e >> P.log_r, n = e & (R - 1);
      const LineMap mp = map_line(P, wg * G + line);
      const int64_t idx = mp.in_base + n;
      fr_t x = ld_elem(P.src, idx);
      if (P.coset_pre) x = mont_mul(x, coset_pow(T, 0, (uint32_t)(idx & nmask)));
      lds_st(lds, n * G + line, x);
    }
  }
}

// Write output k of every line (found at LDS row k, or bitrev(k) after the
// butterfly engine) to HBM, with the pass twiddle w^(rest * k) of the
// size-2^(l+S) sub-problem, or the last pass's N^-1 / g^-k epilogue.
__device__ FRNTT_INLINE void store_lines(const u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg,
                                         bool bitrev) {
  const int T_el = 1 << P.log_t;
  const int G = 1 << P.log_g;
  const int tid = threadIdx.x;
  // two elements in flight per thread: their table loads overlap
#pragma unroll 2
  for (int e = tid; e < T_el; e += kThreads) {
    const int k = e >> P.log_g, line = e & (G - 1);
    const int row = bitrev ? (int)(__builtin_bitreverse32((uint32_t)k) >> (32 - P.log_r)) : k;
    fr_t y = lds_ld(lds, row * G + line);
    const LineMap mp = map_line(P, wg * G + line);
    if (!P.is_last) {
      // y may be below 2^256 but not reduced (MFMA engine): word-scanned operand
      y = mont_mul(pow_tw(T, P.dir, P.log_r + P.log_s, (uint64_t)mp.rest * (uint64_t)k), y);
    } else if (P.post == 1) {
      y = mont_mul(y, ld_elem(T.ninv, P.log_n));
    } else if (P.post == 2) {
      const uint32_t idx = (uint32_t)(mp.poly_off + ((int64_t)k << mp.out_shift));
      y = mont_mul(y, mont_mul(ld_elem(T.ninv, P.log_n), coset_pow(T, 1, idx)));
    }
    st_elem(P.dst, mp.out_base + ((int64_t)k << mp.out_shift), y);
  }
}

// ------------------------------------------------------- butterfly engine

// log_r radix-2 DIF stages over every line, in place in LDS; afterwards row i
// of a line holds output bitrev(i).
__device__ FRNTT_INLINE void bfly_stages(u32x4* lds, const PassParams& P, const DevTables& T) {
  const int half_el = 1 << (P.log_t - 1);
  const int G = 1 << P.log_g;
  const int tid = threadIdx.x;
  const u32x4* w = T.w4096[P.dir];
  for (int s = 0; s < P.log_r; ++s) {
    const int log_span = P.log_r - 1 - s;
    const int span = 1 << log_span;
#pragma unroll 1
    for (int b = tid; b < half_el; b += kThreads) {
      const int line = b & (G - 1);
      const int bb = b >> P.log_g;             // butterfly index inside the line
      const int j = bb & (span - 1);
      const int i0 = ((bb >> log_span) << (log_span + 1)) + j;
      const int e0 = i0 * G + line, e1 = (i0 + span) * G + line;
      const fr_t u = lds_ld(lds, e0), v = lds_ld(lds, e1);
      lds_st(lds, e0, fr_add(u, v));
      // w_{2 span}^j = w_4096^(j * 2^s * 2^(12 - log_r))
      const fr_t tw = ld_elem(w, (j << s) << (12 - P.log_r));
      lds_st(lds, e1, mont_mul(fr_sub(u, v), tw));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ MFMA level

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

// y (9 words, y < 3r after the quotient step) -> canonical
__device__ FRNTT_INLINE void cond_sub_words(uint32_t* y, bool twice) {
  uint32_t d[8], b = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) d[i] = subb(y[i], twice ? two_r_word(i) : fr_mod_word(i), b, &b);
#pragma unroll
  for (int i = 0; i < 8; ++i) y[i] = b ? y[i] : d[i];
}

// Top 32-bit word of r plus one, inverted: floor(top / (r_top + 1)) never
// exceeds the true quotient.
#define FR_INV_RTOP1 (1.0 / 811880051.0)  // r_top = 0x30644e72 = 811880050

// Merge the byte-plane partials of two outputs (acc0 -> output k0 in lanes
// 0..31, acc1 -> k1 in lanes 32..63) and reduce mod r. Lane l holds rows
// h = 8i + 4*(l/32) + j in register 4i + j (the 32x32 MFMA accumulator
// layout), i.e. the partials of 32-bit words 2i + l/32. After the swap of
// the two half-waves each lane holds all 32 partials of its own output,
// y = sum_h P_h 2^(8h) (a multiple of r keeps it positive, below 2^276).
//
// The merge runs on exact fp64 integers: a word group sum_j P_(4w+j) 2^(8j)
// stays below 2^53, and splitting t into floor(t / 2^32) and the remainder
// is exact. A quotient estimate from the top 52 bits, at most 2 below
// floor(y / r), then brings y into [0, 3r); `canonical` finishes in [0, r).
__device__ FRNTT_INLINE fr_t merge_reduce(const i32x16& a0, const i32x16& a1, bool canonical) {
  double w0[4], w1[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w0[i] = __builtin_fma((double)a0[4 * i + 3], 16777216.0,
             __builtin_fma((double)a0[4 * i + 2], 65536.0,
              __builtin_fma((double)a0[4 * i + 1], 256.0, (double)a0[4 * i])));
    w1[i] = __builtin_fma((double)a1[4 * i + 3], 16777216.0,
             __builtin_fma((double)a1[4 * i + 2], 65536.0,
              __builtin_fma((double)a1[4 * i + 1], 256.0, (double)a1[4 * i])));
  }
  double X[4], Y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t b0 = __builtin_bit_cast(uint64_t, w0[i]);
    const uint64_t b1 = __builtin_bit_cast(uint64_t, w1[i]);
    auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b0, (uint32_t)b1, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b0 >> 32), (uint32_t)(b1 >> 32), false, false);
    X[i] = __builtin_bit_cast(double, ((uint64_t)hi[0] << 32) | (uint32_t)lo[0]);  // word 2i
    Y[i] = __builtin_bit_cast(double, ((uint64_t)hi[1] << 32) | (uint32_t)lo[1]);  // word 2i + 1
  }
  uint32_t y[9];
  double t = 0.0, h = 0.0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    t = ((w & 1) ? Y[w >> 1] : X[w >> 1]) + h;
    h = __builtin_floor(t * 2.3283064365386963e-10);  // exact floor(t / 2^32)
    y[w] = (uint32_t)__builtin_fma(h, -4294967296.0, t);
  }
  y[8] = (uint32_t)h;
  // quotient estimate from t = y[8] * 2^32 + y[7] (exact in fp64)
  int32_t q = (int32_t)(t * FR_INV_RTOP1) - 1;
  q = q < 0 ? 0 : q;
  uint32_t carry = 0, br = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint64_t p = (uint64_t)(uint32_t)q * fr_mod_word(i) + carry;
    carry = (uint32_t)(p >> 32);
    y[i] = subb(y[i], (uint32_t)p, br, &br);
  }
  if (canonical) {
    cond_sub_words(y, true);
    cond_sub_words(y, false);
  }
  fr_t o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = y[i];
  return o;
}

__device__ FRNTT_INLINE i32x16 load_init(const i32x4* init, int k, int half) {
  const i32x4* p = init + (k * 2 + half) * 4;
  i32x4 a = p[0], b = p[1], c = p[2], d = p[3];
  i32x16 r;
  r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; r[3] = a[3];
  r[4] = b[0]; r[5] = b[1]; r[6] = b[2]; r[7] = b[3];
  r[8] = c[0]; r[9] = c[1]; r[10] = c[2]; r[11] = c[3];
  r[12] = d[0]; r[13] = d[1]; r[14] = d[2]; r[15] = d[3];
  return r;
}

struct LevelGeom {
  int m;          // log2 radix of this level
  int pprev_log;  // log2 product of earlier radices
  int q_log;      // log2 product of later radices
  int next_m;     // log2 radix of the next level
  int last;
};

// Route output digit k of vector v into the next level's row order (after
// the inter-level twiddle tw = w^(nn * k) of the size-2^(m + q_log)
// sub-problem), or, after the last level, to row k of its line.
__device__ FRNTT_INLINE void level_output(u32x4* lds, const PassParams& P, const LevelGeom& g, int v, int k,
                                          fr_t y, const fr_t& tw) {
  const int line = v & ((1 << P.log_g) - 1);
  const int rem = v >> P.log_g;
  const int kk = rem & ((1 << g.pprev_log) - 1);
  const int nn = rem >> g.pprev_log;
  if (!g.last) {
    // y may be any value below 2^256 here: it is the word-scanned operand
    y = mont_mul(tw, y);
    const int nshift = g.q_log - g.next_m;
    const int n_next = nn >> nshift;
    const int nn2 = nn & ((1 << nshift) - 1);
    const int col = line + ((kk + (k << g.pprev_log) + (nn2 << (g.pprev_log + g.m))) << P.log_g);
    lds_st(lds, (n_next << (P.log_t - g.next_m)) + col, y);
  } else {
    lds_st(lds, ((kk + (k << g.pprev_log)) << P.log_g) + line, y);
  }
}

// One MFMA level. Tiles of 32 vectors are spread over the 8 waves: each wave
// takes TPW tiles, or, when there are fewer tiles than waves, KSPLIT waves
// share a tile and each computes RHO / KSPLIT of its outputs. A wave first
// loads the data fragments of its tiles (lane l: bytes 16*(l/32)..+15 of
// vector l%32 for every input digit n), so that after the barrier the level
// can overwrite LDS in place.
template <int M, int TPW, int KSPLIT>
__device__ FRNTT_INLINE void mfma_level(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                        const LevelGeom& g) {
  constexpr int RHO = 1 << M;
  constexpr int KCNT = RHO / KSPLIT;
  const int V = 1 << (P.log_t - M);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int tile0 = (wave / KSPLIT) * TPW;
  const int kbase = (wave % KSPLIT) * KCNT;
  // stage this radix's constant blocks (RHO KiB) and accumulator seeds
  // (RHO x 2 x 16 int32) in LDS
  const i32x4* bat = T.bat[P.dir][M];
  for (int i = threadIdx.x; i < RHO * 64; i += kThreads) lds_f[i] = bat[i];
  const i32x4* init_g = T.bat_init[P.dir][M];
  i32x4* init = lds_f + kBatMaxRho * 64;
  for (int i = threadIdx.x; i < RHO * 8; i += kThreads) init[i] = init_g[i];
  i32x4 B[TPW][RHO];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int v = (tile0 + t) * 32 + col;
#pragma unroll
    for (int n = 0; n < RHO; ++n) {
      const u32x4 raw = lds[2 * (n * V + v) + half];
      B[t][n] = (i32x4)(raw ^ 0x80808080u);  // unsigned byte u -> signed u - 128
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int v = (tile0 + t) * 32 + col;
#pragma unroll 1
    for (int k0 = kbase; k0 < kbase + KCNT; k0 += 2) {
      const int k = k0 + half;  // this lane's output after the merge
      // issue the inter-level twiddle load before the MFMA chain so its
      // latency hides behind it
      fr_t tw;
      if (!g.last) {
        const int nn = (v >> P.log_g) >> g.pprev_log;
        tw = small_tw(T, P.dir, g.m + g.q_log, (uint32_t)(nn * k));
      }
      i32x16 acc0 = load_init(init, k0, half);
      i32x16 acc1 = load_init(init, k0 + 1, half);
#pragma unroll
      for (int n = 0; n < RHO; ++n) {
        const i32x4 a0 = lds_f[((k0 * n) & (RHO - 1)) * 64 + lane];
        const i32x4 a1 = lds_f[(((k0 + 1) * n) & (RHO - 1)) * 64 + lane];
        acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, B[t][n], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, B[t][n], acc1, 0, 0, 0);
      }
      // outputs that get a twiddle product next may stay in [0, 3r)
      const bool canonical = g.last && P.is_last;
      const fr_t y = merge_reduce(acc0, acc1, canonical);
      level_output(lds, P, g, v, k, y, tw);
    }
  }
  __syncthreads();
}

__device__ FRNTT_INLINE void run_mfma_level(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                            const LevelGeom& g) {
  const int tiles = 1 << (P.log_t - g.m - 5);
  const int tpw = tiles >= kWaves ? tiles / kWaves : 1;
  const int ksplit = tiles >= kWaves ? 1 : kWaves / tiles;
  switch (g.m * 256 + tpw * 16 + ksplit) {
    case 1 * 256 + 8 * 16 + 1: mfma_level<1, 8, 1>(lds, lds_f, P, T, g); break;
    case 1 * 256 + 4 * 16 + 1: mfma_level<1, 4, 1>(lds, lds_f, P, T, g); break;
    case 2 * 256 + 4 * 16 + 1: mfma_level<2, 4, 1>(lds, lds_f, P, T, g); break;
    case 2 * 256 + 2 * 16 + 1: mfma_level<2, 2, 1>(lds, lds_f, P, T, g); break;
    case 3 * 256 + 2 * 16 + 1: mfma_level<3, 2, 1>(lds, lds_f, P, T, g); break;
    case 3 * 256 + 1 * 16 + 1: mfma_level<3, 1, 1>(lds, lds_f, P, T, g); break;
    case 4 * 256 + 1 * 16 + 1: mfma_level<4, 1, 1>(lds, lds_f, P, T, g); break;
    default: break;  // the host only builds supported level shapes
  }
}

__device__ FRNTT_INLINE void mfma_levels(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T) {
  int pprev = 0;
  int rest = P.log_r;
  for (int lev = 0; lev < P.nlev; ++lev) {
    LevelGeom g;
    g.m = P.lev_log[lev];
    rest -= g.m;
    g.pprev_log = pprev;
    g.q_log = rest;
    g.next_m = lev + 1 < P.nlev ? P.lev_log[lev + 1] : 0;
    g.last = lev + 1 == P.nlev;
    run_mfma_level(lds, lds_f, P, T, g);
    pprev += g.m;
  }
}

// ------------------------------------------------------------- one pass

// ENGINE: 0 butterfly only, 1 MFMA only, 2 per-pass choice (P.engine).
template <int ENGINE>
__device__ FRNTT_INLINE void run_pass(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                      int64_t wg) {
  load_lines(lds, P, T, wg);
  __syncthreads();
  const bool use_mfma = ENGINE == 1 || (ENGINE == 2 && P.engine == 1);
  if (use_mfma) mfma_levels(lds, lds_f, P, T);
  else bfly_stages(lds, P, T);
  store_lines(lds, P, T, wg, !use_mfma);
}

}  // namespace frntt
