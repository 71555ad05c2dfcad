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
//   * butterfly: radix-4 (and one radix-2) decimation-in-frequency stages in
//     LDS with Montgomery twiddle products on the VALUs (the paper's
//     butterfly NTT);
//   * MFMA: nested levels of radix rho <= 16. Level l reads LDS row n_l (its
//     input digit) across V = T / rho vectors; the rho-point DFT of 32
//     vectors at a time is a GEMM of the BAT byte-limb constant blocks
//     E[(k,h),(n,a)] (signed digit h of w^(kn) * 2^(8a) mod r) with the data
//     bytes on int8 MFMA (Alg. 1's ByteDecompose and einsum). Outputs come in
//     pairs (k', k' + rho/2): the even-digit and odd-digit sums e, o of
//     w^(k' n) x_n take rho MFMAs, and e + o, e - o are the two outputs
//     (w^((k' + rho/2) n) = (-1)^n w^(k' n)), so a radix-rho level costs
//     rho^2 / 2 MFMAs per 32 vectors. Then the carry merge
//     sum_h P_h 2^(8h) and reduction mod r (ByteMerge and the final
//     correction), the inter-level twiddle, and a write into the row order
//     the next level reads. The vector work of one pair runs between the
//     MFMAs of the next.
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
// coset pre-scale x_n * g^n in the first pass of a coset transform). A thread
// takes U elements at a time: it computes their addresses, issues all their
// loads (data and coset factors), and only then waits, so a full tile arrives
// in one memory round trip instead of one per element. STRIDED: a non-last
// pass, whose pass axis is strided in memory (neighbouring threads take
// neighbouring lines); in the last pass lines are contiguous and
// neighbouring threads take neighbouring n. PRE is the pre-scale: 0 none,
// 1 g^idx from the split tables (two factors per element), 2 the per-line
// part rides in the pass table and (g^(2^S))^n sits at the table's end.
template <int NT, int U, int PRE, bool STRIDED>
__device__ FRNTT_INLINE void load_lines_u(u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  const int T_el = 1 << P.log_t;
  const int G = 1 << P.log_g;
  const int64_t nmask = (1ll << P.log_n) - 1;
  for (int e0 = threadIdx.x; e0 < T_el; e0 += NT * U) {
    int64_t idx[U];
    int pos[U], nn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * NT;
      int line;
      if constexpr (STRIDED) {
        nn[u] = e >> P.log_g;
        line = e & (G - 1);
        pos[u] = e;
      } else {
        line = e >> P.log_r;
        nn[u] = e & ((1 << P.log_r) - 1);
        pos[u] = nn[u] * G + line;
      }
      const int64_t base = line_in_base<STRIDED>(P, wg * G + line);
      idx[u] = base + ((int64_t)nn[u] << (STRIDED ? P.log_s : 0));
    }
    fr_t x[U], f0[U], f1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = ld_elem(P.src, idx[u]);
      if constexpr (PRE == 1) {
        const uint32_t i = (uint32_t)(idx[u] & nmask);
        f0[u] = ld_elem(T.g_lo[0], i & ((1u << kSplit) - 1));
        f1[u] = ld_elem(T.g_hi[0], i >> kSplit);
      } else if constexpr (PRE == 2) {
        f0[u] = ld_elem(P.pass_tw, (1ll << (P.log_r + P.log_s)) + nn[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fr_t y = x[u];
      if constexpr (PRE == 1) y = mont_mul(y, mont_mul(f0[u], f1[u]));
      else if constexpr (PRE == 2) y = mont_mul(y, f0[u]);
      lds_st(lds, pos[u], y);
    }
  }
}

template <int NT, int U, bool STRIDED>
__device__ FRNTT_INLINE void load_lines_s(u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  // the last pass (a single-pass coset transform) takes g^idx from the split
  // tables. With a pre-scale product per element the unrolled body grows
  // large, so fewer elements are kept in flight.
  const int pre = STRIDED ? P.coset_pre : (P.coset_pre ? 1 : 0);
  constexpr int U1 = U > 2 ? 2 : 1;
  if ((1 << P.log_t) < NT * U) {
    // a tile smaller than NT * U elements: one element per thread at a time
    if (pre == 0) load_lines_u<NT, 1, 0, STRIDED>(lds, P, T, wg);
    else if (pre == 2) load_lines_u<NT, 1, 2, STRIDED>(lds, P, T, wg);
    else load_lines_u<NT, 1, 1, STRIDED>(lds, P, T, wg);
  } else if (pre == 0) {
    load_lines_u<NT, U, 0, STRIDED>(lds, P, T, wg);
  } else if (pre == 2) {
    load_lines_u<NT, U1, 2, STRIDED>(lds, P, T, wg);
  } else {
    load_lines_u<NT, U1, 1, STRIDED>(lds, P, T, wg);
  }
}

// NT * U must divide the tile when the tile has at least NT * U elements
// (both are powers of two).
template <int NT, int U>
__device__ FRNTT_INLINE void load_lines(u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  if (P.is_last) load_lines_s<NT, U, false>(lds, P, T, wg);
  else load_lines_s<NT, U, true>(lds, P, T, wg);
}

// Butterfly engine: write output k of every line (found at LDS row
// bitrev(k)) to HBM, applying the pass twiddle w^(rest * k) of the
// size-2^(l+S) sub-problem, or the last pass's N^-1 / N^-1 g^-k epilogue.
// (The MFMA engine applies them in its last level, which stores its outputs
// itself.)
template <int NT>
__device__ FRNTT_INLINE void store_lines(const u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  const int T_el = 1 << P.log_t;
  const int G = 1 << P.log_g;
  const int tid = threadIdx.x;
  // two elements in flight per thread: their table loads overlap
#pragma unroll 2
  for (int e = tid; e < T_el; e += NT) {
    const int k = e >> P.log_g, line = e & (G - 1);
    const int row = (int)(__builtin_bitreverse32((uint32_t)k) >> (32 - P.log_r));
    fr_t y = lds_ld(lds, row * G + line);
    const LineMap mp = map_line(P, wg * G + line);
    if (!P.is_last) {
      const fr_t tw = P.pass_tw ? ld_elem(P.pass_tw, ((int64_t)k << P.log_s) + mp.rest)
                                : pow_tw(T, P.dir, P.log_r + P.log_s, (uint64_t)mp.rest * (uint64_t)k);
      y = mont_mul(tw, y);
    } else if (P.post == 1) {
      y = mont_mul(ld_elem(T.ninv, P.log_n), y);
    } else if (P.post == 2) {
      const uint32_t idx = (uint32_t)(mp.poly_off + ((int64_t)k << mp.out_shift));
      y = mont_mul(mont_mul(ld_elem(T.ninv, P.log_n), coset_pow(T, 1, idx)), y);
    } else if (P.post == 3) {
      const uint32_t idx = (uint32_t)(mp.poly_off + ((int64_t)k << mp.out_shift));
      y = mont_mul(coset_pow(T, 1, idx), y);
    } else if (P.post == 4) {
      y = mont_mul(ld_elem(P.post_tw, k), y);
    }
    st_elem(P.dst, mp.out_base + ((int64_t)k << mp.out_shift), y);
  }
}

// ------------------------------------------------------- butterfly engine

// Radix-2 and radix-4 decimation-in-frequency stages over every line, in
// place in LDS; afterwards row i of a line holds output bitrev(i).
//
// A radix-4 stage is two radix-2 DIF stages fused. With quarter span q,
// w = w_(4q) and j = i mod q, the inputs a, b, c, d at rows i, i + q,
// i + 2q, i + 3q become
//   t0 = a + c, t1 = a - c, t2 = b + d, t3 = (b - d) w_4,
//   row i: t0 + t2,            row i + q:  (t0 - t2) w^(2j),
//   row i + 2q: (t1 + t3) w^j, row i + 3q: (t1 - t3) w^(3j),
// which is what the two radix-2 stages leave in those rows (w^(j+q) =
// w^j w_4 and w_(2q)^j = w^(2j)). One product by w_4 and three twiddle
// products per four elements, the same count as two radix-2 stages, but half
// the LDS round trips and barriers; in the last stage (q = 1, j = 0) the
// three twiddles are 1 and are skipped. An odd log_r starts with one radix-2
// stage.
template <int NT>
__device__ FRNTT_INLINE void bfly_stages(u32x4* lds, const PassParams& P, const DevTables& T) {
  const int G = 1 << P.log_g;
  const int tid = threadIdx.x;
  const u32x4* w = T.w4096[P.dir];
  int left = P.log_r;  // log2 span of the blocks still to split
  if (left & 1) {
    const int half_el = 1 << (P.log_t - 1);
    const int log_span = left - 1;
    const int span = 1 << log_span;
#pragma unroll 1
    for (int b = tid; b < half_el; b += NT) {
      const int line = b & (G - 1);
      const int bb = b >> P.log_g;             // butterfly index inside the line
      const int j = bb & (span - 1);
      const int i0 = ((bb >> log_span) << (log_span + 1)) + j;
      const int e0 = i0 * G + line, e1 = (i0 + span) * G + line;
      const fr_t u = lds_ld(lds, e0), v = lds_ld(lds, e1);
      lds_st(lds, e0, fr_add(u, v));
      // w_(2 span)^j = w_4096^(j * 4096 / (2 span))
      const fr_t tw = ld_elem(w, j << (12 - log_span - 1));
      lds_st(lds, e1, mont_mul(fr_sub(u, v), tw));
    }
    __syncthreads();
    left -= 1;
  }
  const fr_t w4 = ld_elem(w, 1024);  // w_4 = w_4096^1024
  const int quarter_el = 1 << (P.log_t - 2);
  for (; left >= 2; left -= 2) {
    const int log_q = left - 2;
    const int q = 1 << log_q;
    const int tw_shift = 12 - log_q - 2;  // w_(4q)^e = w_4096^(e << tw_shift)
#pragma unroll 1
    for (int b = tid; b < quarter_el; b += NT) {
      const int line = b & (G - 1);
      const int bb = b >> P.log_g;             // radix-4 butterfly index inside the line
      const int j = bb & (q - 1);
      const int i0 = ((bb >> log_q) << (log_q + 2)) + j;
      const int e0 = i0 * G + line, e1 = e0 + q * G, e2 = e1 + q * G, e3 = e2 + q * G;
      const fr_t a = lds_ld(lds, e0), bq = lds_ld(lds, e1), c = lds_ld(lds, e2), d = lds_ld(lds, e3);
      const fr_t t0 = fr_add(a, c), t1 = fr_sub(a, c), t2 = fr_add(bq, d);
      const fr_t t3 = mont_mul(fr_sub(bq, d), w4);
      lds_st(lds, e0, fr_add(t0, t2));
      if (log_q == 0) {
        lds_st(lds, e1, fr_sub(t0, t2));
        lds_st(lds, e2, fr_add(t1, t3));
        lds_st(lds, e3, fr_sub(t1, t3));
      } else {
        lds_st(lds, e1, mont_mul(fr_sub(t0, t2), ld_elem(w, ((2 * j) << tw_shift) & 4095)));
        lds_st(lds, e2, mont_mul(fr_add(t1, t3), ld_elem(w, (j << tw_shift) & 4095)));
        lds_st(lds, e3, mont_mul(fr_sub(t1, t3), ld_elem(w, ((3 * j) << tw_shift) & 4095)));
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ MFMA level

// Top 32-bit word of r plus one, inverted: floor(t / (r_top + 1)) for the
// top bits t of y never exceeds the true quotient floor(y / r).
#define FR_INV_RTOP1 (1.0 / 811880051.0)  // r_top = 0x30644e72 = 811880050

// Merge the byte-plane partials of an output pair and reduce mod r. The
// pair comes as its even-digit and odd-digit accumulators e and o: output k0
// (lanes 0..31 after the swap) has partials e + o, output k1 (lanes 32..63)
// e - o. Lane l holds rows h = 8i + 4*(l/32) + j in register 4i + j (the
// 32x32 MFMA accumulator layout), i.e. the partials of 32-bit words
// 2i + l/32. A word group sum_j P_(4w+j) 2^(8j) of e and of o is a signed
// 64-bit sum of four 32x32+64 multiply-adds; their sum and difference are the
// groups of the two outputs. The seeds lift every partial of e + o and e - o
// into [0, 2^26) (their offsets add a multiple of r), so those groups are
// unsigned values below 2^50. After the swap of the two half-waves each lane
// holds the 8 word groups of its own output; one add-with-carry per word
// then gives y = sum_h P_h 2^(8h) < 2^275 as nine words. A quotient estimate
// from the top 51 bits, at most 2 below floor(y / r), brings y into [0, 3r).
//
// The work is cut into kMergeSteps steps of a few instructions, so that it
// can be spread over the MFMA issue slots of the next outputs.
constexpr int kMergeSteps = 16;

struct Merge {
  i32x16 a0, a1;                // the pair's even and odd accumulators
  uint32_t w1, w8, w16, w24;    // 1, 2^8, 2^16, 2^24 (kernel arguments)
  uint64_t g0[4], g1[4];
  int64_t ge, go;
  uint64_t X[4], Y[4];
  uint32_t y[9];
  uint32_t c;
  int32_t q;
  uint32_t carry, br;

  // signed word group i of accumulator a
  __device__ FRNTT_INLINE int64_t group(const i32x16& a, int i) const {
    int64_t x = (int64_t)a[4 * i] * (int64_t)(int32_t)w1;
    x = (int64_t)a[4 * i + 1] * (int64_t)(int32_t)w8 + x;
    x = (int64_t)a[4 * i + 2] * (int64_t)(int32_t)w16 + x;
    return (int64_t)a[4 * i + 3] * (int64_t)(int32_t)w24 + x;
  }
  __device__ FRNTT_INLINE void swap(int i) {
    auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)g0[i], (uint32_t)g1[i], false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(g0[i] >> 32), (uint32_t)(g1[i] >> 32), false, false);
    X[i] = ((uint64_t)hi[0] << 32) | (uint32_t)lo[0];  // word 2i
    Y[i] = ((uint64_t)hi[1] << 32) | (uint32_t)lo[1];  // word 2i + 1
  }
  __device__ FRNTT_INLINE void carry_word(int w) {
    const uint64_t s = ((w & 1) ? Y[w >> 1] : X[w >> 1]) + (w == 0 ? 0u : c);
    y[w] = (uint32_t)s;
    c = (uint32_t)(s >> 32);
  }
  __device__ FRNTT_INLINE void sub_qr(int i) {
    const uint64_t p = (uint64_t)(uint32_t)q * fr_mod_word(i) + carry;
    carry = (uint32_t)(p >> 32);
    y[i] = subb(y[i], (uint32_t)p, br, &br);
  }
  // step S of kMergeSteps
  template <int S>
  __device__ FRNTT_INLINE void step() {
    if constexpr (S < 8) {
      // even steps: group S/2 of e and o; odd steps: the outputs' groups
      if constexpr ((S & 1) == 0) {
        ge = group(a0, S >> 1);
        go = group(a1, S >> 1);
      } else {
        g0[S >> 1] = (uint64_t)(ge + go);
        g1[S >> 1] = (uint64_t)(ge - go);
      }
    } else if constexpr (S == 8) {
      swap(0); swap(1);
    } else if constexpr (S == 9) {
      swap(2); swap(3);
    } else if constexpr (S < 13) {
      carry_word(2 * (S - 10)); carry_word(2 * (S - 10) + 1);
    } else if constexpr (S == 13) {
      carry_word(6); carry_word(7);
      y[8] = c;
    } else if constexpr (S == 14) {
      // quotient estimate from the top 51 bits y[8] * 2^32 + y[7] (exact in fp64)
      const double t = __builtin_fma((double)y[8], 4294967296.0, (double)y[7]);
      q = (int32_t)(t * FR_INV_RTOP1) - 1;
      q = q < 0 ? 0 : q;
      carry = 0;
      br = 0;
      sub_qr(0); sub_qr(1); sub_qr(2); sub_qr(3);
    } else {
      sub_qr(4); sub_qr(5); sub_qr(6); sub_qr(7);
    }
  }
  __device__ FRNTT_INLINE fr_t result() const {
    fr_t o;
#pragma unroll
    for (int i = 0; i < 8; ++i) o.w[i] = y[i];
    return o;
  }
};

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

// LDS position of output digit k of vector v: the row order the next level
// reads, or, after the last level, row k of its line.
__device__ FRNTT_INLINE int level_out_pos(const PassParams& P, const LevelGeom& g, int v, int k) {
  const int line = v & ((1 << P.log_g) - 1);
  const int rem = v >> P.log_g;
  const int kk = rem & ((1 << g.pprev_log) - 1);
  const int nn = rem >> g.pprev_log;
  if (g.last) return ((kk + (k << g.pprev_log)) << P.log_g) + line;
  const int nshift = g.q_log - g.next_m;
  const int n_next = nn >> nshift;
  const int nn2 = nn & ((1 << nshift) - 1);
  const int col = line + ((kk + (k << g.pprev_log) + (nn2 << (g.pprev_log + g.m))) << P.log_g);
  return (n_next << (P.log_t - g.next_m)) + col;
}

// Constant blocks of radix 2^M (RHO x 64 lanes x 16 B of signed digits)
// followed by the accumulator seeds (RHO x 2 halves x 16 int32), staged in
// LDS: load() issues a thread's loads, store() writes them to LDS (in
// between, other loads can be issued, whose latency the staging then covers).
template <int M, int NT>
struct BatStage {
  static constexpr int RHO = 1 << M;
  static constexpr int NB = (RHO * 64 + NT - 1) / NT, NS = (RHO * 8 + NT - 1) / NT;
  i32x4 b[NB], sd[NS];
  // slot u of the thread lies below `count` (always, when all NT threads' slots do)
  __device__ FRNTT_INLINE static bool in_range(int u, int count) {
    return (u + 1) * NT <= count || (int)threadIdx.x + u * NT < count;
  }
  __device__ FRNTT_INLINE void load(const DevTables& T, int dir) {
    const i32x4* bat = T.bat[dir][M];
    const i32x4* seeds = T.bat_init[dir][M];
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (in_range(u, RHO * 64)) b[u] = bat[tid + u * NT];
#pragma unroll
    for (int u = 0; u < NS; ++u)
      if (in_range(u, RHO * 8)) sd[u] = seeds[tid + u * NT];
  }
  __device__ FRNTT_INLINE void store(i32x4* dst) const {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (in_range(u, RHO * 64)) dst[tid + u * NT] = b[u];
#pragma unroll
    for (int u = 0; u < NS; ++u)
      if (in_range(u, RHO * 8)) dst[RHO * 64 + tid + u * NT] = sd[u];
  }
};

// All loads of a thread first, then its LDS stores: one memory round trip.
template <int M, int NT>
__device__ FRNTT_INLINE void stage_bat(i32x4* dst, const DevTables& T, int dir) {
  BatStage<M, NT> s;
  s.load(T, dir);
  s.store(dst);
}

template <int M>
constexpr int bat_lds_size() { return (1 << M) * 72; }  // i32x4 units

// Per-lane work on one output of a pair, cut into kSteps small steps: the
// carry merge, then
//   KIND 0: nothing (last level of a forward or coset transform: the store
//           reduces y < 3r),
//   KIND 1: the inter-level twiddle w^(nn k) of the size-2^(m + q_log)
//           sub-problem: one Shoup product of the merged value, taken before
//           the merge's own reduction (it accepts inputs below 2^290), output
//           left below 3r,
//   KIND 2: the pass twiddle w^(rest k) of the size-2^(l + S) sub-problem
//           (last level of a non-last pass; the twiddle is the product of two
//           table entries: two Montgomery products, output left below 2r),
//   KIND 3: the inverse transform's N^-1 (last level of the last pass),
//   KIND 4: the coset inverse's N^-1 g^-k (g^-k from two table entries:
//           three Montgomery products),
//   KIND 5: the pass twiddle read from the pass's twiddle table (one
//           Montgomery product, output left below 2r).
// Outputs of a non-last pass stay below 2r: the next pass is on the matrix
// form too (every pass of a transform has a full tile), and its first level
// reads only their 32 bytes.
template <int KIND>
struct PairWork {
  static constexpr int kProducts = KIND == 0 ? 0 : (KIND == 2 || KIND == 6) ? 2 : KIND == 4 ? 3 : 1;
  // KIND 1: the merge without its last two (reduction) steps, then the Shoup
  // product
  static constexpr int kMergeUsed = KIND == 1 ? kMergeSteps - 2 : kMergeSteps;
  static constexpr int kSteps = KIND == 1 ? kMergeUsed + ShoupMul::kSteps : kMergeSteps + 11 * kProducts;
  Merge mg;
  MontMul mm;
  ShoupMul sh;
  fr_t tw, tw2, tw3;  // factors (Montgomery form), loaded when the pair starts
  uint32_t twp[10], tww[9];  // KIND 1: the inter-level twiddle in the Shoup operand form
  fr_t y;             // the output of the pair: below 3r for KIND 0 and 1, canonical otherwise

  // step Q of a Montgomery product a * b -> out (11 steps); a LAZY product
  // leaves its output below 2r (the inter-level twiddle: the next level reads
  // only its 32 bytes)
  template <int Q, bool LAZY = false>
  __device__ FRNTT_INLINE void prod(const fr_t& a, const fr_t& b, fr_t& out) {
    if constexpr (Q == 0) mm.load(a, b);
    else if constexpr (Q <= 9) mm.row(Q - 1);
    else if constexpr (LAZY) out = mm.finish_lazy();
    else out = mm.finish();
  }
  template <int S>
  __device__ FRNTT_INLINE void step() {
    constexpr int P0 = kMergeSteps, P1 = kMergeSteps + 11, P2 = kMergeSteps + 22;
    if constexpr (KIND == 1) {
      if constexpr (S < kMergeUsed) {
        mg.template step<S>();
      } else {
        sh.template step<S - kMergeUsed>(twp, tww, mg.y);
        if constexpr (S == kSteps - 1) y = sh.out;
      }
    } else if constexpr (S < P0) {
      mg.template step<S>();
      if constexpr (S == P0 - 1) y = mg.result();
    } else if constexpr (KIND == 5) {
      prod<S - P0, true>(tw, y, y);
    } else if constexpr (KIND == 3 || KIND == 7) {
      prod<S - P0>(tw, y, y);
    } else if constexpr (KIND == 2) {
      if constexpr (S < P1) prod<S - P0, true>(tw, tw2, tw);
      else prod<S - P1, true>(tw, y, y);
    } else if constexpr (KIND == 6) {
      if constexpr (S < P1) prod<S - P0, true>(tw, tw2, tw);
      else prod<S - P1>(tw, y, y);
    } else {
      if constexpr (S < P1) prod<S - P0>(tw, tw2, tw);          // g^-k
      else if constexpr (S < P2) prod<S - P1>(tw3, tw, tw);     // N^-1 g^-k
      else prod<S - P2>(tw, y, y);
    }
  }
  // steps [S0, S1)
  template <int S0, int S1>
  __device__ FRNTT_INLINE void steps() {
    if constexpr (S0 < S1) {
      step<S0>();
      steps<S0 + 1, S1>();
    }
  }
};

// One pipelined output pair (k', k' + RHO/2) of a tile: the RHO MFMAs of
// digits n = 0..RHO-1 accumulate into e (n even) and o (n odd) with the
// blocks of k' n mod RHO; e + o is output k' and e - o output k' + RHO/2
// (w^((k' + RHO/2) n) = (-1)^n w^(k' n)), formed by the merge. The work `wk` on
// the previous pair (if WORKING) advances through its steps, spread evenly
// over the MFMA issue slots; the constant blocks are read from LDS one digit
// ahead, and a scheduling barrier after each digit keeps the vector work
// between the MFMAs, so the matrix and vector pipes of a SIMD overlap.
template <int RHO, bool WORKING, class W, int N>
struct DigitLoop {
  __device__ FRNTT_INLINE static void run(const i32x4* lds_f, const i32x4 (&Bt)[RHO], int k0, int lane,
                                          i32x16& e, i32x16& o, W& wk, i32x4 a) {
    if constexpr (N < RHO) {
      i32x4 p = a;
      if constexpr (N + 1 < RHO) p = lds_f[((k0 * (N + 1)) & (RHO - 1)) * 64 + lane];
      if constexpr (N & 1) o = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, Bt[N], o, 0, 0, 0);
      else e = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, Bt[N], e, 0, 0, 0);
      if constexpr (WORKING) wk.template steps<N * W::kSteps / RHO, (N + 1) * W::kSteps / RHO>();
      __builtin_amdgcn_sched_barrier(0);
      DigitLoop<RHO, WORKING, W, N + 1>::run(lds_f, Bt, k0, lane, e, o, wk, p);
    }
  }
};

// Seeds of the pair's even and odd accumulators: the signed-digit correction
// of their digits and, on the even one only, the row offsets.
template <int RHO, bool WORKING, class W>
__device__ FRNTT_INLINE void mfma_pair_work(const i32x4* lds_f, const i32x4* init, const i32x4 (&Bt)[RHO], int k0,
                                            int lane, int half, i32x16& e, i32x16& o, W& wk) {
  e = load_init(init, 2 * k0, half);
  o = load_init(init, 2 * k0 + 1, half);
  const i32x4 a = lds_f[lane];  // k' * 0 = 0
  DigitLoop<RHO, WORKING, W, 0>::run(lds_f, Bt, k0, lane, e, o, wk, a);
}

// Unsigned data bytes u -> signed u - 128 (the seeds carry 128 times the
// digit sums).
template <int RHO>
__device__ FRNTT_INLINE void to_signed(i32x4 (&b)[RHO]) {
#pragma unroll
  for (int n = 0; n < RHO; ++n) b[n] = (i32x4)((u32x4)b[n] ^ 0x80808080u);
}

// The output pairs of tile T of a wave (tiles unrolled at compile time, so
// every data-fragment index is static): pair kp is finished while the MFMAs
// of the next pair (of this tile, or the first of the next) run. RAW: the
// fragments of later tiles still hold unsigned bytes straight from HBM; the
// next tile's are converted when this one starts, so that the wait for
// their loads falls after this tile's first MFMAs.
template <int M, int TPW, int KIND, int T, bool RAW>
struct TileLoop {
  __device__ FRNTT_INLINE static void run(u32x4* lds, const i32x4* lds_f, const i32x4* init, const PassParams& P,
                                          const DevTables& Tb, const LevelGeom& g, i32x4 (&B)[TPW][1 << M],
                                          int tile0, int col, int half, int lane, int64_t wg, i32x16& n0,
                                          i32x16& n1, PairWork<KIND>& wk) {
    if constexpr (T < TPW) {
      constexpr int RHO = 1 << M;
      constexpr int NKP = RHO / 2;
      if constexpr (RAW && T + 1 < TPW) to_signed<RHO>(B[T + 1]);
      const int v = (tile0 + T) * 32 + col;
      const int rem = v >> P.log_g;
      const int nn = rem >> g.pprev_log;                 // KIND 1: the vector's twiddle row
      const int kk = rem & ((1 << g.pprev_log) - 1);     // KIND 2: earlier output digits
      // KIND 2, 5: the line's pass-twiddle row; KIND 4: the line's output base
      // and stride inside its polynomial
      LineMap mp{};
      if (KIND != 1) mp = map_line(P, wg * (1 << P.log_g) + (v & ((1 << P.log_g) - 1)));
      const int64_t rest = mp.rest;
      // KIND 5: the pass twiddle comes from an HBM table; it is loaded one pair
      // earlier than the other factors, so that its latency is covered by a
      // whole pair of MFMAs
      fr_t tw_next;
      if (KIND == 5) tw_next = ld_elem(P.pass_tw, ((int64_t)(kk + ((half * NKP) << g.pprev_log)) << P.log_s) + rest);
#pragma unroll 1
      for (int kp = 0; kp < NKP; ++kp) {
        const int k = kp + half * NKP;  // this lane's output digit: pair kp holds kp and kp + RHO/2
        wk.mg.a0 = n0;
        wk.mg.a1 = n1;
        if (KIND == 1) small_tw_shoup(Tb, P.dir, g.m + g.q_log, (uint32_t)(nn * k), wk.twp, wk.tww);
        if (KIND == 2) {
          const uint64_t e = (uint64_t)rest * (uint64_t)(kk + (k << g.pprev_log));
          const uint32_t E = (uint32_t)((e << (kMasterLog - P.log_r - P.log_s)) & ((1u << kMasterLog) - 1));
          wk.tw = ld_elem(Tb.tw_lo[P.dir], E & ((1u << kSplit) - 1));
          wk.tw2 = ld_elem(Tb.tw_hi[P.dir], E >> kSplit);
        }
        if (KIND == 5) {
          wk.tw = tw_next;
          if (kp + 1 < NKP) tw_next = ld_elem(P.pass_tw, ((int64_t)(kk + ((k + 1) << g.pprev_log)) << P.log_s) + rest);
        }
        if (KIND == 3) wk.tw = ld_elem(Tb.ninv, P.log_n);
        if (KIND == 7) wk.tw = ld_elem(P.post_tw, kk + (k << g.pprev_log));
        if (KIND == 4 || KIND == 6) {
          const uint32_t idx = (uint32_t)(mp.poly_off + ((int64_t)(kk + (k << g.pprev_log)) << mp.out_shift));
          wk.tw = ld_elem(Tb.g_lo[1], idx & ((1u << kSplit) - 1));
          wk.tw2 = ld_elem(Tb.g_hi[1], idx >> kSplit);
          if (KIND == 4) wk.tw3 = ld_elem(Tb.ninv, P.log_n);
        }
        if (kp + 1 < NKP) {
          mfma_pair_work<RHO, true>(lds_f, init, B[T], kp + 1, lane, half, n0, n1, wk);
        } else if constexpr (T + 1 < TPW) {
          mfma_pair_work<RHO, true>(lds_f, init, B[T + 1], 0, lane, half, n0, n1, wk);
        } else {
          wk.template steps<0, PairWork<KIND>::kSteps>();
        }
        if constexpr (KIND == 1) {
          lds_st(lds, level_out_pos(P, g, v, k), wk.y);
        } else {
          // last level: the output goes straight to HBM, while the next
          // pairs compute (forward outputs of the last pass are below 3r)
          fr_t y = wk.y;
          if constexpr (KIND == 0) y = fr_reduce_3r(y);
          st_elem(P.dst, mp.out_base + ((int64_t)(kk + (k << g.pprev_log)) << mp.out_shift), y);
        }
      }
      TileLoop<M, TPW, KIND, T + 1, RAW>::run(lds, lds_f, init, P, Tb, g, B, tile0, col, half, lane, wg, n0, n1, wk);
    }
  }
};

// Nothing to stage (the constant blocks are in LDS already).
struct NoStage {
  __device__ FRNTT_INLINE void store() const {}
};

// One MFMA level. The 2^(log_t - m) vectors form tiles of 32; each of the 8
// waves takes TPW whole tiles. A wave first loads the data fragments of its
// tiles (lane l: bytes 16*(l/32)..+15 of vector l%32 for every input digit
// n), so that after the barrier the level can overwrite LDS in place. The
// output pairs of a wave form a software pipeline: while the MFMAs of pair
// i + 1 run, pair i is merged, reduced below 3r, multiplied by its
// inter-level or pass twiddle and written to the position the next level
// reads, or, in the last level, straight to its place in HBM (KIND: see
// PairWork).
//
// HBM: the first level of a pass without a pre-scale reads its fragments
// straight from the pass's input instead of from a tile staged in LDS, so
// that no load phase precedes the MFMAs: a wave issues all its fragment
// loads, then `st` writes the constant blocks whose loads were issued before
// (covering part of the fragments' latency), and the first pair waits only
// for the first tile's fragments. Input digit n of vector v = (n_low, line)
// is element n * R / rho + n_low of the line, which the staged tile would
// have held at row n of vector v.
template <int M, int TPW, int KIND, bool HBM = false, class ST = NoStage>
__device__ FRNTT_INLINE void mfma_level(u32x4* lds, i32x4* blk, const PassParams& P, const DevTables& T,
                                        const LevelGeom& g, bool stage, int64_t wg, const ST& st = ST()) {
  constexpr int RHO = 1 << M;
  constexpr int NKP = RHO / 2;  // output pairs per tile
  const int V = 1 << (P.log_t - M);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int tile0 = wave * TPW;
  // this radix's constant blocks and accumulator seeds (staged here, or for
  // the whole pass before its loads)
  if (stage) stage_bat<M, kMfmaThreads>(blk, T, P.dir);
  const i32x4* lds_f = blk;
  const i32x4* init = blk + RHO * 64;
  i32x4 B[TPW][RHO];
  if constexpr (HBM) {
    const int G = 1 << P.log_g;
    const int row_log = P.log_r - M;  // log2 of R / rho
    const int shift = P.is_last ? 0 : P.log_s;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int v = (tile0 + t) * 32 + col;
      const int line = v & (G - 1);
      const int n_low = v >> P.log_g;
      const int64_t l = wg * G + line;
      const int64_t base = P.is_last ? line_in_base<false>(P, l) : line_in_base<true>(P, l);
#pragma unroll
      for (int n = 0; n < RHO; ++n) {
        const int64_t idx = base + ((int64_t)((n << row_log) + n_low) << shift);
        B[t][n] = (i32x4)P.src[2 * idx + half];
      }
    }
    st.store();
    __syncthreads();
    to_signed<RHO>(B[0]);
  } else {
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
  }
  PairWork<KIND> wk;
  wk.mg.w1 = T.byte_w[3];
  wk.mg.w8 = T.byte_w[0];
  wk.mg.w16 = T.byte_w[1];
  wk.mg.w24 = T.byte_w[2];
  i32x16 n0, n1;
  mfma_pair_work<RHO, false>(lds_f, init, B[0], 0, lane, half, n0, n1, wk);
  TileLoop<M, TPW, KIND, 0, HBM>::run(lds, lds_f, init, P, T, g, B, tile0, col, half, lane, wg, n0, n1, wk);
  __syncthreads();
}

// A pass of the matrix form (tile of 4096 elements) whose levels are known
// at compile time: radices 2^M0, then 2^M1 if M1 > 0, then 2^M2 if M2 > 0.
// The constant blocks of its (at most two) distinct radices are staged once,
// together with the tile's HBM loads, and every level shape is fixed.
template <int M0, int M1, int M2>
struct PassPlan {
  static constexpr int kLevels = M2 > 0 ? 3 : M1 > 0 ? 2 : 1;
  static_assert(M1 > 0 || M2 == 0, "levels are given in order");
  static_assert(M1 == 0 || M1 == M0 || M2 == 0 || M2 == M0 || M2 == M1, "at most two distinct radices");
  // LDS offsets of the blocks of each level: the first radix at 0, the
  // other distinct radix (M1, or M2 when M1 == M0) after it
  static constexpr int kOff1 = M1 == M0 || M1 == 0 ? 0 : bat_lds_size<M0>();
  static constexpr int kOff2 = M2 == M0 ? 0 : (M2 == M1 ? kOff1 : bat_lds_size<M0>());
  static constexpr bool kStage1 = M1 > 0 && M1 != M0;
  static constexpr bool kStage2 = M2 > 0 && M2 != M0 && M2 != M1;
  static constexpr int kLds = bat_lds_size<M0>() + (kStage1 ? bat_lds_size<(M1 > 0 ? M1 : 1)>() : 0) +
                              (kStage2 ? bat_lds_size<(M2 > 0 ? M2 : 1)>() : 0);
};
constexpr int kPlanBatLds = bat_lds_size<4>() + bat_lds_size<3>();

__device__ FRNTT_INLINE LevelGeom level_geom(int m, int pprev, int q, int next_m) {
  LevelGeom g;
  g.m = m;
  g.pprev_log = pprev;
  g.q_log = q;
  g.next_m = next_m;
  g.last = next_m == 0;
  return g;
}

// Last level of a planned pass: the pass twiddle, or the last pass's
// epilogue, rides on it.
template <int M>
__device__ FRNTT_INLINE void plan_last_level(u32x4* lds, i32x4* blk, const PassParams& P, const DevTables& T,
                                             const LevelGeom& g, int64_t wg) {
  constexpr int TPW = 1 << (kMaxLogT - M - 8);
  if (!P.is_last && P.pass_tw) mfma_level<M, TPW, 5>(lds, blk, P, T, g, false, wg);
  else if (!P.is_last) mfma_level<M, TPW, 2>(lds, blk, P, T, g, false, wg);
  else if (P.post == 1) mfma_level<M, TPW, 3>(lds, blk, P, T, g, false, wg);
  else if (P.post == 2) mfma_level<M, TPW, 4>(lds, blk, P, T, g, false, wg);
  else if (P.post == 3) mfma_level<M, TPW, 6>(lds, blk, P, T, g, false, wg);
  else if (P.post == 4) mfma_level<M, TPW, 7>(lds, blk, P, T, g, false, wg);
  else mfma_level<M, TPW, 0>(lds, blk, P, T, g, false, wg);
}

// The constant blocks of a pass's distinct radices, loaded before the first
// level's fragment loads are issued and stored to LDS after them (nothing if
// `on` is false: a workgroup running several tiles of one pass in a row
// stages them once).
template <int M0, int M1, int M2>
struct PlanStage {
  using PL = PassPlan<M0, M1, M2>;
  BatStage<M0, kMfmaThreads> s0;
  BatStage<(M1 > 0 ? M1 : 1), kMfmaThreads> s1;
  BatStage<(M2 > 0 ? M2 : 1), kMfmaThreads> s2;
  i32x4* dst;
  bool on;
  __device__ FRNTT_INLINE void load(const DevTables& T, int dir) {
    if (!on) return;
    s0.load(T, dir);
    if constexpr (PL::kStage1) s1.load(T, dir);
    if constexpr (PL::kStage2) s2.load(T, dir);
  }
  __device__ FRNTT_INLINE void store() const {
    if (!on) return;
    s0.store(dst);
    if constexpr (PL::kStage1) s1.store(dst + PL::kOff1);
    if constexpr (PL::kStage2) s2.store(dst + PL::kOff2);
  }
};

template <int M0, int M1, int M2>
__device__ FRNTT_INLINE void run_pass_plan(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                           int64_t wg, bool stage = true) {
  using PL = PassPlan<M0, M1, M2>;
  constexpr int LT = kMaxLogT;  // staged elements 2^12
  if constexpr (M1 == 0) {
    if (stage) stage_bat<M0, kMfmaThreads>(lds_f, T, P.dir);
    load_lines<kMfmaThreads, (1 << kMaxLogT) / kMfmaThreads>(lds, P, T, wg);
    __syncthreads();
    plan_last_level<M0>(lds, lds_f, P, T, level_geom(M0, 0, 0, 0), wg);
  } else {
    constexpr int TPW0 = 1 << (LT - M0 - 8);
    const LevelGeom g0 = level_geom(M0, 0, M1 + M2, M1);
    if (P.coset_pre == 0) {
      // the first level reads its fragments from HBM
      PlanStage<M0, M1, M2> st;
      st.dst = lds_f;
      st.on = stage;
      st.load(T, P.dir);
      mfma_level<M0, TPW0, 1, true>(lds, lds_f, P, T, g0, false, wg, st);
    } else {
      // the coset pre-scale is applied while the tile is staged in LDS
      if (stage) {
        stage_bat<M0, kMfmaThreads>(lds_f, T, P.dir);
        if constexpr (PL::kStage1) stage_bat<(M1 > 0 ? M1 : 1), kMfmaThreads>(lds_f + PL::kOff1, T, P.dir);
        if constexpr (PL::kStage2) stage_bat<(M2 > 0 ? M2 : 1), kMfmaThreads>(lds_f + PL::kOff2, T, P.dir);
      }
      load_lines<kMfmaThreads, (1 << kMaxLogT) / kMfmaThreads>(lds, P, T, wg);
      __syncthreads();
      mfma_level<M0, TPW0, 1>(lds, lds_f, P, T, g0, false, wg);
    }
    if constexpr (M2 > 0) {
      mfma_level<M1, (1 << (LT - M1 - 8)), 1>(lds, lds_f + PL::kOff1, P, T, level_geom(M1, M0, M2, M2), false, wg);
      plan_last_level<M2>(lds, lds_f + PL::kOff2, P, T, level_geom(M2, M0 + M1, 0, 0), wg);
    } else {
      plan_last_level<M1>(lds, lds_f + PL::kOff1, P, T, level_geom(M1, M0, 0, 0), wg);
    }
  }
  // the last level has written the pass's outputs to HBM
}

// One pass on the butterfly engine with NT threads per workgroup.
template <int NT>
__device__ FRNTT_INLINE void run_pass_bfly(u32x4* lds, const PassParams& P, const DevTables& T, int64_t wg) {
  load_lines<NT, 2>(lds, P, T, wg);
  __syncthreads();
  bfly_stages<NT>(lds, P, T);
  store_lines<NT>(lds, P, T, wg);
}

// Plan kernels of the matrix form, one per level split of a 4096-element
// tile (each in a translation unit of its own, so that they compile in
// parallel), and the dispatcher that finds the one for a split.
// The first twelve are the splits of a pass radix 2^12 .. 2^1 into the
// fewest levels of at most 16, larger first; the last four are the other
// orders of the 2^10 and 2^11 splits. Three-level defaults start with the
// smallest radix (3,4,3 and 3,4,4); the autotuner may choose any order.
#define FRNTT_PLAN_KERNELS(X) \
  X(4, 4, 4) X(4, 4, 3) X(4, 3, 3) X(3, 3, 3) X(4, 4, 0) X(4, 3, 0) X(3, 3, 0) X(3, 2, 0) \
  X(4, 0, 0) X(3, 0, 0) X(2, 0, 0) X(1, 0, 0) X(3, 4, 3) X(3, 3, 4) X(3, 4, 4) X(4, 3, 4)
#define FRNTT_DECLARE_PLAN_KERNEL(a, b, c) __global__ void ntt_plan_kernel_##a##b##c(PassParams P, DevTables T);
FRNTT_PLAN_KERNELS(FRNTT_DECLARE_PLAN_KERNEL)
#define FRNTT_DEFINE_PLAN_KERNEL(a, b, c)                                                  \
  __global__ __launch_bounds__(kMfmaThreads) void ntt_plan_kernel_##a##b##c(PassParams P, DevTables T) { \
    __shared__ u32x4 lds[2 << kMaxLogT];                                                 \
    __shared__ i32x4 lds_f[PassPlan<a, b, c>::kLds];                                     \
    run_pass_plan<a, b, c>(lds, lds_f, P, T, logical_wg(P));                             \
  }

}  // namespace frntt
