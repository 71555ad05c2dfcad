// Device-side structures shared by the transform kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr.hpp"

namespace frntt {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

constexpr int kMaxLogT = 12;           // elements staged per workgroup: 2^12 x 32 B = 128 KiB
// Threads per workgroup. The butterfly engine runs 16 waves (4 per SIMD, at
// most 128 registers each); the MFMA engine runs 8 waves, whose 256-register
// budget holds a level's data fragments and constant blocks together.
constexpr int kBflyThreads = 1024;
constexpr int kMfmaThreads = 512;
constexpr int kMfmaWaves = kMfmaThreads / 64;
constexpr int kMaxLevels = 6;
constexpr int kMasterLog = 28;         // two-adicity of r
constexpr int kSplit = 14;             // master twiddle exponent split 14 + 14 bits

// Device constant tables built at context creation. Field elements are 32 B
// (two u32x4); "mont" marks Montgomery form (value * 2^261 mod r).
struct DevTables {
  const u32x4* tw_lo[2];      // [dir] mont w28^(+-j), j < 2^14            (w28 = w_{2^28})
  const u32x4* tw_hi[2];      // [dir] mont w28^(+-(2^14 j)), j < 2^14
  const u32x4* w4096[2];      // [dir] mont w_4096^(+-j), j < 4096
  const u32x4* w4096_s[2];    // [dir] w_4096^(+-j) (not Montgomery) in the Shoup operand form:
                              // 10 limbs of floor(w 2^290 / r), 9 limbs of w (5 x 16 B per entry)
  const u32x4* g_lo[2];       // [0] mont g^j, [1] mont g^-j, j < 2^14 (g = 5)
  const u32x4* g_hi[2];       // [0] mont g^(2^14 j), [1] g^-(2^14 j)
  const u32x4* ninv;          // mont 2^-L for L = 0..28
  const i32x4* bat[2][6];     // [dir][log rho] rho blocks x 64 lanes x 16 B of signed digits
  const i32x4* bat_init[2][6];// [dir][log rho] rho x 2 halves x 16 int32 accumulator seeds
  // 2^8, 2^16, 2^24 and 1: the byte-plane weights of the carry merge, passed
  // as kernel arguments so that the word sums stay 32x32+64-bit multiply-adds
  // (which overlap with MFMA) instead of becoming 64-bit shift-adds
  uint32_t byte_w[4];
};

// One HBM pass of the multi-pass transform.
struct PassParams {
  const u32x4* src;
  u32x4* dst;
  int64_t wg_count;
  int log_n;        // log2 polynomial size L
  int log_r;        // log2 radix of this pass l_p
  int log_s;        // log2 of the stride of the pass axis S_p (0 for the last pass)
  int log_d;        // D_p = sum of earlier pass radices
  int log_g;        // log2 lines per workgroup
  int log_t;        // log_r + log_g (elements per workgroup)
  int is_last;
  int n_pass;       // number of passes P
  int pass_log[4];  // all pass radices, in order
  int nlev;         // levels inside this pass
  int lev_log[kMaxLevels];
  int engine;       // 0: butterfly stages, 1: MFMA levels (lev_log)
  int dir;          // 0: forward roots, 1: inverse roots
  int coset_pre;    // first pass of a coset transform: x_n *= g^n on load; 1: g^n from the
                   // split tables; 2: g^(j 2^log_s) for line element j from the tail of the
                   // pass table, whose entries carry the line's g^rest
  int post;         // last pass: 0 none, 1 scale by N^-1, 2 scale by N^-1 g^-k, 3 scale by g^-k
                   // (2^-log_n then rides in the first pass's twiddle table), 4 scale by
                   // post_tw[K >> log_d] = g^-(K - K mod 2^log_d) (N^-1 g^-(K mod 2^log_d)
                   // ride in the first pass's table; two-pass plans)
  int xcd_remap;    // map consecutive logical workgroups onto one XCD
  const u32x4* pass_tw;  // non-last pass: table of its twiddles at [k][rest], or nullptr
  const u32x4* post_tw;  // last pass with post 4: factor of output K at [K >> log_d]
};

// Descriptor tables of one persistent batch launch (see ntt_batch_kernel).
struct BatchParams {
  const PassParams* passes;   // all passes of all jobs
  const int64_t* item_pass;   // pass of each work item, items ordered stage by stage
  const int64_t* item_wg;     // first workgroup (tile) of each item inside its pass
  const int* item_cnt;        // consecutive workgroups (tiles) of each item
  int64_t item_begin;         // this launch's items: [item_begin, item_end)
  int64_t item_end;
  unsigned int* queue;        // this launch's next item (zeroed before the launches)
  const DevTables* tables;    // the context's tables (a copy in the batch buffer)
};

// Specialised MFMA pass kernel for a 4096-element tile with these levels, or
// nullptr (then the generic kernel runs).
typedef void (*MfmaPassKernel)(PassParams, DevTables);
MfmaPassKernel mfma_plan_kernel(int nlev, const int* lev);

// ---- element access -------------------------------------------------------

__device__ FRNTT_INLINE fr_t ld_elem(const u32x4* p, int64_t e) {
  u32x4 a = p[2 * e], b = p[2 * e + 1];
  fr_t x;
  x.w[0] = a.x; x.w[1] = a.y; x.w[2] = a.z; x.w[3] = a.w;
  x.w[4] = b.x; x.w[5] = b.y; x.w[6] = b.z; x.w[7] = b.w;
  return x;
}

__device__ FRNTT_INLINE void st_elem(u32x4* p, int64_t e, const fr_t& x) {
  u32x4 a = {x.w[0], x.w[1], x.w[2], x.w[3]};
  u32x4 b = {x.w[4], x.w[5], x.w[6], x.w[7]};
  p[2 * e] = a;
  p[2 * e + 1] = b;
}

__device__ FRNTT_INLINE void st_elem_nt(u32x4* p, int64_t e, const fr_t& x) {
  u32x4 a = {x.w[0], x.w[1], x.w[2], x.w[3]};
  u32x4 b = {x.w[4], x.w[5], x.w[6], x.w[7]};
  __builtin_nontemporal_store(a, p + 2 * e);
  __builtin_nontemporal_store(b, p + 2 * e + 1);
}

// ---- twiddles -----------------------------------------------------------

// Montgomery form of w28^E (E < 2^28) from the split master tables.
__device__ FRNTT_INLINE fr_t master_tw(const DevTables& T, int dir, uint32_t E) {
  fr_t lo = ld_elem(T.tw_lo[dir], E & ((1u << kSplit) - 1));
  fr_t hi = ld_elem(T.tw_hi[dir], E >> kSplit);
  return mont_mul(lo, hi);
}

// Montgomery form of w_{2^log_m}^e (any e; reduced mod 2^log_m).
__device__ FRNTT_INLINE fr_t pow_tw(const DevTables& T, int dir, int log_m, uint64_t e) {
  uint32_t E = (uint32_t)((e << (kMasterLog - log_m)) & ((1u << kMasterLog) - 1));
  return master_tw(T, dir, E);
}

// Montgomery form of w_R^e for R = 2^log_r <= 4096 (e reduced mod R).
__device__ FRNTT_INLINE fr_t small_tw(const DevTables& T, int dir, int log_r, uint32_t e) {
  uint32_t idx = (e & ((1u << log_r) - 1)) << (12 - log_r);
  return ld_elem(T.w4096[dir], idx);
}

// The same twiddle w_R^e (plain, not Montgomery) in the operand form of the
// Shoup product: wp = the ten 29-bit limbs of floor(w 2^290 / r), w = the
// nine limbs of w.
__device__ FRNTT_INLINE void small_tw_shoup(const DevTables& T, int dir, int log_r, uint32_t e, uint32_t* wp,
                                            uint32_t* w) {
  const uint32_t idx = (e & ((1u << log_r) - 1)) << (12 - log_r);
  const u32x4* p = T.w4096_s[dir] + 5 * idx;
  const u32x4 a = p[0], b = p[1], c = p[2], d = p[3], f = p[4];
  wp[0] = a.x; wp[1] = a.y; wp[2] = a.z; wp[3] = a.w;
  wp[4] = b.x; wp[5] = b.y; wp[6] = b.z; wp[7] = b.w;
  wp[8] = c.x; wp[9] = c.y;
  w[0] = c.z; w[1] = c.w;
  w[2] = d.x; w[3] = d.y; w[4] = d.z; w[5] = d.w;
  w[6] = f.x; w[7] = f.y; w[8] = f.z;
}

// Montgomery form of g^(+-i) (i < 2^28).
__device__ FRNTT_INLINE fr_t coset_pow(const DevTables& T, int inv, uint32_t i) {
  fr_t lo = ld_elem(T.g_lo[inv], i & ((1u << kSplit) - 1));
  fr_t hi = ld_elem(T.g_hi[inv], i >> kSplit);
  return mont_mul(lo, hi);
}

// ---- pass geometry --------------------------------------------------------

__device__ FRNTT_INLINE int64_t logical_wg(const PassParams& P) {
  int64_t b = blockIdx.x;
  if (P.xcd_remap && (P.wg_count & 7) == 0) {
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // range of logical workgroups so neighbouring lines share its L2
    int64_t per = P.wg_count >> 3;
    b = (b & 7) * per + (b >> 3);
  }
  return b;
}

// Digits k_1..k_{P-1} of the output base `ob` (k_1 least significant) laid
// out as they sit in the last pass's input (k_1 most significant).
__device__ FRNTT_INLINE int64_t digit_reverse(const PassParams& P, int64_t ob) {
  // at most three earlier passes; a pass beyond the plan contributes no digit
  // (straight-line code, so that callers can keep many elements in flight)
  int64_t kp = 0;
  int d = 0;
  int s = P.log_n - P.pass_log[P.n_pass - 1];  // bits of kp
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int l = q < P.n_pass - 1 ? P.pass_log[q] : 0;
    const int64_t k = (ob >> d) & ((1ll << l) - 1);
    s -= l;
    kp |= k << s;
    d += l;
  }
  return kp;
}

// Element index (in the whole buffer) of input n of pass line `line`.
struct LineMap {
  int64_t in_base;   // element index of n = 0
  int64_t out_base;  // element index of k = 0
  int in_shift;      // log2 stride along n
  int out_shift;     // log2 stride along k
  int64_t rest;      // non-last pass: position inside the sub-problem (twiddle)
  int64_t poly_off;  // last pass: offset of k = 0 inside its polynomial
};

// Element index of input n = 0 of a line: a non-last pass (STRIDED) or the
// last pass.
template <bool STRIDED>
__device__ FRNTT_INLINE int64_t line_in_base(const PassParams& P, int64_t line) {
  if constexpr (STRIDED) {
    const int64_t hi = line >> P.log_s;
    const int64_t rest = line & ((1ll << P.log_s) - 1);
    return (hi << (P.log_r + P.log_s)) | rest;
  } else {
    const int64_t poly = line >> P.log_d;
    const int64_t ob = line & ((1ll << P.log_d) - 1);
    const int64_t kp = P.n_pass > 1 ? digit_reverse(P, ob) : 0;
    return (poly << P.log_n) + (kp << P.log_r);
  }
}

__device__ FRNTT_INLINE LineMap map_line(const PassParams& P, int64_t line) {
  LineMap m;
  if (!P.is_last) {
    int64_t rest = line & ((1ll << P.log_s) - 1);
    int64_t base = line_in_base<true>(P, line);
    m.in_base = base;
    m.out_base = base;
    m.in_shift = P.log_s;
    m.out_shift = P.log_s;
    m.rest = rest;
    m.poly_off = 0;
  } else {
    int64_t poly = line >> P.log_d;
    int64_t ob = line & ((1ll << P.log_d) - 1);
    m.in_base = line_in_base<false>(P, line);
    m.out_base = (poly << P.log_n) + ob;
    m.in_shift = 0;
    m.out_shift = P.log_d;
    m.rest = 0;
    m.poly_off = ob;
  }
  return m;
}

}  // namespace frntt
