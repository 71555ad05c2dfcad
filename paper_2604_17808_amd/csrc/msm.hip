// Multi-scalar multiplication sum_n S_n P_n over a twisted Edwards curve by
// the layout-stationary Pippenger method (the paper's Alg. 2, LS-PPG):
// Bucketize, Bucket Accumulation, a tree-form Bucket Reduction and Window
// Merging, each a launch (the reduction one launch per tree level).
//
// The curve is a x^2 + y^2 = 1 + d x^2 y^2 over Fr (BN254's scalar field),
// a = 168700, d = 168696 (Baby Jubjub). a is a square and d is not, so the
// unified addition law in extended coordinates (X : Y : Z : T), x = X/Z,
// y = Y/Z, T Z = X Y, has no exceptional cases (zero point (0 : 1 : 1 : 0),
// as in the paper). Coordinates are kept in Montgomery form (R = 2^261) and
// multiplied with the library's 29-bit-limb Montgomery product.
//
// Bucketize is a counting sort per window (histogram, exclusive scan, then
// scatter of point indices), which is the argsort of the paper's step; the
// order of indices inside a bucket is left free, since a bucket's sum does
// not depend on it. The paper's "layout stationary" point is kept: the
// sorted index lists are gathered once, and every bucket, window and tree
// level is a separate data-parallel axis of a launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr.hpp"
#include "frntt_internal.hpp"
#include "host_field.hpp"

namespace frntt {
namespace {

constexpr int kMsmThreads = 256;
constexpr int kScanThreads = 1024;
constexpr uint32_t kCurveA = 168700, kCurveD = 168696;

struct MsmConsts {
  fr_t r2;   // 2^522 mod r (into Montgomery form)
  fr_t one;  // 2^261 mod r
  fr_t a;    // a 2^261 mod r
  fr_t d;    // d 2^261 mod r
};

// extended coordinates, Montgomery form
struct ept {
  fr_t X, Y, Z, T;
};

__device__ FRNTT_INLINE fr_t load_fr(const u32x4* p) {
  const u32x4 lo = p[0], hi = p[1];
  fr_t x;
  x.w[0] = lo.x; x.w[1] = lo.y; x.w[2] = lo.z; x.w[3] = lo.w;
  x.w[4] = hi.x; x.w[5] = hi.y; x.w[6] = hi.z; x.w[7] = hi.w;
  return x;
}

__device__ FRNTT_INLINE void store_fr(u32x4* p, const fr_t& x) {
  p[0] = u32x4{x.w[0], x.w[1], x.w[2], x.w[3]};
  p[1] = u32x4{x.w[4], x.w[5], x.w[6], x.w[7]};
}

__device__ FRNTT_INLINE ept load_ept(const u32x4* p) {
  ept e;
  e.X = load_fr(p);
  e.Y = load_fr(p + 2);
  e.Z = load_fr(p + 4);
  e.T = load_fr(p + 6);
  return e;
}

__device__ FRNTT_INLINE void store_ept(u32x4* p, const ept& e) {
  store_fr(p, e.X);
  store_fr(p + 2, e.Y);
  store_fr(p + 4, e.Z);
  store_fr(p + 6, e.T);
}

__device__ FRNTT_INLINE ept ept_zero(const MsmConsts& C) {
  ept e;
  e.X = fr_zero();
  e.Y = C.one;
  e.Z = C.one;
  e.T = fr_zero();
  return e;
}

// P + (x2, y2) for an affine point given as x2, y2 and d x2 y2 (Montgomery
// form): the unified addition with Z2 = 1 (9 products).
__device__ FRNTT_INLINE ept add_mixed(const ept& P, const fr_t& x2, const fr_t& y2, const fr_t& dt2,
                                      const MsmConsts& C) {
  const fr_t A = mont_mul(P.X, x2);
  const fr_t B = mont_mul(P.Y, y2);
  const fr_t Cc = mont_mul(P.T, dt2);
  const fr_t E = fr_sub(fr_sub(mont_mul(fr_add(P.X, P.Y), fr_add(x2, y2)), A), B);
  const fr_t F = fr_sub(P.Z, Cc);
  const fr_t G = fr_add(P.Z, Cc);
  const fr_t H = fr_sub(B, mont_mul(C.a, A));
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// P + Q, the unified addition (11 products).
__device__ FRNTT_INLINE ept add_full(const ept& P, const ept& Q, const MsmConsts& C) {
  const fr_t A = mont_mul(P.X, Q.X);
  const fr_t B = mont_mul(P.Y, Q.Y);
  const fr_t Cc = mont_mul(mont_mul(P.T, Q.T), C.d);
  const fr_t D = mont_mul(P.Z, Q.Z);
  const fr_t E = fr_sub(fr_sub(mont_mul(fr_add(P.X, P.Y), fr_add(Q.X, Q.Y)), A), B);
  const fr_t F = fr_sub(D, Cc);
  const fr_t G = fr_add(D, Cc);
  const fr_t H = fr_sub(B, mont_mul(C.a, A));
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// 2 P, the doubling formula derived from the unified addition (it uses
// neither T nor d; 9 products): with A = X^2, B = Y^2, G = a A + B, the
// affine result is (2 x y / G, (B - a A) / (2 - G)) scaled by Z^2.
__device__ FRNTT_INLINE ept dbl(const ept& P, const MsmConsts& C) {
  const fr_t A = mont_mul(P.X, P.X);
  const fr_t B = mont_mul(P.Y, P.Y);
  const fr_t Z2 = mont_mul(P.Z, P.Z);
  const fr_t Cc = fr_add(Z2, Z2);
  const fr_t XY = fr_add(P.X, P.Y);
  const fr_t E = fr_sub(fr_sub(mont_mul(XY, XY), A), B);
  const fr_t Da = mont_mul(C.a, A);
  const fr_t G = fr_add(Da, B);
  const fr_t F = fr_sub(G, Cc);
  const fr_t H = fr_sub(Da, B);
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// c-bit digit k of a 256-bit scalar (zero beyond bit 255)
__device__ FRNTT_INLINE uint32_t window_digit(const uint32_t* s, int c, int k) {
  const int bit = c * k, wi = bit >> 5, sh = bit & 31;
  if (wi >= 8) return 0;
  uint32_t v = s[wi] >> sh;
  if (sh + c > 32 && wi + 1 < 8) v |= s[wi + 1] << (32 - sh);
  return v & ((1u << c) - 1);
}

__device__ FRNTT_INLINE void load_scalar(const u32x4* p, uint32_t* s) {
  const u32x4 lo = p[0], hi = p[1];
  s[0] = lo.x; s[1] = lo.y; s[2] = lo.z; s[3] = lo.w;
  s[4] = hi.x; s[5] = hi.y; s[6] = hi.z; s[7] = hi.w;
}

// ---- Bucketize ------------------------------------------------------------

// Points into Montgomery form with d x y beside them (96 bytes per point),
// and the histogram of every window's nonzero digits.
__global__ __launch_bounds__(kMsmThreads) void msm_prep_kernel(const u32x4* __restrict__ pts,
                                                               const u32x4* __restrict__ sc, int64_t n, int c,
                                                               int K, u32x4* __restrict__ prep,
                                                               uint32_t* __restrict__ counts, MsmConsts C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const fr_t xm = mont_mul(load_fr(pts + 4 * i), C.r2);
    const fr_t ym = mont_mul(load_fr(pts + 4 * i + 2), C.r2);
    const fr_t dt = mont_mul(mont_mul(xm, ym), C.d);
    store_fr(prep + 6 * i, xm);
    store_fr(prep + 6 * i + 2, ym);
    store_fr(prep + 6 * i + 4, dt);
    uint32_t s[8];
    load_scalar(sc + 2 * i, s);
    for (int k = 0; k < K; ++k) {
      const uint32_t dg = window_digit(s, c, k);
      if (dg) atomicAdd(counts + ((int64_t)k << c) + dg, 1u);
    }
  }
}

// Exclusive scan of one window's bucket counts (one workgroup per window):
// the start of each bucket's index list, and a copy the scatter advances.
__global__ __launch_bounds__(kScanThreads) void msm_scan_kernel(const uint32_t* __restrict__ counts,
                                                                uint32_t* __restrict__ start,
                                                                uint32_t* __restrict__ cursor, int c) {
  __shared__ uint32_t part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x << c;
  const int nb = 1 << c, per = (nb + kScanThreads - 1) / kScanThreads, t = threadIdx.x;
  const int lo = t * per, hi = lo + per < nb ? lo + per : nb;
  uint32_t s = 0;
  for (int j = lo; j < hi; ++j) s += counts[base + j];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t ? part[t - 1] : 0u;
  for (int j = lo; j < hi; ++j) {
    start[base + j] = run;
    cursor[base + j] = run;
    run += counts[base + j];
  }
}

// Each point's index into the list of its bucket in every window.
__global__ __launch_bounds__(kMsmThreads) void msm_scatter_kernel(const u32x4* __restrict__ sc, int64_t n, int c,
                                                                  int K, uint32_t* __restrict__ cursor,
                                                                  uint32_t* __restrict__ idx) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t s[8];
    load_scalar(sc + 2 * i, s);
    for (int k = 0; k < K; ++k) {
      const uint32_t dg = window_digit(s, c, k);
      if (dg) {
        const uint32_t pos = atomicAdd(cursor + ((int64_t)k << c) + dg, 1u);
        idx[(int64_t)k * n + pos] = (uint32_t)i;
      }
    }
  }
}

// ---- Bucket Accumulation --------------------------------------------------

// B_(k,j) = sum of the points in bucket (k, j); one bucket per thread. The
// first point of a bucket is taken as it is (T = x y), the rest are added.
__global__ __launch_bounds__(kMsmThreads) void msm_accum_kernel(const u32x4* __restrict__ prep,
                                                                const uint32_t* __restrict__ idx,
                                                                const uint32_t* __restrict__ start,
                                                                const uint32_t* __restrict__ counts, int64_t n,
                                                                int c, int K, u32x4* __restrict__ B, MsmConsts C) {
  const int64_t total = (int64_t)K << c;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cnt = counts[g];
    ept acc = ept_zero(C);
    if (cnt) {
      const uint32_t* list = idx + (g >> c) * n + start[g];
      const u32x4* p0 = prep + 6 * (int64_t)list[0];
      acc.X = load_fr(p0);
      acc.Y = load_fr(p0 + 2);
      acc.T = mont_mul(acc.X, acc.Y);
      for (uint32_t i = 1; i < cnt; ++i) {
        const u32x4* p = prep + 6 * (int64_t)list[i];
        acc = add_mixed(acc, load_fr(p), load_fr(p + 2), load_fr(p + 4), C);
      }
    }
    store_ept(B + 8 * g, acc);
  }
}

// ---- Bucket Reduction (tree form) -----------------------------------------

// One tree level: for the 2^s bucket pairs (2b, 2b + 1) of every window,
// W_b <- W_2b + W_(2b+1) + B_(2b+1) and B_b <- 2 (B_2b + B_(2b+1)).
// Entries of window k sit at k 2^c + index in every buffer. On the first
// level every W is zero; on the last one (s = 0) the new B is not needed.
__global__ __launch_bounds__(kMsmThreads) void msm_reduce_kernel(const u32x4* __restrict__ Bin,
                                                                 const u32x4* __restrict__ Win,
                                                                 u32x4* __restrict__ Bout,
                                                                 u32x4* __restrict__ Wout, int c, int K, int s,
                                                                 int first, MsmConsts C) {
  const int64_t total = (int64_t)K << s;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g >> s, b = g & ((1 << s) - 1);
    const int64_t l = (k << c) + 2 * b, o = (k << c) + b;
    const ept BR = load_ept(Bin + 8 * (l + 1));
    ept w = BR;
    if (!first) w = add_full(add_full(load_ept(Win + 8 * l), load_ept(Win + 8 * (l + 1)), C), BR, C);
    store_ept(Wout + 8 * o, w);
    if (s > 0) store_ept(Bout + 8 * o, dbl(add_full(load_ept(Bin + 8 * l), BR, C), C));
  }
}

// ---- Window Merging and the affine result ---------------------------------

__device__ FRNTT_INLINE bool words_is_one(const uint32_t* u) {
  uint32_t acc = u[0] ^ 1u;
#pragma unroll
  for (int i = 1; i < 8; ++i) acc |= u[i];
  return acc == 0;
}

__device__ FRNTT_INLINE bool words_is_zero(const uint32_t* u) {
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) acc |= u[i];
  return acc == 0;
}

__device__ FRNTT_INLINE void words_shr1(uint32_t* u) {
#pragma unroll
  for (int i = 0; i < 7; ++i) u[i] = (u[i] >> 1) | (u[i + 1] << 31);
  u[7] >>= 1;
}

// x / 2 mod r for x < r: x / 2, or (x + r) / 2 for odd x (x + r < 2^255)
__device__ FRNTT_INLINE void half_mod(uint32_t* x) {
  if (x[0] & 1u) {
    uint32_t cy = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = addc(x[i], fr_mod_word(i), cy, &cy);
  }
  words_shr1(x);
}

__device__ FRNTT_INLINE bool words_geq(const uint32_t* u, const uint32_t* v) {
  uint32_t br = 0, d;
#pragma unroll
  for (int i = 0; i < 8; ++i) d = subb(u[i], v[i], br, &br);
  (void)d;
  return br == 0;
}

__device__ FRNTT_INLINE void words_sub(uint32_t* u, const uint32_t* v) {
  uint32_t br = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) u[i] = subb(u[i], v[i], br, &br);
}

// a^-1 mod r for 0 < a < r by the binary extended Euclidean algorithm
// (invariants u = x1 a, v = x2 a mod r; every pass halves u or v or
// subtracts the smaller from the larger). Zero maps to zero. The pass count
// is bounded, so the loop ends on any input.
__device__ fr_t fr_inverse(const fr_t& a) {
  uint32_t u[8], v[8], x1[8], x2[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    u[i] = a.w[i];
    v[i] = fr_mod_word(i);
    x1[i] = i == 0 ? 1u : 0u;
    x2[i] = 0;
  }
  fr_t o = fr_zero();
  if (words_is_zero(u)) return o;
  for (int it = 0; it < 2048 && !words_is_one(u) && !words_is_one(v); ++it) {
    while (!(u[0] & 1u) && !words_is_zero(u)) {
      words_shr1(u);
      half_mod(x1);
    }
    while (!(v[0] & 1u) && !words_is_zero(v)) {
      words_shr1(v);
      half_mod(x2);
    }
    fr_t f1, f2;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      f1.w[i] = x1[i];
      f2.w[i] = x2[i];
    }
    if (words_geq(u, v)) {
      words_sub(u, v);
      const fr_t t = fr_sub(f1, f2);
#pragma unroll
      for (int i = 0; i < 8; ++i) x1[i] = t.w[i];
    } else {
      words_sub(v, u);
      const fr_t t = fr_sub(f2, f1);
#pragma unroll
      for (int i = 0; i < 8; ++i) x2[i] = t.w[i];
    }
  }
  const bool one_u = words_is_one(u);
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = one_u ? x1[i] : x2[i];
  return o;
}

// MSM = sum_k 2^(c k) W_k from the top window down, then (x, y) = (X/Z, Y/Z)
// in canonical form: out[0..7] = x, out[8..15] = y.
__global__ __launch_bounds__(64) void msm_merge_kernel(const u32x4* __restrict__ W, int c, int K,
                                                       uint32_t* __restrict__ out, MsmConsts C) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  ept acc = ept_zero(C);
  for (int k = K - 1; k >= 0; --k) {
    if (k != K - 1)
      for (int i = 0; i < c; ++i) acc = dbl(acc, C);
    acc = add_full(acc, load_ept(W + 8 * ((int64_t)k << c)), C);
  }
  fr_t one_c = fr_zero();
  one_c.w[0] = 1;
  const fr_t zi = fr_inverse(mont_mul(acc.Z, one_c));
  const fr_t x = mont_mul(acc.X, zi), y = mont_mul(acc.Y, zi);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    out[i] = x.w[i];
    out[8 + i] = y.w[i];
  }
}

// ---- batch scalar multiplication ------------------------------------------

// out_i = S_i P_i in affine form (out: x then y, 16 words per point), by
// left-to-right double-and-add over the 256 scalar bits.
__global__ __launch_bounds__(kMsmThreads) void ec_mul_kernel(const u32x4* __restrict__ sc,
                                                             const u32x4* __restrict__ pts, int64_t n,
                                                             u32x4* __restrict__ out, MsmConsts C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const fr_t xm = mont_mul(load_fr(pts + 4 * i), C.r2);
    const fr_t ym = mont_mul(load_fr(pts + 4 * i + 2), C.r2);
    const fr_t dt = mont_mul(mont_mul(xm, ym), C.d);
    uint32_t s[8];
    load_scalar(sc + 2 * i, s);
    ept acc = ept_zero(C);
    for (int b = 255; b >= 0; --b) {
      acc = dbl(acc, C);
      if ((s[b >> 5] >> (b & 31)) & 1u) acc = add_mixed(acc, xm, ym, dt, C);
    }
    fr_t one_c = fr_zero();
    one_c.w[0] = 1;
    const fr_t zi = fr_inverse(mont_mul(acc.Z, one_c));
    store_fr(out + 4 * i, mont_mul(acc.X, zi));
    store_fr(out + 4 * i + 2, mont_mul(acc.Y, zi));
  }
}

// ---- host side -------------------------------------------------------------

void fe_words(const host::Fe& a, fr_t* o) {
  for (int i = 0; i < 4; ++i) {
    o->w[2 * i] = (uint32_t)a.v[i];
    o->w[2 * i + 1] = (uint32_t)(a.v[i] >> 32);
  }
}

// x 2^k mod r by k modular doublings
host::Fe times_pow2(host::Fe x, int k) {
  for (int i = 0; i < k; ++i) x = host::add(x, x);
  return x;
}

MsmConsts make_consts() {
  MsmConsts C;
  fe_words(times_pow2(host::from_u64(1), 522), &C.r2);
  fe_words(times_pow2(host::from_u64(1), 261), &C.one);
  fe_words(times_pow2(host::from_u64(kCurveA), 261), &C.a);
  fe_words(times_pow2(host::from_u64(kCurveD), 261), &C.d);
  return C;
}

struct MsmDeviceGuard {
  int prev = -1;
  explicit MsmDeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~MsmDeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

constexpr int kMsmMaxWindow = 20;
constexpr int64_t kMsmMaxPoints = (int64_t)1 << 28;

int windows_for(int c) { return (256 + c - 1) / c; }

// Workspace: prepared points, counts, starts, cursors, index lists, and two
// (B, W) buffer pairs of K 2^c extended points.
size_t msm_workspace_bytes(int64_t n, int c) {
  const size_t K = (size_t)windows_for(c), nb = K << c;
  const size_t prep = (size_t)n * 96, cnt = nb * 4 * 3, idx = K * (size_t)n * 4, pts = nb * 128 * 4;
  const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return up(prep) + up(cnt) + up(idx) + up(pts);
}

int grid_of(const frntt_ctx* ctx, int64_t items, bool capped) {
  int64_t g = (items + kMsmThreads - 1) / kMsmThreads;
  if (g < 1) g = 1;
  const int64_t cap = capped ? (int64_t)ctx->cu_count * 8 : (int64_t)1 << 30;
  return (int)(g < cap ? g : cap);
}

int msm_status(frntt_ctx* ctx) {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? FRNTT_OK : set_hip_error(ctx, e);
}

}  // namespace
}  // namespace frntt

using namespace frntt;

extern "C" {

int frntt_msm_window(int64_t n) {
  if (n < 0) return FRNTT_EINVAL;
  // cost model: K (n + 5 2^c) point additions (accumulation, then about four
  // additions per bucket in the tree reduction)
  int best = 1;
  double best_cost = 0;
  for (int c = 1; c <= kMsmMaxWindow; ++c) {
    const double cost = (double)windows_for(c) * ((double)n + 5.0 * (double)(1 << c));
    if (c == 1 || cost < best_cost) {
      best = c;
      best_cost = cost;
    }
  }
  return best;
}

size_t frntt_msm_workspace_bytes(int64_t n, int window) {
  if (n < 0 || n > kMsmMaxPoints) return 0;
  const int c = window ? window : frntt_msm_window(n);
  if (c < 1 || c > kMsmMaxWindow) return 0;
  return msm_workspace_bytes(n, c);
}

int frntt_msm(frntt_ctx* ctx, const void* scalars, const void* points, int64_t n, int window, void* out,
              void* stream) {
  if (!ctx || !out || n < 0 || (n > 0 && (!scalars || !points))) return FRNTT_EINVAL;
  if (n > kMsmMaxPoints || window < 0 || window > kMsmMaxWindow) return FRNTT_ERANGE;
  if ((((uintptr_t)scalars | (uintptr_t)points) & 15) != 0) return FRNTT_EALIGN;
  const int c = window ? window : frntt_msm_window(n);
  const int K = n ? windows_for(c) : 0;
  const hipStream_t st = (hipStream_t)stream;
  MsmDeviceGuard guard(ctx->device);
  static const MsmConsts C = make_consts();
  if (n == 0) {
    msm_merge_kernel<<<1, 64, 0, st>>>(nullptr, c, 0, (uint32_t*)out, C);
    return msm_status(ctx);
  }
  const int64_t nb = (int64_t)K << c;
  void* ws = nullptr;
  int rc = get_scratch(ctx, st, msm_workspace_bytes(n, c), &ws);
  if (rc != FRNTT_OK) return rc;
  const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* p = (char*)ws;
  u32x4* prep = (u32x4*)p;
  p += up((size_t)n * 96);
  uint32_t* counts = (uint32_t*)p;
  uint32_t* start = counts + nb;
  uint32_t* cursor = start + nb;
  p += up((size_t)nb * 12);
  uint32_t* idx = (uint32_t*)p;
  p += up((size_t)K * n * 4);
  u32x4* B0 = (u32x4*)p;
  u32x4* W0 = B0 + 8 * nb;
  u32x4* B1 = W0 + 8 * nb;
  u32x4* W1 = B1 + 8 * nb;

  zero_words_kernel<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(counts, nb);
  msm_prep_kernel<<<grid_of(ctx, n, true), kMsmThreads, 0, st>>>((const u32x4*)points, (const u32x4*)scalars, n,
                                                                  c, K, prep, counts, C);
  msm_scan_kernel<<<K, kScanThreads, 0, st>>>(counts, start, cursor, c);
  msm_scatter_kernel<<<grid_of(ctx, n, true), kMsmThreads, 0, st>>>((const u32x4*)scalars, n, c, K, cursor, idx);
  msm_accum_kernel<<<grid_of(ctx, nb, false), kMsmThreads, 0, st>>>(prep, idx, start, counts, n, c, K, B0, C);
  u32x4 *bi = B0, *wi = W0, *bo = B1, *wo = W1;
  for (int s = c - 1; s >= 0; --s) {
    msm_reduce_kernel<<<grid_of(ctx, (int64_t)K << s, false), kMsmThreads, 0, st>>>(bi, wi, bo, wo, c, K, s,
                                                                                   s == c - 1, C);
    u32x4* t = bi;
    bi = bo;
    bo = t;
    t = wi;
    wi = wo;
    wo = t;
  }
  msm_merge_kernel<<<1, 64, 0, st>>>(wi, c, K, (uint32_t*)out, C);
  return msm_status(ctx);
}

int frntt_ec_mul(frntt_ctx* ctx, const void* scalars, const void* points, int64_t n, void* out, void* stream) {
  if (!ctx || n < 0 || (n > 0 && (!scalars || !points || !out))) return FRNTT_EINVAL;
  if (n > kMsmMaxPoints) return FRNTT_ERANGE;
  if ((((uintptr_t)scalars | (uintptr_t)points | (uintptr_t)out) & 15) != 0) return FRNTT_EALIGN;
  if (n == 0) return FRNTT_OK;
  MsmDeviceGuard guard(ctx->device);
  static const MsmConsts C = make_consts();
  ec_mul_kernel<<<grid_of(ctx, n, false), kMsmThreads, 0, (hipStream_t)stream>>>(
      (const u32x4*)scalars, (const u32x4*)points, n, (u32x4*)out, C);
  return msm_status(ctx);
}

}  // extern "C"
