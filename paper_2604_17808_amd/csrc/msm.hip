// Multi-scalar multiplication sum_n S_n P_n over a twisted Edwards curve by
// the layout-stationary Pippenger method (the paper's Alg. 2, LS-PPG):
// Bucketize, Bucket Accumulation, a tree-form Bucket Reduction and Window
// Merging, each a launch (the reduction one launch per tree level).
//
// The curve is a x^2 + y^2 = 1 + d x^2 y^2 over Fr (BN254's scalar field),
// a = 168700, d = 168696 (Baby Jubjub). Inside, points live on the
// isomorphic curve -x'^2 + y^2 = 1 + d' x'^2 y^2 with x' = s x, s^2 = -a,
// d' = -d / a (-1 and a are squares mod r, so s exists; d' is a non-square
// like d), where the extended-coordinate formulas of Hisil, Wong, Carter and
// Dawson (2008) for a = -1 are cheapest and complete: (X : Y : Z : T),
// x' = X/Z, y = Y/Z, T Z = X Y, zero point (0 : 1 : 1 : 0) as in the paper.
// Coordinates are kept in Montgomery form (R = 2^261) and multiplied with the
// library's 29-bit-limb Montgomery product.
//
// Bucketize is one stable radix sort of every window's digits (the argsort
// of the paper's step); the order of points inside a bucket is free, since
// a bucket's sum does not depend on it. The dataflow is the paper's layout-
// stationary one: the accumulation reads each point through the sorted
// entries, and no presorted copy of the points is written to HBM (the
// Presort-PPG baseline, which writes one, is kept beside it for comparison).
// Every bucket, window and tree level is a data-parallel axis of a launch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fr.hpp"
#include "frntt_internal.hpp"
#include "host_field.hpp"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include <mutex>

namespace frntt {
namespace {

constexpr int kMsmThreads = 256;
constexpr int kPrepStride = 8;  // u32x4 per prepared point (96 bytes used of 128)
constexpr uint32_t kCurveA = 168700, kCurveD = 168696;

struct MsmConsts {
  fr_t r2;    // 2^522 mod r (into Montgomery form)
  fr_t one;   // 2^261 mod r
  fr_t s;     // s = sqrt(-a), Montgomery form
  fr_t sinv;  // s^-1, Montgomery form
  fr_t k;     // 2 d' = -2 d / a, Montgomery form
  fr_t r2s;   // s 2^522 mod r: x -> x s in Montgomery form, one product
  fr_t r3sk;  // 2 d' s 2^783 mod r: (x y 2^-261) -> 2 d' s x y in Montgomery form
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

// x / 2 mod r for canonical x: x / 2, or (x + r) / 2 for odd x (x + r < 2^255)
__device__ FRNTT_INLINE fr_t fr_half(const fr_t& a) {
  fr_t x = a;
  if (x.w[0] & 1u) {
    uint32_t cy = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) x.w[i] = addc(x.w[i], fr_mod_word(i), cy, &cy);
  }
#pragma unroll
  for (int i = 0; i < 7; ++i) x.w[i] = (x.w[i] >> 1) | (x.w[i + 1] << 31);
  x.w[7] >>= 1;
  return x;
}

// P + Q for Q = (x2', y2) affine, given as y2 - x2', y2 + x2' and 2 d' x2' y2
// (the mixed addition with Z2 = 1: 7 products).
__device__ FRNTT_INLINE ept add_mixed(const ept& P, const fr_t& ymx2, const fr_t& ypx2, const fr_t& kt2,
                                      const MsmConsts& C) {
  const fr_t A = mont_mul(fr_sub(P.Y, P.X), ymx2);
  const fr_t B = mont_mul(fr_add(P.Y, P.X), ypx2);
  const fr_t Cc = mont_mul(P.T, kt2);
  const fr_t D = fr_add(P.Z, P.Z);
  const fr_t E = fr_sub(B, A), F = fr_sub(D, Cc), G = fr_add(D, Cc), H = fr_add(B, A);
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// P + Q, the unified addition (9 products).
__device__ FRNTT_INLINE ept add_full(const ept& P, const ept& Q, const MsmConsts& C) {
  const fr_t A = mont_mul(fr_sub(P.Y, P.X), fr_sub(Q.Y, Q.X));
  const fr_t B = mont_mul(fr_add(P.Y, P.X), fr_add(Q.Y, Q.X));
  const fr_t Cc = mont_mul(mont_mul(P.T, Q.T), C.k);
  const fr_t ZZ = mont_mul(P.Z, Q.Z);
  const fr_t D = fr_add(ZZ, ZZ);
  const fr_t E = fr_sub(B, A), F = fr_sub(D, Cc), G = fr_add(D, Cc), H = fr_add(B, A);
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// 2 P (8 products; uses neither T nor d'): with A = X^2, B = Y^2 and the
// curve's -1, the affine result is (2 x' y / (B - A), (-A - B) / (B - A - 2))
// scaled by Z^2.
__device__ FRNTT_INLINE ept dbl(const ept& P, const MsmConsts& C) {
  const fr_t A = mont_mul(P.X, P.X);
  const fr_t B = mont_mul(P.Y, P.Y);
  const fr_t Z2 = mont_mul(P.Z, P.Z);
  const fr_t XY = fr_add(P.X, P.Y);
  const fr_t E = fr_sub(fr_sub(mont_mul(XY, XY), A), B);
  const fr_t G = fr_sub(B, A);
  const fr_t F = fr_sub(G, fr_add(Z2, Z2));
  const fr_t H = fr_sub(fr_zero(), fr_add(A, B));
  ept o;
  o.X = mont_mul(E, F);
  o.Y = mont_mul(G, H);
  o.Z = mont_mul(F, G);
  o.T = mont_mul(E, H);
  return o;
}

// The extended point of a prepared one: x' = ((y + x') - (y - x')) / 2,
// y = ((y + x') + (y - x')) / 2, Z = 1, T = x' y (one product).
__device__ FRNTT_INLINE ept from_prepared(const fr_t& ymx, const fr_t& ypx, const MsmConsts& C) {
  ept e;
  e.X = fr_half(fr_sub(ypx, ymx));
  e.Y = fr_half(fr_add(ypx, ymx));
  e.Z = C.one;
  e.T = mont_mul(e.X, e.Y);
  return e;
}

// Prepared form of an affine input point (x, y): y - x', y + x', 2 d' x' y
// in Montgomery form (x' = s x).
__device__ FRNTT_INLINE void prepare_point(const u32x4* in, fr_t* ymx, fr_t* ypx, fr_t* kt, const MsmConsts& C) {
  const fr_t x = load_fr(in), y = load_fr(in + 2);
  const fr_t xp = mont_mul(x, C.r2s);
  const fr_t ym = mont_mul(y, C.r2);
  *ymx = fr_sub(ym, xp);
  *ypx = fr_add(ym, xp);
  *kt = mont_mul(mont_mul(x, y), C.r3sk);
}

// Affine (x, y) = (X / (s Z), Y / Z) in canonical form
__device__ fr_t fr_inverse(const fr_t& a);
__device__ FRNTT_INLINE void to_affine(const ept& P, const MsmConsts& C, fr_t* x, fr_t* y) {
  fr_t one_c = fr_zero();
  one_c.w[0] = 1;
  const fr_t zi = fr_inverse(mont_mul(P.Z, one_c));
  *x = mont_mul(mont_mul(P.X, zi), C.sinv);
  *y = mont_mul(P.Y, zi);
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
//
// The argsort of every window's digits is one stable radix sort of all
// windows' entries (rocPRIM's device radix sort), with each entry's
// position k n + i as its value. For c <= 16 the key is the digit alone
// (two 8-bit passes): the input is window-major and the sort is stable, so
// the entries of bucket (k, digit) still form one run (runs of equal digits,
// split by window). For wider windows the key is k 2^c + digit, which takes
// no more passes than the digit alone, and the values are read from an
// array rather than a counting iterator (measured faster at those sizes).
// The runs are the bucket lists.
constexpr int kDigitOnlyMaxWindow = 16;

// Points into their prepared form (96 bytes in a 128-byte slot per point:
// a gather of one point then reads one 128-byte line, where 96-byte slots
// straddle two lines half the time), and the sort keys:
// digit k of point i (or k 2^c + digit) at k n + i, with the value k n + i
// written beside it when vals is not null. Digit-only keys (c <= 16) are
// 16-bit words, which trims the radix sort's traffic.
template <typename KeyT>
__global__ __launch_bounds__(kMsmThreads) void msm_prep_kernel(const u32x4* __restrict__ pts,
                                                               const u32x4* __restrict__ sc, int64_t n, int c,
                                                               int K, u32x4* __restrict__ prep,
                                                               KeyT* __restrict__ keys,
                                                               uint32_t* __restrict__ vals, MsmConsts C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    fr_t ymx, ypx, kt;
    prepare_point(pts + 4 * i, &ymx, &ypx, &kt, C);
    store_fr(prep + kPrepStride * i, ymx);
    store_fr(prep + kPrepStride * i + 2, ypx);
    store_fr(prep + kPrepStride * i + 4, kt);
    uint32_t s[8];
    load_scalar(sc + 2 * i, s);
    for (int k = 0; k < K; ++k) {
      keys[(int64_t)k * n + i] = (KeyT)((c > kDigitOnlyMaxWindow ? (uint32_t)k << c : 0u) | window_digit(s, c, k));
      if (vals) vals[(int64_t)k * n + i] = (uint32_t)((int64_t)k * n + i);
    }
  }
}

// Run bounds of the sorted entries: first[g] = start of bucket g's run and
// last[g] = its end (both zero for buckets without entries). Each thread
// takes four consecutive entries per step: one aligned load per array (the
// workspace arrays start on 256-byte boundaries) plus the two
// neighbours, so a wave's loads cover whole lines and several are in
// flight per thread.
constexpr int kBoundsPerThread = 4;

// Bucket (k 2^c + digit) of a sorted entry: its key, or for digit-only keys
// the digit and the window of its value k n + i.
__device__ FRNTT_INLINE int64_t bucket_from(uint32_t key, uint32_t val, uint32_t n, int c) {
  if (c > kDigitOnlyMaxWindow) return key;
  return ((int64_t)(val / n) << c) | key;
}

// four keys from an aligned address
__device__ FRNTT_INLINE void load_keys4(const uint32_t* p, uint32_t* o) {
  const u32x4 v = *reinterpret_cast<const u32x4*>(p);
  o[0] = v.x;
  o[1] = v.y;
  o[2] = v.z;
  o[3] = v.w;
}
__device__ FRNTT_INLINE void load_keys4(const uint16_t* p, uint32_t* o) {
  typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
  const u32x2 v = *reinterpret_cast<const u32x2*>(p);
  o[0] = v.x & 0xffffu;
  o[1] = v.x >> 16;
  o[2] = v.y & 0xffffu;
  o[3] = v.y >> 16;
}

template <typename KeyT>
__global__ __launch_bounds__(kMsmThreads) void msm_bounds_kernel(const KeyT* __restrict__ keys,
                                                                 const uint32_t* __restrict__ vals, int64_t n,
                                                                 int c, int64_t total,
                                                                 uint32_t* __restrict__ first,
                                                                 uint32_t* __restrict__ last) {
  const uint32_t n32 = (uint32_t)n;
  const bool digit_only = c <= kDigitOnlyMaxWindow;
  const int64_t steps = (total + kBoundsPerThread - 1) / kBoundsPerThread;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < steps;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q0 = kBoundsPerThread * t;
    // entries q0 - 1 .. q0 + 4
    uint32_t kq[kBoundsPerThread + 2] = {}, vq[kBoundsPerThread + 2] = {};
    if (q0 + kBoundsPerThread <= total) {
      load_keys4(keys + q0, kq + 1);
      if (digit_only) {
        const u32x4 v4 = *reinterpret_cast<const u32x4*>(vals + q0);
        vq[1] = v4.x;
        vq[2] = v4.y;
        vq[3] = v4.z;
        vq[4] = v4.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kBoundsPerThread; ++j)
        if (q0 + j < total) {
          kq[1 + j] = keys[q0 + j];
          if (digit_only) vq[1 + j] = vals[q0 + j];
        }
    }
    if (q0 > 0) {
      kq[0] = keys[q0 - 1];
      if (digit_only) vq[0] = vals[q0 - 1];
    }
    if (q0 + kBoundsPerThread < total) {
      kq[kBoundsPerThread + 1] = keys[q0 + kBoundsPerThread];
      if (digit_only) vq[kBoundsPerThread + 1] = vals[q0 + kBoundsPerThread];
    }
    // their buckets; -1 outside [0, total)
    int64_t g[kBoundsPerThread + 2];
#pragma unroll
    for (int j = 0; j < kBoundsPerThread + 2; ++j) {
      const int64_t q = q0 - 1 + j;
      g[j] = (q >= 0 && q < total) ? bucket_from(kq[j], vq[j], n32, c) : -1;
    }
#pragma unroll
    for (int j = 1; j <= kBoundsPerThread; ++j) {
      const int64_t q = q0 - 1 + j;
      if (g[j] < 0) break;
      if (g[j - 1] != g[j]) first[g[j]] = (uint32_t)q;
      if (g[j + 1] != g[j]) last[g[j]] = (uint32_t)(q + 1);
    }
  }
}

// Bucket sizes and list starts; bucket 0 (digit zero) is left empty, since
// its points never reach the result.
__global__ __launch_bounds__(kMsmThreads) void msm_counts_kernel(uint32_t* __restrict__ first,
                                                                 const uint32_t* __restrict__ last,
                                                                 uint32_t* __restrict__ counts, int c, int K) {
  const int64_t total = (int64_t)K << c;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cnt = (g & ((1 << c) - 1)) ? last[g] - first[g] : 0u;
    counts[g] = cnt;
    if (!cnt) first[g] = 0u;
  }
}

// ---- Bucket Accumulation --------------------------------------------------
//
// A reduce-by-bucket in levels, so that no thread adds more than a fixed
// number of terms whatever the digit distribution (a bucket may hold every
// point, e.g. when all scalars are equal, or a third of them in a top window
// of two bits). Level 0 cuts each bucket's index list into chunks of kChunk0
// points and sums each chunk; every further level cuts each bucket's list of
// partial sums into chunks of kChunk; the last one sums each bucket's (at
// most kChunk) partials into B_(k,j). Chunks of window k sit at k CW + the
// exclusive scan of the bucket chunk counts, CW bounding a window's chunks.

// 16 points per thread measured best (2.5-3.5% ahead of 32, ahead of 8,
// 12, 24, 48 and 64 at 2^20 to 2^24 points): shorter chunks balance the
// waves better than the extra partial sums cost
constexpr int kChunk0 = 16, kChunk = 32;

// Item i of bucket j's list: a point (its prepared form,
// reached through the index list) or a partial sum.
struct PointItems {
  const u32x4* prep;
  const uint32_t* idx;    // sorted entries: k n + point index
  const uint32_t* start;  // bucket list starts in the sorted entries
  int64_t n;
};
// The same points already gathered into bucket order (the presorted layout
// of the Presort-PPG baseline), at the positions of the sorted entries.
struct SortedItems {
  const u32x4* pts;
  const uint32_t* start;
};
struct PartialItems {
  const u32x4* part;      // window k's partials at part + 8 k CW
  const uint32_t* base;   // bucket partial starts within the window
  int64_t cw;
};

// Sum of items [lo, hi) of bucket g (window k), hi > lo
__device__ FRNTT_INLINE ept sum_items(const PointItems& S, int64_t g, int64_t k, uint32_t lo, uint32_t hi,
                                      const MsmConsts& C) {
  const uint32_t* list = S.idx + S.start[g];
  const uint32_t off = (uint32_t)(k * S.n);
  const u32x4* p0 = S.prep + kPrepStride * (int64_t)(list[lo] - off);
  ept acc = from_prepared(load_fr(p0), load_fr(p0 + 2), C);
  for (uint32_t i = lo + 1; i < hi; ++i) {
    const u32x4* p = S.prep + kPrepStride * (int64_t)(list[i] - off);
    acc = add_mixed(acc, load_fr(p), load_fr(p + 2), load_fr(p + 4), C);
  }
  return acc;
}

__device__ FRNTT_INLINE ept sum_items(const SortedItems& S, int64_t g, int64_t k, uint32_t lo, uint32_t hi,
                                      const MsmConsts& C) {
  const u32x4* list = S.pts + 6 * (int64_t)S.start[g];
  const u32x4* p0 = list + 6 * (int64_t)lo;
  ept acc = from_prepared(load_fr(p0), load_fr(p0 + 2), C);
  for (uint32_t i = lo + 1; i < hi; ++i) {
    const u32x4* q = list + 6 * (int64_t)i;
    acc = add_mixed(acc, load_fr(q), load_fr(q + 2), load_fr(q + 4), C);
  }
  return acc;
}

__device__ FRNTT_INLINE ept sum_items(const PartialItems& S, int64_t g, int64_t k, uint32_t lo, uint32_t hi,
                                      const MsmConsts& C) {
  const u32x4* list = S.part + 8 * (k * S.cw + S.base[g]);
  ept acc = load_ept(list + 8 * (int64_t)lo);
  for (uint32_t i = lo + 1; i < hi; ++i) acc = add_full(acc, load_ept(list + 8 * (int64_t)i), C);
  return acc;
}

// Chunk counts of one level and their exclusive scan within each window, in
// tiles of kTile buckets: a tile-sum launch, then a launch in which every
// tile adds the sums of the window's earlier tiles to its own block scan.
// Level 0 cuts every bucket (ceil(m / len)); a later level only the buckets
// with more than len partials (the others are final after the level before).
constexpr int kTile = 1024, kTileThreads = 256;

__device__ FRNTT_INLINE uint32_t chunk_count(uint32_t m, int len, int heavy_only) {
  return heavy_only && m <= (uint32_t)len ? 0u : (m + (uint32_t)len - 1) / (uint32_t)len;
}

__device__ FRNTT_INLINE uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
  return v;
}

// sum over the block (kTileThreads threads), returned to every thread
__device__ FRNTT_INLINE uint32_t block_sum(uint32_t v, uint32_t* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kTileThreads / 64; ++i) r += lds[i];
  __syncthreads();
  return r;
}

// exclusive prefix over the block in thread order
__device__ FRNTT_INLINE uint32_t block_exclusive(uint32_t v, uint32_t* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)inc, off);
    if (lane >= off) inc += t;
  }
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  for (int i = 0; i < w; ++i) pre += lds[i];
  __syncthreads();
  return pre + inc - v;
}

__device__ FRNTT_INLINE int tiles_per_window(int c) { return c > 10 ? 1 << (c - 10) : 1; }

__global__ __launch_bounds__(kTileThreads) void msm_tile_sum_kernel(const uint32_t* __restrict__ m,
                                                                    uint32_t* __restrict__ tsum, int c, int len,
                                                                    int heavy_only) {
  __shared__ uint32_t lds[kTileThreads / 64];
  const int tiles = tiles_per_window(c), nb = 1 << c;
  const int64_t tile = blockIdx.x, k = tile / tiles;
  const int lo = (int)(tile - k * tiles) * kTile;
  uint32_t s = 0;
  for (int e = threadIdx.x; e < kTile && lo + e < nb; e += kTileThreads)
    s += chunk_count(m[(k << c) + lo + e], len, heavy_only);
  s = block_sum(s, lds);
  if (threadIdx.x == 0) tsum[tile] = s;
}

__global__ __launch_bounds__(kTileThreads) void msm_tile_scan_kernel(const uint32_t* __restrict__ m,
                                                                     const uint32_t* __restrict__ tsum,
                                                                     uint32_t* __restrict__ nch,
                                                                     uint32_t* __restrict__ base, int c, int len,
                                                                     int heavy_only) {
  __shared__ uint32_t lds[kTileThreads / 64];
  const int tiles = tiles_per_window(c), nb = 1 << c;
  const int64_t tile = blockIdx.x, k = tile / tiles, t = tile - k * tiles;
  const int lo = (int)t * kTile;
  uint32_t pre = 0;
  for (int64_t e = threadIdx.x; e < t; e += kTileThreads) pre += tsum[k * tiles + e];
  pre = block_sum(pre, lds);
  constexpr int kPer = kTile / kTileThreads;
  const int j0 = lo + kPer * threadIdx.x;
  uint32_t v[kPer], loc = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    v[q] = j0 + q < nb ? chunk_count(m[(k << c) + j0 + q], len, heavy_only) : 0u;
    loc += v[q];
  }
  uint32_t run = pre + block_exclusive(loc, lds);
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    if (j0 + q < nb) {
      base[(k << c) + j0 + q] = run;
      nch[(k << c) + j0 + q] = v[q];
      run += v[q];
    }
  }
}

// One level: chunk q of window k (thread per chunk slot) sums items
// [r len, min(r len + len, m_j)) of its bucket j, r = q - base_j.
template <class Items>
__global__ __launch_bounds__(kMsmThreads) void msm_chunk_kernel(Items S, const uint32_t* __restrict__ m_in,
                                                                const uint32_t* __restrict__ nch,
                                                                const uint32_t* __restrict__ base, int c, int K,
                                                                int len, int64_t cw_out,
                                                                u32x4* __restrict__ out, MsmConsts C) {
  const int64_t total = (int64_t)K * cw_out;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = g / cw_out, q = g - k * cw_out, w0 = k << c, last = w0 + (1 << c) - 1;
    if (q >= (int64_t)base[last] + nch[last]) continue;
    // the bucket whose chunks contain q: the last j with base_j <= q
    int64_t lo = w0, hi = last + 1;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)base[mid] <= q) lo = mid;
      else hi = mid;
    }
    const uint32_t r = (uint32_t)(q - base[lo]), first = r * (uint32_t)len;
    const uint32_t end = m_in[lo] - first < (uint32_t)len ? m_in[lo] : first + (uint32_t)len;
    store_ept(out + 8 * g, sum_items(S, lo, k, first, end, C));
  }
}

// Presort-PPG baseline: every window's points written out in bucket order
// (96 bytes per (window, point) pair) before the accumulation reads them.
__global__ __launch_bounds__(kMsmThreads) void msm_gather_kernel(const u32x4* __restrict__ prep,
                                                                 const uint32_t* __restrict__ idx, int64_t n,
                                                                 int64_t total, u32x4* __restrict__ sorted) {
  const uint32_t n32 = (uint32_t)n;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * blockDim.x) {
    const u32x4* src = prep + kPrepStride * (int64_t)(idx[p] % n32);
#pragma unroll
    for (int i = 0; i < 6; ++i) sorted[6 * p + i] = src[i];
  }
}

// Without chunk levels (n <= kChunk0): B_(k,j) = the sum of bucket j's
// points, or the zero point for an empty bucket; one bucket per thread.
template <class Items>
__global__ __launch_bounds__(kMsmThreads) void msm_bucket_points_kernel(Items S,
                                                                        const uint32_t* __restrict__ counts, int c,
                                                                        int K, u32x4* __restrict__ B, MsmConsts C) {
  const int64_t total = (int64_t)K << c;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cnt = counts[g];
    store_ept(B + 8 * g, cnt ? sum_items(S, g, g >> c, 0, cnt, C) : ept_zero(C));
  }
}

constexpr int kMaxChunkLevels = 8;

// The partial sums of every chunk level: level l's chunk counts and starts
// per bucket and its partials (window k at part + 8 k cw).
struct ChunkLevels {
  const u32x4* part[kMaxChunkLevels];
  const uint32_t* m[kMaxChunkLevels];
  const uint32_t* base[kMaxChunkLevels];
  int64_t cw[kMaxChunkLevels];
  int levels;
};

// B_(k,j) = the sum of bucket j's partials at the first level where they
// fit one chunk (level 0 for all but the buckets that are far above the
// mean size), or the zero point; one bucket per thread.
__global__ __launch_bounds__(kMsmThreads) void msm_bucket_final_kernel(ChunkLevels L, int c, int K,
                                                                       u32x4* __restrict__ B, MsmConsts C) {
  const int64_t total = (int64_t)K << c;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lv = 0;
    uint32_t cnt = L.m[0][g];
    while (cnt > (uint32_t)kChunk && lv + 1 < L.levels) cnt = L.m[++lv][g];
    ept acc = ept_zero(C);
    if (cnt) acc = sum_items(PartialItems{L.part[lv], L.base[lv], L.cw[lv]}, g, g >> c, 0, cnt, C);
    store_ept(B + 8 * g, acc);
  }
}

// ---- Bucket Reduction (tree form) -----------------------------------------

// One tree level: for the 2^s bucket pairs (2b, 2b + 1) of every window,
// W_b <- W_2b + W_(2b+1) + B_(2b+1) and B_b <- 2 (B_2b + B_(2b+1)).
// Entries of window k sit at k 2^c + index in every buffer. On the first
// level every W is zero; on the last one (s = 0) the new B is not needed.
// The two updates are independent chains of about 17 products each, so
// they run on alternate whole waves (even waves W, odd waves B): the small
// levels, where a level's time is one thread's chain, take half as long,
// and no wave diverges. Launched with two threads per pair.
__global__ __launch_bounds__(kMsmThreads) void msm_reduce_kernel(const u32x4* __restrict__ Bin,
                                                                 const u32x4* __restrict__ Win,
                                                                 u32x4* __restrict__ Bout,
                                                                 u32x4* __restrict__ Wout, int c, int K, int s,
                                                                 int first, MsmConsts C) {
  const int64_t total = (int64_t)K << s;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t pair_waves = ((int64_t)gridDim.x * blockDim.x) >> 7;  // blockDim is a multiple of 128
  const bool form_b = (wave & 1) != 0;
  if (form_b && s == 0) return;
  for (int64_t g = (wave >> 1) * 64 + (threadIdx.x & 63); g < total; g += pair_waves * 64) {
    const int64_t k = g >> s, b = g & ((1 << s) - 1);
    const int64_t l = (k << c) + 2 * b, o = (k << c) + b;
    const ept BR = load_ept(Bin + 8 * (l + 1));
    if (form_b) {
      store_ept(Bout + 8 * o, dbl(add_full(load_ept(Bin + 8 * l), BR, C), C));
    } else {
      ept w = BR;
      if (!first) w = add_full(add_full(load_ept(Win + 8 * l), load_ept(Win + 8 * (l + 1)), C), BR, C);
      store_ept(Wout + 8 * o, w);
    }
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

// Lane-parallel forms of the doubling and the addition for the serial
// window merging: the independent products of each step run on separate
// lanes of one wave (lane l takes product min(l, n - 1) of the step), and
// every lane reads all of them back, so that the state stays replicated.
__device__ FRNTT_INLINE fr_t read_lane(const fr_t& x, int l) {
  fr_t o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.w[i] = (uint32_t)__builtin_amdgcn_readlane((int)x.w[i], l);
  return o;
}

// operand l of up to five, as a masked blend of values (every operand is
// read, so the selection never becomes a choice of address, which would put
// the operands in scratch memory)
__device__ FRNTT_INLINE fr_t pick(int l, const fr_t& a0, const fr_t& a1, const fr_t& a2, const fr_t& a3,
                                  const fr_t& a4) {
  const uint32_t m0 = 0u - (uint32_t)(l == 0), m1 = 0u - (uint32_t)(l == 1), m2 = 0u - (uint32_t)(l == 2),
                 m3 = 0u - (uint32_t)(l == 3), m4 = 0u - (uint32_t)(l == 4);
  fr_t o;
#pragma unroll
  for (int i = 0; i < 8; ++i)
    o.w[i] = (a0.w[i] & m0) | (a1.w[i] & m1) | (a2.w[i] & m2) | (a3.w[i] & m3) | (a4.w[i] & m4);
  return o;
}

// X3 = E F, Y3 = G H, Z3 = F G, T3 = E H on lanes 0..3
__device__ FRNTT_INLINE ept finish_lanes(int lane, const fr_t& E, const fr_t& F, const fr_t& G, const fr_t& H) {
  const int l = lane < 3 ? lane : 3;
  const fr_t r = mont_mul(pick(l, E, G, F, E, E), pick(l, F, H, G, H, H));
  ept o;
  o.X = read_lane(r, 0);
  o.Y = read_lane(r, 1);
  o.Z = read_lane(r, 2);
  o.T = read_lane(r, 3);
  return o;
}

__device__ FRNTT_INLINE ept dbl_lanes(int lane, const ept& P) {
  const int l = lane < 3 ? lane : 3;
  const fr_t xy = fr_add(P.X, P.Y);
  const fr_t s = pick(l, P.X, P.Y, P.Z, xy, xy);
  const fr_t r = mont_mul(s, s);
  const fr_t A = read_lane(r, 0), B = read_lane(r, 1), Z2 = read_lane(r, 2), S = read_lane(r, 3);
  const fr_t E = fr_sub(fr_sub(S, A), B);
  const fr_t G = fr_sub(B, A);
  const fr_t F = fr_sub(G, fr_add(Z2, Z2));
  const fr_t H = fr_sub(fr_zero(), fr_add(A, B));
  return finish_lanes(lane, E, F, G, H);
}

// P + Q with 2 d' T_Q given
__device__ FRNTT_INLINE ept add_lanes(int lane, const ept& P, const ept& Q, const fr_t& kTQ) {
  const int l = lane < 3 ? lane : 3;
  const fr_t ymx = fr_sub(P.Y, P.X), ypx = fr_add(P.Y, P.X);
  const fr_t r = mont_mul(pick(l, ymx, ypx, P.T, P.Z, P.Z),
                          pick(l, fr_sub(Q.Y, Q.X), fr_add(Q.Y, Q.X), kTQ, Q.Z, Q.Z));
  const fr_t A = read_lane(r, 0), B = read_lane(r, 1), Cc = read_lane(r, 2), ZZ = read_lane(r, 3);
  const fr_t D = fr_add(ZZ, ZZ);
  const fr_t E = fr_sub(B, A), F = fr_sub(D, Cc), G = fr_add(D, Cc), H = fr_add(B, A);
  return finish_lanes(lane, E, F, G, H);
}

constexpr int kMergeMaxK = 256;

// MSM = sum_k 2^(c k) W_k from the top window down (one wave; the W_k and
// their 2 d' T are staged in LDS first), then the affine (x, y) in canonical
// form: out[0..7] = x, out[8..15] = y.
__global__ __launch_bounds__(64) void msm_merge_kernel(const u32x4* __restrict__ W, int c, int K,
                                                       uint32_t* __restrict__ out, MsmConsts C) {
  __shared__ fr_t sw[kMergeMaxK][5];
  const int lane = threadIdx.x;
  for (int k = lane; k < K; k += 64) {
    const ept w = load_ept(W + 8 * ((int64_t)k << c));
    sw[k][0] = w.X;
    sw[k][1] = w.Y;
    sw[k][2] = w.Z;
    sw[k][3] = w.T;
    sw[k][4] = mont_mul(w.T, C.k);
  }
  __syncthreads();
  ept acc = ept_zero(C);
  for (int k = K - 1; k >= 0; --k) {
    if (k != K - 1)
      for (int i = 0; i < c; ++i) acc = dbl_lanes(lane, acc);
    ept w;
    w.X = sw[k][0];
    w.Y = sw[k][1];
    w.Z = sw[k][2];
    w.T = sw[k][3];
    acc = add_lanes(lane, acc, w, sw[k][4]);
  }
  fr_t x, y;
  to_affine(acc, C, &x, &y);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      out[i] = x.w[i];
      out[8 + i] = y.w[i];
    }
  }
}

// ---- batch scalar multiplication ------------------------------------------

// out_i = S_i P_i in affine form (out: x then y, 16 words per point), by
// left-to-right double-and-add over the 256 scalar bits.
__global__ __launch_bounds__(kMsmThreads) void ec_mul_kernel(const u32x4* __restrict__ sc,
                                                             const u32x4* __restrict__ pts, int64_t n,
                                                             u32x4* __restrict__ out, MsmConsts C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    fr_t ymx, ypx, kt;
    prepare_point(pts + 4 * i, &ymx, &ypx, &kt, C);
    uint32_t s[8];
    load_scalar(sc + 2 * i, s);
    ept acc = ept_zero(C);
    for (int b = 255; b >= 0; --b) {
      acc = dbl(acc, C);
      if ((s[b >> 5] >> (b & 31)) & 1u) acc = add_mixed(acc, ymx, ypx, kt, C);
    }
    fr_t x, y;
    to_affine(acc, C, &x, &y);
    store_fr(out + 4 * i, x);
    store_fr(out + 4 * i + 2, y);
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

bool fe_eq(const host::Fe& a, const host::Fe& b) {
  return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2] && a.v[3] == b.v[3];
}

// A square root of a quadratic residue a mod r by Tonelli and Shanks
// (r - 1 = 2^28 q with q odd; 5 generates Fr^*, so it is a non-residue).
host::Fe fe_sqrt(const host::Field& F, const host::Fe& a) {
  host::Fe q = host::kR;
  q.v[0] -= 1;
  int S = 0;
  while ((q.v[0] & 1) == 0) {
    for (int i = 0; i < 4; ++i) q.v[i] = (q.v[i] >> 1) | (i < 3 ? (q.v[i + 1] << 63) : 0);
    ++S;
  }
  host::Fe q1 = q;  // (q + 1) / 2
  host::add_in(q1, host::from_u64(1));
  for (int i = 0; i < 4; ++i) q1.v[i] = (q1.v[i] >> 1) | (i < 3 ? (q1.v[i + 1] << 63) : 0);
  const host::Fe one = host::from_u64(1);
  host::Fe c = F.pow(host::from_u64(5), q), t = F.pow(a, q), x = F.pow(a, q1);
  int m = S;
  while (!fe_eq(t, one)) {
    int i = 0;
    host::Fe t2 = t;
    while (!fe_eq(t2, one) && i < m) {
      t2 = F.mul(t2, t2);
      ++i;
    }
    if (i >= m) break;  // not a residue (cannot happen for -a)
    host::Fe b = c;
    for (int j = 0; j < m - i - 1; ++j) b = F.mul(b, b);
    m = i;
    c = F.mul(b, b);
    t = F.mul(t, c);
    x = F.mul(x, b);
  }
  return x;
}

MsmConsts make_consts() {
  const host::Field F;
  MsmConsts C;
  fe_words(times_pow2(host::from_u64(1), 522), &C.r2);
  fe_words(times_pow2(host::from_u64(1), 261), &C.one);
  const host::Fe a = host::from_u64(kCurveA), d = host::from_u64(kCurveD);
  const host::Fe s = fe_sqrt(F, host::sub(host::from_u64(0), a));
  const host::Fe sinv = F.inv(s);
  // 2 d' = -2 d / a
  const host::Fe k = host::sub(host::from_u64(0), F.mul(host::add(d, d), F.inv(a)));
  fe_words(times_pow2(s, 261), &C.s);
  fe_words(times_pow2(sinv, 261), &C.sinv);
  fe_words(times_pow2(k, 261), &C.k);
  fe_words(times_pow2(s, 522), &C.r2s);
  fe_words(times_pow2(F.mul(k, s), 783), &C.r3sk);
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
constexpr int64_t kMsmMaxPoints = (int64_t)1 << 26;

int windows_for(int c) { return (256 + c - 1) / c; }

// Chunk-slot bounds CW of the accumulation levels: level 0 has at most
// ceil(n / kChunk0) + 2^c chunks per window; a later level cuts only buckets
// with more than kChunk partials, into fewer than a sixteenth as many
// chunks, so at most CW_prev / 16 + 1. Levels are added until no bucket can
// have more than kChunk partials. Returns the level count (0: the buckets
// are summed from the points directly, n <= kChunk0).
int chunk_levels(int64_t n, int c, int64_t* cw) {
  if (n <= kChunk0) return 0;
  int lv = 0;
  int64_t bound = (n + kChunk0 - 1) / kChunk0;
  cw[lv++] = bound + ((int64_t)1 << c);
  while (bound > kChunk) {
    bound = (bound + kChunk - 1) / kChunk;
    cw[lv] = cw[lv - 1] / 16 + 1;
    ++lv;
  }
  return lv;
}

struct MsmLayout {
  size_t prep, cnt, lvl, idx, sort, sort_tmp, part, pts, sorted, total;
  unsigned key_bits;
  int64_t cw[kMaxChunkLevels];
  int64_t part_off[kMaxChunkLevels];  // first partial of each level (points)
  int levels;
};

// Workspace: prepared points; counts, run starts and ends, tile sums; the
// chunk counts and starts of every level; the sorted entries; the sort's
// input and output keys (and input values for wide windows) and its
// temporary storage; the partial sums of every level; two (B, W) buffer pairs of
// K 2^c points; for the Presort-PPG baseline, the points in bucket order.
MsmLayout msm_layout(int64_t n, int c, bool presort) {
  MsmLayout L;
  const size_t K = (size_t)windows_for(c), nb = K << c;
  L.levels = chunk_levels(n, c, L.cw);
  int64_t off = 0;
  for (int i = 0; i < L.levels; ++i) {
    L.part_off[i] = off;
    off += (int64_t)K * L.cw[i];
  }
  const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  L.prep = up((size_t)n * 16 * kPrepStride);
  L.cnt = up(nb * 4 * 4);
  L.lvl = up(nb * 4 * 2 * (size_t)L.levels);
  L.idx = up(K * (size_t)n * 4);
  const bool digit_only = c <= kDigitOnlyMaxWindow;
  L.sort = (digit_only ? 2 : 3) * L.idx;
  L.key_bits = (unsigned)c;
  if (!digit_only)
    while (((size_t)1 << L.key_bits) < nb) ++L.key_bits;
  size_t tmp = 0;
  if (digit_only)
    (void)rocprim::radix_sort_pairs(nullptr, tmp, (const uint16_t*)nullptr, (uint16_t*)nullptr,
                                    rocprim::counting_iterator<uint32_t>(0u), (uint32_t*)nullptr, K * (size_t)n, 0u,
                                    L.key_bits);
  else
    (void)rocprim::radix_sort_pairs(nullptr, tmp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                    (const uint32_t*)nullptr, (uint32_t*)nullptr, K * (size_t)n, 0u, L.key_bits);
  L.sort_tmp = up(tmp);
  L.part = up((size_t)off * 128);
  L.pts = up(nb * 128 * 4);
  L.sorted = presort ? up(K * (size_t)n * 96) : 0;
  L.total = L.prep + L.cnt + L.lvl + L.idx + L.sort + L.sort_tmp + L.part + L.pts + L.sorted;
  return L;
}

size_t msm_workspace_bytes(int64_t n, int c, bool presort) { return msm_layout(n, c, presort).total; }

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
  // From 2^13 points on: the width that measured fastest on MI355X for
  // each floor(log2 n), with uniform field elements as scalars (254 bits).
  // Beyond the additions the cost model below counts, it reflects the
  // number of radix passes (two for c <= 16) and how full the top window is
  // (with 254-bit scalars c = 15 leaves it empty, c = 14 leaves two bits).
  static const int kMeasured[27] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
                                    8, 8, 9, 10, 12, 13, 15, 15, 15, 16, 16, 16, 19, 20};
  if (n >= ((int64_t)1 << 13)) {
    int lg = 63 - __builtin_clzll((unsigned long long)n);
    if (lg > 26) lg = 26;
    return kMeasured[lg];
  }
  // below: K (n + 5 2^c) point additions (accumulation, then about four
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
  return msm_workspace_bytes(n, c, false);
}

}  // extern "C"

namespace frntt {
namespace {

// The whole MSM. With presort (the Presort-PPG baseline) every window's
// points are first written out in bucket order and the accumulation reads
// that copy; otherwise (LS-PPG) it reads the points through the sorted
// index lists, and no presorted copy exists.
template <class Items>
void launch_accumulation(const frntt_ctx* ctx, const Items& items, const MsmLayout& lay, uint32_t* counts,
                         uint32_t* tsum, uint32_t* lvl, u32x4* part, int c, int K, u32x4* B0, hipStream_t st,
                         const MsmConsts& C) {
  const int64_t nb = (int64_t)K << c;
  if (lay.levels == 0) {
    msm_bucket_points_kernel<Items><<<grid_of(ctx, nb, false), kMsmThreads, 0, st>>>(items, counts, c, K, B0, C);
    return;
  }
  const int tiles = c > 10 ? 1 << (c - 10) : 1;
  ChunkLevels CL;
  CL.levels = lay.levels;
  for (int lv = 0; lv < lay.levels; ++lv) {
    uint32_t* m_out = lvl + (size_t)2 * lv * nb;
    uint32_t* b_out = m_out + nb;
    u32x4* dst = part + 8 * lay.part_off[lv];
    const uint32_t* m_in = lv == 0 ? counts : CL.m[lv - 1];
    const int len = lv == 0 ? kChunk0 : kChunk;
    msm_tile_sum_kernel<<<(unsigned)(K * tiles), kTileThreads, 0, st>>>(m_in, tsum, c, len, lv > 0);
    msm_tile_scan_kernel<<<(unsigned)(K * tiles), kTileThreads, 0, st>>>(m_in, tsum, m_out, b_out, c, len, lv > 0);
    const int grid = grid_of(ctx, (int64_t)K * lay.cw[lv], false);
    if (lv == 0)
      msm_chunk_kernel<Items><<<grid, kMsmThreads, 0, st>>>(items, m_in, m_out, b_out, c, K, len, lay.cw[lv], dst,
                                                             C);
    else
      msm_chunk_kernel<PartialItems><<<grid, kMsmThreads, 0, st>>>(
          PartialItems{CL.part[lv - 1], CL.base[lv - 1], CL.cw[lv - 1]}, m_in, m_out, b_out, c, K, len,
          lay.cw[lv], dst, C);
    CL.part[lv] = dst;
    CL.m[lv] = m_out;
    CL.base[lv] = b_out;
    CL.cw[lv] = lay.cw[lv];
  }
  msm_bucket_final_kernel<<<grid_of(ctx, nb, false), kMsmThreads, 0, st>>>(CL, c, K, B0, C);
}

int msm_run(frntt_ctx* ctx, const void* scalars, const void* points, int64_t n, int window, void* out,
            void* stream, bool presort) {
  if (!ctx || !out || n < 0 || (n > 0 && (!scalars || !points))) return FRNTT_EINVAL;
  if (n > kMsmMaxPoints || window < 0 || window > kMsmMaxWindow) return FRNTT_ERANGE;
  if ((((uintptr_t)scalars | (uintptr_t)points) & 15) != 0) return FRNTT_EALIGN;
  const int c = window ? window : frntt_msm_window(n);
  const int K = n ? windows_for(c) : 0;
  const hipStream_t st = (hipStream_t)stream;
  // the radix sort clears its counters with memset nodes, which graph
  // replays do not redo reliably: an MSM is never captured
  if (stream_capturing(st)) return FRNTT_ESTATE;
  MsmDeviceGuard guard(ctx->device);
  static const MsmConsts C = make_consts();
  if (n == 0) {
    msm_merge_kernel<<<1, 64, 0, st>>>(nullptr, c, 0, (uint32_t*)out, C);
    return msm_status(ctx);
  }
  const int64_t nb = (int64_t)K << c;
  const MsmLayout lay = msm_layout(n, c, presort);
  void* ws = nullptr;
  int rc = get_scratch(ctx, st, lay.total, &ws);
  if (rc != FRNTT_OK) return rc;
  char* p = (char*)ws;
  u32x4* prep = (u32x4*)p;
  p += lay.prep;
  uint32_t* counts = (uint32_t*)p;
  uint32_t* start = counts + nb;
  uint32_t* ends = start + nb;
  uint32_t* tsum = ends + nb;
  p += lay.cnt;
  uint32_t* lvl = (uint32_t*)p;  // level l: chunk counts at 2 l nb, starts at (2 l + 1) nb
  p += lay.lvl;
  uint32_t* idx = (uint32_t*)p;
  p += lay.idx;
  const bool digit_only = c <= kDigitOnlyMaxWindow;
  // 16-bit keys for digit-only sorts, 32-bit otherwise (buffers sized for the latter)
  void* keys_in = p;
  void* keys_out = p + lay.idx;
  uint32_t* vals_in = digit_only ? nullptr : (uint32_t*)(p + 2 * lay.idx);
  p += lay.sort;
  void* sort_tmp = p;
  p += lay.sort_tmp;
  u32x4* part = (u32x4*)p;
  p += lay.part;
  u32x4* B0 = (u32x4*)p;
  u32x4* W0 = B0 + 8 * nb;
  u32x4* B1 = W0 + 8 * nb;
  u32x4* W1 = B1 + 8 * nb;
  p += lay.pts;
  u32x4* sorted = (u32x4*)p;

  const int64_t total = (int64_t)K * n;
  zero_words_kernel<<<(unsigned)((2 * nb + 255) / 256), 256, 0, st>>>(start, 2 * nb);
  size_t tmp_bytes = lay.sort_tmp;
  const int64_t bound_steps = (total + kBoundsPerThread - 1) / kBoundsPerThread;
  if (digit_only) {
    msm_prep_kernel<uint16_t><<<grid_of(ctx, n, false), kMsmThreads, 0, st>>>(
        (const u32x4*)points, (const u32x4*)scalars, n, c, K, prep, (uint16_t*)keys_in, nullptr, C);
    const hipError_t se = rocprim::radix_sort_pairs(sort_tmp, tmp_bytes, (const uint16_t*)keys_in,
                                                    (uint16_t*)keys_out, rocprim::counting_iterator<uint32_t>(0u),
                                                    idx, (size_t)total, 0u, lay.key_bits, st);
    if (se != hipSuccess) return set_hip_error(ctx, se);
    msm_bounds_kernel<uint16_t><<<grid_of(ctx, bound_steps, true), kMsmThreads, 0, st>>>(
        (const uint16_t*)keys_out, idx, n, c, total, start, ends);
  } else {
    msm_prep_kernel<uint32_t><<<grid_of(ctx, n, false), kMsmThreads, 0, st>>>(
        (const u32x4*)points, (const u32x4*)scalars, n, c, K, prep, (uint32_t*)keys_in, vals_in, C);
    const hipError_t se = rocprim::radix_sort_pairs(sort_tmp, tmp_bytes, (const uint32_t*)keys_in,
                                                    (uint32_t*)keys_out, (const uint32_t*)vals_in, idx,
                                                    (size_t)total, 0u, lay.key_bits, st);
    if (se != hipSuccess) return set_hip_error(ctx, se);
    msm_bounds_kernel<uint32_t><<<grid_of(ctx, bound_steps, true), kMsmThreads, 0, st>>>(
        (const uint32_t*)keys_out, idx, n, c, total, start, ends);
  }
  msm_counts_kernel<<<grid_of(ctx, nb, false), kMsmThreads, 0, st>>>(start, ends, counts, c, K);
  if (presort) {
    msm_gather_kernel<<<grid_of(ctx, total, false), kMsmThreads, 0, st>>>(prep, idx, n, total, sorted);
    launch_accumulation(ctx, SortedItems{sorted, start}, lay, counts, tsum, lvl, part, c, K, B0, st, C);
  } else {
    launch_accumulation(ctx, PointItems{prep, idx, start, n}, lay, counts, tsum, lvl, part, c, K, B0, st, C);
  }
  u32x4 *bi = B0, *wi = W0, *bo = B1, *wo = W1;
  for (int s = c - 1; s >= 0; --s) {
    msm_reduce_kernel<<<grid_of(ctx, (int64_t)K << (s + 1), false), kMsmThreads, 0, st>>>(bi, wi, bo, wo, c, K, s,
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

}  // namespace

// Side streams of frntt_msm_batch: independent MSMs run on them so that one
// MSM's latency-bound tail (small reduction levels, the one-wave merge)
// overlaps another's accumulation. Default stream priority throughout.
constexpr int kMsmSideStreams = 3;

struct MsmStreams {
  hipStream_t s[kMsmSideStreams] = {};
  hipEvent_t start = nullptr;  // recorded on the caller's stream
  hipEvent_t done[kMsmSideStreams] = {};
  std::mutex mu;               // one batch's enqueue sequence at a time
};

void destroy_msm_streams(frntt_ctx* ctx) {
  MsmStreams* m = ctx->msm_streams;
  if (!m) return;
  for (int i = 0; i < kMsmSideStreams; ++i) {
    if (m->s[i]) (void)hipStreamDestroy(m->s[i]);
    if (m->done[i]) (void)hipEventDestroy(m->done[i]);
  }
  if (m->start) (void)hipEventDestroy(m->start);
  delete m;
  ctx->msm_streams = nullptr;
}

namespace {

int get_msm_streams(frntt_ctx* ctx, MsmStreams** out) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->msm_streams) {
    MsmStreams* m = new MsmStreams();
    hipError_t e = hipEventCreateWithFlags(&m->start, hipEventDisableTiming);
    for (int i = 0; i < kMsmSideStreams && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&m->s[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&m->done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      ctx->msm_streams = m;
      destroy_msm_streams(ctx);
      return set_hip_error(ctx, e);
    }
    ctx->msm_streams = m;
  }
  *out = ctx->msm_streams;
  return FRNTT_OK;
}

int msm_args_ok(const void* scalars, const void* points, int64_t n, const void* out) {
  if (!out || n < 0 || (n > 0 && (!scalars || !points))) return FRNTT_EINVAL;
  if (n > kMsmMaxPoints) return FRNTT_ERANGE;
  if ((((uintptr_t)scalars | (uintptr_t)points) & 15) != 0) return FRNTT_EALIGN;
  return FRNTT_OK;
}

}  // namespace
}  // namespace frntt

extern "C" {

int frntt_msm_batch(frntt_ctx* ctx, const void* const* scalars, const void* const* points, const int64_t* n,
                    int count, int window, void* const* out, void* stream) {
  if (!ctx || count < 0 || (count > 0 && (!scalars || !points || !n || !out))) return FRNTT_EINVAL;
  if (window < 0 || window > kMsmMaxWindow) return FRNTT_ERANGE;
  for (int i = 0; i < count; ++i) {
    const int rc = msm_args_ok(scalars[i], points[i], n[i], out[i]);
    if (rc != FRNTT_OK) return rc;
  }
  if (count == 0) return FRNTT_OK;
  const hipStream_t st = (hipStream_t)stream;
  if (stream_capturing(st)) return FRNTT_ESTATE;
  MsmDeviceGuard guard(ctx->device);
  MsmStreams* ms = nullptr;
  int rc = get_msm_streams(ctx, &ms);
  if (rc != FRNTT_OK) return rc;
  std::lock_guard<std::mutex> lk(ms->mu);
  const int used = count < kMsmSideStreams ? count : kMsmSideStreams;
  hipError_t e = hipEventRecord(ms->start, st);
  for (int j = 0; j < used && e == hipSuccess; ++j) e = hipStreamWaitEvent(ms->s[j], ms->start, 0);
  if (e != hipSuccess) return set_hip_error(ctx, e);
  for (int i = 0; i < count && rc == FRNTT_OK; ++i)
    rc = msm_run(ctx, scalars[i], points[i], n[i], window, out[i], ms->s[i % used], false);
  // the caller's stream waits for everything that was enqueued, also after
  // an error
  for (int j = 0; j < used; ++j) {
    e = hipEventRecord(ms->done[j], ms->s[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ms->done[j], 0);
    if (e != hipSuccess && rc == FRNTT_OK) rc = set_hip_error(ctx, e);
  }
  return rc;
}

int frntt_msm(frntt_ctx* ctx, const void* scalars, const void* points, int64_t n, int window, void* out,
              void* stream) {
  return msm_run(ctx, scalars, points, n, window, out, stream, false);
}

int frntt_msm_presort(frntt_ctx* ctx, const void* scalars, const void* points, int64_t n, int window, void* out,
                      void* stream) {
  return msm_run(ctx, scalars, points, n, window, out, stream, true);
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
