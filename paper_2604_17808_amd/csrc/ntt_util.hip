// Small utility kernels: seeded inputs, input validation, zero fill.
#include "ntt_device.hpp"

namespace frntt {

__device__ FRNTT_INLINE uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// Seeded uniform elements of [0, r) (SplitMix64 counter stream, rejection
// against r, 64 attempts; see the project's input generator).
__global__ void generate_kernel(u32x4* out, uint64_t seed, uint64_t stream_id, uint64_t start,
                                uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t base = seed * 0x9E3779B97F4A7C15ull + (stream_id << 40) + ((start + i) << 8);
  const uint64_t r64[4] = {((uint64_t)FR_R1 << 32) | FR_R0, ((uint64_t)FR_R3 << 32) | FR_R2,
                           ((uint64_t)FR_R5 << 32) | FR_R4, ((uint64_t)FR_R7 << 32) | FR_R6};
  uint64_t w[4];
  for (int t = 0; t < 64; ++t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = mix64(base + ((uint64_t)t << 2) + (uint64_t)j);
    w[3] &= (1ull << 62) - 1;
    bool lt = false, eq = true;
#pragma unroll
    for (int j = 3; j >= 0; --j) {
      lt = lt || (eq && w[j] < r64[j]);
      eq = eq && (w[j] == r64[j]);
    }
    if (lt) break;
    if (t == 63) {
      uint64_t b = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t d = w[j] - r64[j] - b;
        b = (w[j] < r64[j] || (w[j] == r64[j] && b)) ? 1 : 0;
        w[j] = d;
      }
    }
  }
  u32x4 a = {(uint32_t)w[0], (uint32_t)(w[0] >> 32), (uint32_t)w[1], (uint32_t)(w[1] >> 32)};
  u32x4 b = {(uint32_t)w[2], (uint32_t)(w[2] >> 32), (uint32_t)w[3], (uint32_t)(w[3] >> 32)};
  out[2 * i] = a;
  out[2 * i + 1] = b;
}

// Flag any element >= r.
__global__ void validate_kernel(const u32x4* data, uint64_t count, unsigned int* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const fr_t x = ld_elem(data, (int64_t)i);
  uint32_t b = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) subb(x.w[j], fr_mod_word(j), b, &b);
  if (!b) atomicOr(flag, 1u);
}

// Zero `n` 32-bit words (used instead of a memset node so that graph
// captures contain only kernels).
__global__ void zero_words_kernel(unsigned int* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Twiddles of a non-last pass, w_(2^(log_r + log_s))^(rest * k) in
// Montgomery form, at index k * 2^log_s + rest (k < 2^log_r, rest < 2^log_s):
// the stores of a pass then read them contiguously along its lines. With
// scale_log >= 0 every entry also carries the factor 2^-scale_log: the N^-1
// of an inverse transform is one constant factor on every output, so the
// first pass can apply it with its twiddle instead of the last pass spending
// a product on it.
// With coset = 1 (first pass of a coset transform, element index
// n = rest + j 2^log_s): g^n = g^rest * (g^(2^log_s))^j, and g^rest is
// constant along the line, so it commutes with the line's DFT and rides in
// the entry [k][rest]; 2^log_r more entries at N + j hold (g^(2^log_s))^j for
// the load-time pre-scale, one product per element instead of two.
// With coset = 2 (first pass of a two-pass coset INTT, output index
// K = k + 2^log_r k'): g^-K = g^-k * (g^-(2^log_r))^k', and g^-k rides in
// the entries of row k; 2^log_s more entries at N + k' hold
// (g^-(2^log_r))^k' for the last pass's epilogue (one product, not two).
__global__ void pass_twiddle_kernel(u32x4* dst, DevTables T, int dir, int log_r, int log_s, int scale_log,
                                    int coset) {
  const int64_t n = 1ll << (log_r + log_s);
  const int64_t total = n + (coset == 1 ? (1ll << log_r) : coset == 2 ? (1ll << log_s) : 0);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i >= n) {
      const uint32_t e = coset == 1 ? (uint32_t)((i - n) << log_s) : (uint32_t)((i - n) << log_r);
      st_elem(dst, i, coset_pow(T, coset == 1 ? 0 : 1, e));
      continue;
    }
    const uint64_t k = (uint64_t)i >> log_s;
    const uint64_t rest = (uint64_t)i & ((1ull << log_s) - 1);
    fr_t w = pow_tw(T, dir, log_r + log_s, rest * k);
    if (scale_log >= 0) w = mont_mul(ld_elem(T.ninv, scale_log), w);
    if (coset == 1) w = mont_mul(coset_pow(T, 0, (uint32_t)rest), w);
    if (coset == 2) w = mont_mul(coset_pow(T, 1, (uint32_t)k), w);
    st_elem(dst, i, w);
  }
}

}  // namespace frntt
