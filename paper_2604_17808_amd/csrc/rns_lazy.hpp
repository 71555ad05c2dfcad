// RNS lazy modular product (the paper's Alg. 1, "MXU RNS Lazy"): shapes of
// the three field widths and the per-field constants the kernels take.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_device.hpp"

namespace frntt {

constexpr uint32_t kRnsBound = (1u << 31) - (1u << 24);  // every RNS modulus lies below this
constexpr int kRnsMaxI = 49, kRnsMaxJ = 25, kRnsMaxMW = 24, kRnsMaxL = 26;

// One field width: I residues in the base Q (Q > 2 M^2), J in the base P
// (P > twice the lazy output bound), MW 32-bit words per canonical element,
// L 29-bit limbs of the radix Montgomery baseline. Elements are stored
// element-major: base Q in QW words (residues, then zeros), base P in PW.
// The int8 products run K steps of 32 bytes and row blocks of 32 rows.
template <int I_, int J_, int MW_, int L_>
struct RnsShape {
  static constexpr int I = I_, J = J_, MW = MW_, L = L_;
  static constexpr int QW = 4 * ((I + 3) / 4), PW = 4 * ((J + 3) / 4);
  static constexpr int KSQ = (I + 7) / 8, KSP = (J + 7) / 8, KSC = (MW + 7) / 8;
  static constexpr int RBE = (4 * I + 31) / 32;       // encode: rows (i, h)
  static constexpr int RBM = (4 * J + 3 + 31) / 32;   // Main: rows (j, h), then 3 rows of f digits
  static constexpr int RBD = (4 * MW + 3 + 31) / 32;  // decode: rows = output bytes, then 3 f rows
  // table sizes (i32x4 units): A fragments [rb][ks][64 lanes], then seeds [rb][2 halves][4]
  static constexpr int ENC_FRAG = RBE * KSC * 64, MUL_FRAG = RBM * KSQ * 64, DEC_FRAG = RBD * KSP * 64;
  static constexpr int ENC = ENC_FRAG + RBE * 8, MUL = MUL_FRAG + RBM * 8, DEC = DEC_FRAG + RBD * 8;
};
using Rns254 = RnsShape<17, 9, 8, 9>;
using Rns377 = RnsShape<25, 13, 12, 13>;
using Rns753 = RnsShape<49, 25, 24, 26>;

// Per-field scalars, passed to the kernels by value (indices into these
// arrays are compile-time constants in the kernels).
struct RnsConsts {
  uint32_t q[kRnsMaxI + 7];     // q_i (unused slots 1)
  uint32_t qneg[kRnsMaxI + 7];  // -q_i^-1 mod 2^32 (residue-wise Montgomery product, w = 32)
  uint32_t p[kRnsMaxJ + 7];     // p_j (unused slots 1)
  uint32_t g[kRnsMaxJ + 7];     // g_j = (-z (Q mod M)) mod p_j
  double qinv[kRnsMaxI + 7];    // 1 / q_i and 1 / p_j (quotient estimates of the residue reductions)
  double pinv[kRnsMaxJ + 7];
  uint32_t m[kRnsMaxMW];        // the field modulus M, little-endian words
  uint32_t gdec[kRnsMaxMW];     // (-P) mod M: the decode's overflow correction
  uint32_t m29[kRnsMaxL];       // M as 29-bit limbs (Montgomery baseline)
  uint32_t mneg29;              // -M^-1 mod 2^29
  double inv_mtop1;             // 1 / (top word of M + 1): decode's quotient estimate
  int u_mul, u_dec;             // fraction bits of k in Main and in the decode
};

}  // namespace frntt
