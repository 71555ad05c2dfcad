// RNS lazy modular product (the paper's Alg. 1, "MXU RNS Lazy"): constants
// shared by the host table builder and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_device.hpp"

namespace frntt {

constexpr int kRnsI = 17;        // residues of the base Q (Q > 2 r^2)
constexpr int kRnsJ = 9;         // residues of the base P (P > 2 x the lazy output bound)
constexpr int kRnsQWords = 20;   // words per element in base Q: 17 residues, 3 zero words
constexpr int kRnsPWords = 12;   // words per element in base P: 9 residues, 3 zero words
constexpr int kRnsU = 15;        // fraction bits of the overflow count estimate
constexpr uint32_t kRnsBound = (1u << 31) - (1u << 24);  // every modulus lies below this

// Per-modulus scalars, passed to the kernels by value.
struct RnsConsts {
  uint32_t q[24];      // q_i (i < 17; unused slots 1)
  uint32_t qneg[24];   // -q_i^-1 mod 2^32 (residue-wise Montgomery product, w = 32)
  uint32_t p[12];      // p_j (j < 9; unused slots 1)
  uint32_t g[12];      // g_j = (-z (Q mod r)) mod p_j
  uint32_t gdec[8];    // (-P) mod r: the decode's overflow correction
  double qinv[24];     // 1 / q_i and 1 / p_j (quotient estimates of the residue reductions)
  double pinv[12];
};

// Operand tables of the three int8 matrix products, in the A-fragment layout
// of v_mfma_i32_32x32x32_i8 (lane l: row l % 32, K bytes 16 (l / 32) .. +15)
// for each (row block, K step), followed by the accumulator seeds of each
// (row block, lane half) (16 int32 each: register r <-> row 8 (r / 4) +
// 4 half + r % 4 of the block).
struct RnsTables {
  const i32x4* enc;   // encode: 3 row blocks x 1 K step; rows (i, h), K = input byte b
  const i32x4* mul;   // Alg. 1 Main: 2 row blocks x 3 K steps; rows (j, h) and the f rows, K = (i, b)
  const i32x4* dec;   // decode: 2 row blocks x 2 K steps; rows = output bytes and the f rows, K = (j, b)
  RnsConsts c;
};

// Fragment and seed counts of each table (i32x4 units).
constexpr int kRnsEncFrag = 3 * 1 * 64, kRnsMulFrag = 2 * 3 * 64, kRnsDecFrag = 2 * 2 * 64;
constexpr int kRnsEncSeed = 3 * 2 * 4, kRnsMulSeed = 2 * 2 * 4, kRnsDecSeed = 2 * 2 * 4;

}  // namespace frntt
