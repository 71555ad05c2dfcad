// Sustained instruction rates of this GPU, for the roofline the benchmark
// reports (not part of the transform library).
//
// Two saturating kernels, each one workgroup per CU (the LDS request keeps a
// second one off the CU) with `waves_per_simd` waves on each of its SIMDs:
//   * v_mad_u64_u32, the 32x32+64-bit multiply-add every Montgomery product
//     and carry merge of the transforms is built from: 8 independent chains
//     per lane;
//   * v_mfma_i32_32x32x32_i8, the int8 matrix instruction of the sub-DFTs:
//     4 independent accumulator chains per wave.
// Each thread writes one word of `sink` (grid x block words) so that no chain
// is optimised away.
#include <hip/hip_runtime.h>

#include <stdint.h>

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

constexpr int kLdsWords = 24 * 1024;  // 96 KiB: one workgroup per CU

__global__ __launch_bounds__(1024) void mad_rate_kernel(int iters, uint32_t seed, uint32_t* sink) {
  __shared__ uint32_t lds[kLdsWords];
  if (threadIdx.x == 0) lds[0] = seed;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63;
  uint64_t m[8];
  uint32_t x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    x[j] = lds[0] * (j + 3) + lane;
    m[j] = ((uint64_t)lane << 20) + j;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 64; ++i) {
      const int j = i & 7;
      m[j] = (uint64_t)(uint32_t)m[j] * x[j] + m[j];
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc += (uint32_t)m[j] ^ (uint32_t)(m[j] >> 32);
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(1024) void mfma_rate_kernel(int iters, uint32_t seed, uint32_t* sink) {
  __shared__ uint32_t lds[kLdsWords];
  if (threadIdx.x == 0) lds[0] = seed;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const i32x4 a = {lane, (int)lds[0], 3, 5}, b = {(int)lds[0], lane, 7, 9};
  i32x16 c0 = {}, c1 = {}, c2 = {}, c3 = {};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c1, 0, 0, 0);
      c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c2, 0, 0, 0);
      c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c3, 0, 0, 0);
    }
  }
  int acc = 0;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc += c0[j] + c1[j] + c2[j] + c3[j];
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)acc;
}

extern "C" {

// Run one rate kernel on `device`: kind 0 = v_mad_u64_u32, 1 = int8 MFMA.
// grid = `cus` workgroups of 256 * waves_per_simd threads (1 <= waves_per_simd
// <= 4). Writes the kernel time (ms, HIP events) and the work done: lane
// multiply-adds for kind 0, int8 operations (2 per multiply-accumulate) for
// kind 1. Returns 0, or the hipError_t of the first failing call.
int frntt_peaks_run(int device, int kind, int cus, int waves_per_simd, int iters, double* ms, double* work) {
  if (kind < 0 || kind > 1 || cus < 1 || waves_per_simd < 1 || waves_per_simd > 4 || iters < 1 || !ms || !work)
    return (int)hipErrorInvalidValue;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return (int)e;
  const int threads = 256 * waves_per_simd;
  uint32_t* sink = nullptr;
  e = hipMalloc(&sink, (size_t)cus * threads * sizeof(uint32_t));
  if (e != hipSuccess) return (int)e;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) == hipSuccess) e = hipEventCreate(&e1);
  float t = 0.f;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run only warms up
    const int n = rep == 0 ? 8 : iters;
    e = hipEventRecord(e0, nullptr);
    if (e != hipSuccess) break;
    if (kind == 0)
      hipLaunchKernelGGL(mad_rate_kernel, dim3(cus), dim3(threads), 0, nullptr, n, 1u, sink);
    else
      hipLaunchKernelGGL(mfma_rate_kernel, dim3(cus), dim3(threads), 0, nullptr, n, 1u, sink);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (e != hipSuccess) return (int)e;
  *ms = t;
  const double lanes = (double)cus * threads;
  *work = kind == 0 ? lanes * iters * 64.0 : (double)cus * (threads / 64) * iters * 16.0 * 32 * 32 * 32 * 2;
  return 0;
}

}  // extern "C"
