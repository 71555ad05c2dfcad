// Persistent kernel for uneven batches: resident workgroups pull (pass,
// workgroup) items of one stage (the s-th pass of every job) from a device
// queue. The stages of a batch are consecutive launches, so a pass finds the
// previous pass of its job complete without any wait or fence.
#include "ntt_levels.hpp"

namespace frntt {

// One (pass, workgroup) item. A matrix-form pass (always a full
// 4096-element tile) runs the level code specialised to its level split (the
// same bodies as the plan kernels of single transforms); a butterfly-form pass
// runs the butterfly stages with this kernel's 512 threads.
#define FRNTT_BATCH_LDS_OK(a, b, c) static_assert(PassPlan<a, b, c>::kLds <= kPlanBatLds, "plan blocks fit");
FRNTT_PLAN_KERNELS(FRNTT_BATCH_LDS_OK)
#undef FRNTT_BATCH_LDS_OK

// The pass descriptors and tables of a batch sit in global memory and are
// read-only during the launch: the pass bodies read them through the
// constant address space, at a wave-uniform address, so the reads become
// scalar loads that no store can invalidate (through a plain reference they
// would be reloaded from memory after every store, inside the pair loops).
// The address passes through an empty asm statement, so that loads through
// two references made in different iterations of a loop are not merged and
// hoisted out of it (that would keep every field live in scalar registers
// across the whole loop).
template <class S>
__device__ FRNTT_INLINE const S& constant_ref(const S& g) {
  const uint64_t a = (uint64_t)(uintptr_t)&g;
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  __asm__ volatile("" : "+s"(lo), "+s"(hi));
  const __attribute__((address_space(4))) S* c =
      (const __attribute__((address_space(4))) S*)(((uint64_t)hi << 32) | lo);
  return *(const S*)c;
}

// Each plan body is a function of its own (not inlined into the persistent
// loop), so that its registers are allocated for it alone. P and T must be
// references into global memory (the batch buffer): they are re-read through
// the constant address space.
// A call runs the item's `count` consecutive tiles, staging the constant
// blocks for the first only.
template <int M0, int M1, int M2>
__device__ __attribute__((noinline)) void batch_plan_pass(u32x4* lds, i32x4* lds_f, const PassParams& P,
                                                          const DevTables& T, int64_t wg, int count) {
  for (int t = 0; t < count; ++t) run_pass_plan<M0, M1, M2>(lds, lds_f, constant_ref(P), constant_ref(T), wg + t, t == 0);
}

__device__ __attribute__((noinline)) void batch_bfly_pass(u32x4* lds, const PassParams& P, const DevTables& T,
                                                          int64_t wg, int count) {
  for (int t = 0; t < count; ++t) {
    run_pass_bfly<kMfmaThreads>(lds, constant_ref(P), constant_ref(T), wg + t);
    __syncthreads();  // the next tile's loads overwrite the LDS rows this one stored from
  }
}

__device__ FRNTT_INLINE void run_batch_pass(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                            int64_t wg, int count) {
  const int nlev = P.nlev;
  const int code = __builtin_amdgcn_readfirstlane(
      P.engine == 1 ? nlev * 1000 + P.lev_log[0] * 100 + (nlev > 1 ? P.lev_log[1] : 0) * 10 + (nlev > 2 ? P.lev_log[2] : 0)
                    : 0);
  switch (code) {
#define FRNTT_BATCH_CASE(a, b, c) \
    case (c > 0 ? 3 : b > 0 ? 2 : 1) * 1000 + a * 100 + b * 10 + c: batch_plan_pass<a, b, c>(lds, lds_f, P, T, wg, count); return;
    FRNTT_PLAN_KERNELS(FRNTT_BATCH_CASE)
#undef FRNTT_BATCH_CASE
    default: batch_bfly_pass(lds, P, T, wg, count);
  }
}

__global__ __launch_bounds__(kMfmaThreads) void ntt_batch_kernel(BatchParams B) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[kPlanBatLds];
  // the item slot shares the constant-block area: it is written and read
  // only between passes, when no MFMA level uses that area
  int& item_sh = *reinterpret_cast<int*>(&lds_f[0]);
  // The loop skeleton has no lane-divergent branches: the queue atomic is
  // issued by all 64 lanes of wave 0 (lane 0 adds 1, the others 0) and every
  // loop condition is made wave-uniform with readfirstlane. A thread-0-only
  // block at the end of a loop that contains barriers lets the compiler
  // restructure the loop around lane 0, and the barriers then no longer pair
  // up.
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned int one = (threadIdx.x & 63) == 0 ? 1u : 0u;
  for (;;) {
    if (wave == 0) item_sh = (int)__builtin_amdgcn_readfirstlane(atomicAdd(B.queue, one));
    __syncthreads();
    const int64_t item = B.item_begin + __builtin_amdgcn_readfirstlane(item_sh);
    __syncthreads();
    if (item >= B.item_end) break;
    const int p = __builtin_amdgcn_readfirstlane((int)B.item_pass[item]);
    const PassParams& P = B.passes[p];  // global memory
    const int64_t wg = B.item_wg[item];
    const int count = __builtin_amdgcn_readfirstlane(B.item_cnt[item]);
    run_batch_pass(lds, lds_f, P, *B.tables, wg, count);
    __syncthreads();  // the next fetch rewrites the item slot
  }
}

}  // namespace frntt
