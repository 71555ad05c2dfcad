// Persistent kernel for uneven batches: resident workgroups pull (pass,
// workgroup) items from a device queue; a pass waits for the previous pass
// of its job.
#include "ntt_levels.hpp"

namespace frntt {

// One (pass, workgroup) item. A matrix-form pass (always a full
// 4096-element tile) runs the level code specialised to its level split (the
// same bodies as the plan kernels of single transforms); a butterfly-form pass
// runs the butterfly stages with this kernel's 512 threads.
#define FRNTT_BATCH_LDS_OK(a, b, c) static_assert(PassPlan<a, b, c>::kLds <= kPlanBatLds, "plan blocks fit");
FRNTT_PLAN_KERNELS(FRNTT_BATCH_LDS_OK)
#undef FRNTT_BATCH_LDS_OK

// Each plan body is a function of its own (not inlined into the persistent
// loop), so that its registers are allocated for it alone.
template <int M0, int M1, int M2>
__device__ __attribute__((noinline)) void batch_plan_pass(u32x4* lds, i32x4* lds_f, const PassParams& P,
                                                          const DevTables& T, int64_t wg) {
  run_pass_plan<M0, M1, M2>(lds, lds_f, P, T, wg);
}

__device__ __attribute__((noinline)) void batch_bfly_pass(u32x4* lds, const PassParams& P, const DevTables& T,
                                                          int64_t wg) {
  run_pass_bfly<kMfmaThreads>(lds, P, T, wg);
}

__device__ FRNTT_INLINE void run_batch_pass(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                            int64_t wg) {
  const int nlev = P.nlev;
  const int code = __builtin_amdgcn_readfirstlane(
      P.engine == 1 ? nlev * 1000 + P.lev_log[0] * 100 + (nlev > 1 ? P.lev_log[1] : 0) * 10 + (nlev > 2 ? P.lev_log[2] : 0)
                    : 0);
  switch (code) {
#define FRNTT_BATCH_CASE(a, b, c) \
    case (c > 0 ? 3 : b > 0 ? 2 : 1) * 1000 + a * 100 + b * 10 + c: batch_plan_pass<a, b, c>(lds, lds_f, P, T, wg); return;
    FRNTT_PLAN_KERNELS(FRNTT_BATCH_CASE)
#undef FRNTT_BATCH_CASE
    default: batch_bfly_pass(lds, P, T, wg);
  }
}

__global__ __launch_bounds__(kMfmaThreads) void ntt_batch_kernel(BatchParams B, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[kPlanBatLds];
  // the item slot shares the constant-block area: it is written and read
  // only between passes, when no MFMA level uses that area
  int& item_sh = *reinterpret_cast<int*>(&lds_f[0]);
  // The loop skeleton has no lane-divergent branches: the queue and counter
  // atomics are issued by all 64 lanes of wave 0 (lane 0 adds 1, the others
  // 0) and every loop condition is made wave-uniform with readfirstlane.
  // A thread-0-only block at the end of a loop that contains barriers lets
  // the compiler restructure the loop around lane 0, and the barriers then
  // no longer pair up.
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const unsigned int one = (threadIdx.x & 63) == 0 ? 1u : 0u;
  for (;;) {
    if (wave == 0) item_sh = (int)__builtin_amdgcn_readfirstlane(atomicAdd(B.queue, one));
    __syncthreads();
    const int64_t item = __builtin_amdgcn_readfirstlane(item_sh);
    __syncthreads();
    if (item >= B.n_items) break;
    const int p = __builtin_amdgcn_readfirstlane((int)B.item_pass[item]);
    const int dep = __builtin_amdgcn_readfirstlane(B.pass_dep[p]);
    if (dep >= 0) {
      // items are handed out pass by pass, so every workgroup of `dep` was
      // taken by a running workgroup before this one: the wait always ends
      if (wave == 0) {
        const unsigned int need = (unsigned int)__builtin_amdgcn_readfirstlane((int)B.pass_wgs[dep]);
        for (;;) {
          const unsigned int d = (unsigned int)__builtin_amdgcn_readfirstlane(
              (int)__hip_atomic_load(&B.done[dep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
          if (d >= need) break;
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
    }
    // every thread reads the pass descriptor straight from global memory
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const PassParams& P = B.passes[p];
    const int64_t wg = B.item_wg[item];
    run_batch_pass(lds, lds_f, P, T, wg);
    __syncthreads();
    if (wave == 0) {
      __threadfence();
      __hip_atomic_fetch_add(&B.done[p], one, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace frntt
