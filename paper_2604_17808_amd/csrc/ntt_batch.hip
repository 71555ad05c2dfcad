// Persistent kernel for uneven batches: resident workgroups pull (pass,
// workgroup) items from a device queue; a pass waits for the previous pass
// of its job.
#include "ntt_levels.hpp"

namespace frntt {

__global__ __launch_bounds__(kThreads) void ntt_batch_kernel(BatchParams B, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[kBatMaxRho * 64];
  __shared__ int64_t item_sh;
  for (;;) {
    if (threadIdx.x == 0) item_sh = (int64_t)atomicAdd(B.queue, 1u);
    __syncthreads();
    const int64_t item = item_sh;
    __syncthreads();
    if (item >= B.n_items) break;
    const int64_t p = B.item_pass[item];
    const int dep = B.pass_dep[p];
    if (dep >= 0) {
      // items are handed out pass by pass, so every workgroup of `dep` was
      // taken by a running workgroup before this one: the wait always ends
      if (threadIdx.x == 0) {
        const unsigned int need = (unsigned int)B.pass_wgs[dep];
        while (__hip_atomic_load(&B.done[dep], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need)
          __builtin_amdgcn_s_sleep(2);
      }
      __syncthreads();
    }
    // every thread reads the pass descriptor straight from global memory
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const PassParams& P = B.passes[p];
    run_pass<2>(lds, lds_f, P, T, B.item_wg[item]);
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence();
      __hip_atomic_fetch_add(&B.done[p], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}


}  // namespace frntt
