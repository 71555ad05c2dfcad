// Persistent kernel for uneven batches: resident workgroups pull (pass,
// workgroup) items from a device queue; a pass waits for the previous pass
// of its job.
#include "ntt_levels.hpp"

namespace frntt {

// One (pass, workgroup) item. A matrix-form pass with a full 4096-element
// tile runs the level code specialised to its level split (the same bodies
// as the plan kernels of single transforms); other passes take the generic
// per-pass path.
static_assert(PassPlan<4, 4, 4>::kLds <= kPlanBatLds && PassPlan<4, 4, 3>::kLds <= kPlanBatLds &&
                  PassPlan<4, 3, 3>::kLds <= kPlanBatLds && PassPlan<3, 3, 3>::kLds <= kPlanBatLds &&
                  PassPlan<4, 4, 0>::kLds <= kPlanBatLds && PassPlan<4, 3, 0>::kLds <= kPlanBatLds &&
                  PassPlan<3, 3, 0>::kLds <= kPlanBatLds && PassPlan<3, 2, 0>::kLds <= kPlanBatLds,
              "the batch kernel's constant-block area holds every plan's blocks");

__device__ FRNTT_INLINE void run_batch_pass(u32x4* lds, i32x4* lds_f, const PassParams& P, const DevTables& T,
                                            int64_t wg) {
  const int nlev = P.nlev;
  const int code = __builtin_amdgcn_readfirstlane(
      P.engine == 1 && P.log_t == kMaxLogT
          ? nlev * 1000 + P.lev_log[0] * 100 + (nlev > 1 ? P.lev_log[1] : 0) * 10 + (nlev > 2 ? P.lev_log[2] : 0)
          : 0);
  switch (code) {
    case 3444: run_pass_plan<4, 4, 4>(lds, lds_f, P, T, wg); return;
    case 3443: run_pass_plan<4, 4, 3>(lds, lds_f, P, T, wg); return;
    case 3433: run_pass_plan<4, 3, 3>(lds, lds_f, P, T, wg); return;
    case 3333: run_pass_plan<3, 3, 3>(lds, lds_f, P, T, wg); return;
    case 2440: run_pass_plan<4, 4, 0>(lds, lds_f, P, T, wg); return;
    case 2430: run_pass_plan<4, 3, 0>(lds, lds_f, P, T, wg); return;
    case 2330: run_pass_plan<3, 3, 0>(lds, lds_f, P, T, wg); return;
    case 2320: run_pass_plan<3, 2, 0>(lds, lds_f, P, T, wg); return;
    default: run_pass<2, kMfmaThreads>(lds, lds_f, P, T, wg);
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
