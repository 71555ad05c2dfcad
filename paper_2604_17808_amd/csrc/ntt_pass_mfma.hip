// One HBM pass with its levels on int8 MFMA (the matrix form): a generic
// kernel that reads the level radices from the pass descriptor, and kernels
// specialised for the level splits of a 4096-element tile.
#include "ntt_levels.hpp"

namespace frntt {

__global__ __launch_bounds__(kMfmaThreads) void ntt_pass_mfma_kernel(PassParams P, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[kPlanBatLds];
  run_pass<1, kMfmaThreads>(lds, lds_f, P, T, logical_wg(P));
}

template <int M0, int M1, int M2>
__global__ __launch_bounds__(kMfmaThreads) void ntt_pass_mfma_plan_kernel(PassParams P, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[PassPlan<M0, M1, M2>::kLds];
  run_pass_plan<M0, M1, M2>(lds, lds_f, P, T, logical_wg(P));
}

// Kernel for a pass with a 4096-element tile and these levels, or nullptr.
MfmaPassKernel mfma_plan_kernel(int nlev, const int* lev) {
  const int a = lev[0], b = nlev > 1 ? lev[1] : 0, c = nlev > 2 ? lev[2] : 0;
  if (nlev == 3 && a == 4 && b == 4 && c == 4) return ntt_pass_mfma_plan_kernel<4, 4, 4>;
  if (nlev == 3 && a == 4 && b == 4 && c == 3) return ntt_pass_mfma_plan_kernel<4, 4, 3>;
  if (nlev == 3 && a == 4 && b == 3 && c == 3) return ntt_pass_mfma_plan_kernel<4, 3, 3>;
  if (nlev == 3 && a == 3 && b == 3 && c == 3) return ntt_pass_mfma_plan_kernel<3, 3, 3>;
  if (nlev == 2 && a == 4 && b == 4) return ntt_pass_mfma_plan_kernel<4, 4, 0>;
  if (nlev == 2 && a == 4 && b == 3) return ntt_pass_mfma_plan_kernel<4, 3, 0>;
  if (nlev == 2 && a == 3 && b == 3) return ntt_pass_mfma_plan_kernel<3, 3, 0>;
  if (nlev == 2 && a == 3 && b == 2) return ntt_pass_mfma_plan_kernel<3, 2, 0>;
  return nullptr;
}

}  // namespace frntt
