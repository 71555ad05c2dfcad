// The matrix form's pass kernels: the dispatcher from a level split of a
// 4096-element tile to its plan kernel (the kernels themselves are defined in
// ntt_plan_*.hip).
#include "ntt_levels.hpp"

namespace frntt {

MfmaPassKernel mfma_plan_kernel(int nlev, const int* lev) {
  const int a = nlev > 0 ? lev[0] : 0, b = nlev > 1 ? lev[1] : 0, c = nlev > 2 ? lev[2] : 0;
  if (nlev < 1 || nlev > 3) return nullptr;
#define FRNTT_MATCH_PLAN(x, y, z) \
  if (a == x && b == y && c == z) return ntt_plan_kernel_##x##y##z;
  FRNTT_PLAN_KERNELS(FRNTT_MATCH_PLAN)
#undef FRNTT_MATCH_PLAN
  return nullptr;
}

}  // namespace frntt
