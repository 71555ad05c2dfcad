// One HBM pass with its levels on int8 MFMA (the matrix form); levels the
// MFMA tiling cannot cover run on the VALUs.
#include "ntt_levels.hpp"

namespace frntt {

__global__ __launch_bounds__(kThreads) void ntt_pass_mfma_kernel(PassParams P, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  __shared__ i32x4 lds_f[kBatMaxRho * 64 + kBatMaxRho * 8];
  run_pass<1>(lds, lds_f, P, T, logical_wg(P));
}

}  // namespace frntt
