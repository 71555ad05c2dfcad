// One HBM pass with every level on the VALUs (the butterfly form).
#include "ntt_levels.hpp"

namespace frntt {

__global__ __launch_bounds__(kBflyThreads) void ntt_pass_bfly_kernel(PassParams P, DevTables T) {
  __shared__ u32x4 lds[2 << kMaxLogT];
  run_pass_bfly<kBflyThreads>(lds, P, T, logical_wg(P));
}

}  // namespace frntt
