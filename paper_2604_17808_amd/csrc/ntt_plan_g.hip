// Plan kernels of the matrix form (see FRNTT_PLAN_KERNELS in ntt_levels.hpp).
#include "ntt_levels.hpp"

namespace frntt {

FRNTT_DEFINE_PLAN_KERNEL(4, 0, 0)
FRNTT_DEFINE_PLAN_KERNEL(3, 0, 0)
FRNTT_DEFINE_PLAN_KERNEL(2, 0, 0)
FRNTT_DEFINE_PLAN_KERNEL(1, 0, 0)

}  // namespace frntt
