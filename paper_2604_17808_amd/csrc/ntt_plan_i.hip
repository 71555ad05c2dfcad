// Plan kernels of the matrix form (see FRNTT_PLAN_KERNELS in ntt_levels.hpp).
#include "ntt_levels.hpp"

namespace frntt {

FRNTT_DEFINE_PLAN_KERNEL(3, 4, 4)
FRNTT_DEFINE_PLAN_KERNEL(4, 3, 4)

}  // namespace frntt
