// The other lane forms of asum / dot for BF16 storage (instantiations of
// lift_reduce_lanes.hpp).
#include "lift_reduce_lanes.hpp"

namespace lift {

const void *reduce_lanes_kernel_bf16(int op, int vec_bytes, int unroll, int form)
{
    return pick_lanes<BF16>(op, vec_bytes, unroll, form);
}

}  // namespace lift
