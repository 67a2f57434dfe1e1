// The other lane forms of asum / dot for F32 storage (instantiations of
// lift_reduce_lanes.hpp).
#include "lift_reduce_lanes.hpp"

namespace lift {

const void *reduce_lanes_kernel_f32(int op, int vec_bytes, int unroll, int form)
{
    return pick_lanes<F32>(op, vec_bytes, unroll, form);
}

}  // namespace lift
