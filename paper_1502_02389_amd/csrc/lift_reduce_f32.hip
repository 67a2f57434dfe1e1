// asum / dot kernels for F32 storage (instantiations of lift_reduce.hpp).
#include "lift_reduce.hpp"

namespace lift {

const void *reduce_kernel_f32(int op, int acc, int vec_bytes, int unroll)
{
    return pick_reduce<F32>(op, acc, vec_bytes, unroll);
}

}  // namespace lift
