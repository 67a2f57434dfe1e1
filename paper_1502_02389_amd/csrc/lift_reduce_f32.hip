// asum / dot kernels for F32 storage (instantiations of lift_reduce.hpp).
#include "lift_reduce.hpp"

namespace lift {

const void *reduce_kernel_f32(int op, int acc, int vec_bytes, int unroll)
{
    return pick_reduce<F32>(op, acc, vec_bytes, unroll);
}

const void *reduce_kernel_stamped_f32(int op, int unroll)
{
    return op == OP_DOT ? pick_stamped<OP_DOT>(unroll) : pick_stamped<OP_ASUM>(unroll);
}

}  // namespace lift
