// asum / dot kernels for BF16 storage (instantiations of lift_reduce.hpp).
#include "lift_reduce.hpp"

namespace lift {

const void *reduce_kernel_bf16(int op, int acc, int vec_bytes, int unroll)
{
    return pick_reduce<BF16>(op, acc, vec_bytes, unroll);
}

}  // namespace lift
