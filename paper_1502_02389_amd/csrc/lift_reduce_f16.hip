// asum / dot kernels for F16 storage (instantiations of lift_reduce.hpp).
#include "lift_reduce.hpp"

namespace lift {

const void *reduce_kernel_f16(int op, int acc, int vec_bytes, int unroll)
{
    return pick_reduce<F16>(op, acc, vec_bytes, unroll);
}

}  // namespace lift
