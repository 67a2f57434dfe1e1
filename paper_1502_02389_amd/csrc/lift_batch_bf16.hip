// Batched-form kernels for BF16 storage (instantiations of lift_batch.hpp).
#include "lift_batch.hpp"

namespace lift {

const void *batch_kernel_bf16(int acc, int vec_bytes, int unroll, bool gemv)
{
    return pick_batch<BF16>(acc, vec_bytes, unroll, gemv);
}

const void *batch_stamped_bf16(int vec_bytes, int unroll, bool gemv)
{
    return pick_batch_stamped<BF16>(vec_bytes, unroll, gemv);
}

}  // namespace lift
