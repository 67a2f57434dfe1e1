// Batched-form kernels for F32 storage (instantiations of lift_batch.hpp).
#include "lift_batch.hpp"

namespace lift {

const void *batch_kernel_f32(int acc, int vec_bytes, int unroll, bool gemv)
{
    return pick_batch<F32>(acc, vec_bytes, unroll, gemv);
}

const void *batch_stamped_f32(int vec_bytes, int unroll, bool gemv)
{
    return pick_batch_stamped<F32>(vec_bytes, unroll, gemv);
}

}  // namespace lift
