// gemv kernels for BF16 storage of A (instantiations of lift_gemv.hpp).
#include "lift_gemv.hpp"

namespace lift {

const void *gemv_kernel_bf16(int acc, int vec_bytes, int rows, int unroll)
{
    return pick_gemv<BF16>(acc, vec_bytes, rows, unroll);
}

const void *gemv_split_kernel_bf16(int acc, int vec_bytes, int rows, int unroll, bool x_stationary)
{
    return pick_gemv_split<BF16>(acc, vec_bytes, rows, unroll, x_stationary);
}

}  // namespace lift
