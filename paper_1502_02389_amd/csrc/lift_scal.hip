// scal: out = map(mult(alpha), x)  (Fig. 5).
//
// Lowered as join o map-workgroup(asScalar o map-local(vect(mult(alpha)))
// o asVector) o split^chunk -- the structure of the paper's vector-scaling
// example (Fig. 2b) -- with VB-byte vectors, U loads in flight per lane, and
// a scalar head / tail so any element-aligned pointer pair works.  Every
// element gets exactly one binary32 multiply.  x is read and out written
// with nontemporal hints (each byte is touched once).
#include "lift_device.hpp"
#include "lift_internal.hpp"

namespace lift {

template <int VB>
__device__ __forceinline__ typename Vec<VB>::type scale_vec(typename Vec<VB>::type v, float alpha)
{
    if constexpr (VB == 4) {
        return __builtin_bit_cast(uint32_t, alpha * bits_to_float(v));
    } else {
#pragma unroll
        for (int i = 0; i < VB / 4; ++i)
            v[i] = __builtin_bit_cast(uint32_t, alpha * bits_to_float(v[i]));
        return v;
    }
}

template <int VB, int U>
__global__ void __launch_bounds__(1024) scal_kernel_t(ScalArgs a)
{
    constexpr int E = VB / 4;
    using V = typename Vec<VB>::type;
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const char *xv = reinterpret_cast<const char *>(a.x) + a.head * 4;
    char *ov = reinterpret_cast<char *>(a.out) + a.head * 4;

    const int64_t vbeg = (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = min(vbeg + a.chunk, a.nvec);
    const int64_t step = B * U;
    int64_t base = vbeg;
    for (; base + step <= vend; base += step) {
        V v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = load_stream<VB>(xv, base + t + k * B);
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k)
            store_stream<VB>(ov, base + t + k * B, scale_vec<VB>(v[k], a.alpha));
    }
    for (int64_t i = base + t; i < vend; i += B)
        store_stream<VB>(ov, i, scale_vec<VB>(load_stream<VB>(xv, i), a.alpha));

    if (blockIdx.x == 0 && t < a.head)
        a.out[t] = a.alpha * a.x[t];
    const int64_t tail0 = a.head + a.nvec * E;
    if (blockIdx.x == gridDim.x - 1 && t < a.n - tail0)
        a.out[tail0 + t] = a.alpha * a.x[tail0 + t];
}

template <int VB>
static const void *scal_pick_unroll(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&scal_kernel_t<VB, 1>);
    case 2: return reinterpret_cast<const void *>(&scal_kernel_t<VB, 2>);
    case 4: return reinterpret_cast<const void *>(&scal_kernel_t<VB, 4>);
    case 8: return reinterpret_cast<const void *>(&scal_kernel_t<VB, 8>);
    default: return nullptr;
    }
}

const void *scal_kernel(int vec_bytes, int unroll)
{
    switch (vec_bytes) {
    case 4: return scal_pick_unroll<4>(unroll);
    case 8: return scal_pick_unroll<8>(unroll);
    case 16: return scal_pick_unroll<16>(unroll);
    default: return nullptr;
    }
}

}  // namespace lift
