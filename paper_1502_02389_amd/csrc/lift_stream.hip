// Bandwidth reference kernels: a flat read and a flat copy of n floats.
//
// They carry none of the paper's arithmetic.  They exist to measure, with
// the same loads, launch shapes and partition as the library's own streaming
// kernels, what one launch of a given size can move on this device: the
// read kernel is asum without its per-element work and without the
// cross-work-group combine, the copy kernel is scal without its multiply.
// The difference between a reduction and the read kernel of the same bytes
// is what the reduction's own work (fold, tree, combine tail) costs.
//
// Read: every lane folds its 16-byte vectors with XOR (integer, one
// instruction per word) and writes its fold to `sink` only if it equals a
// fixed tag, which keeps every load live without a store per work-group.
// Copy: 16-byte nontemporal loads and stores, U in flight per lane.
#include "lift_device.hpp"
#include "lift_internal.hpp"

namespace lift {

constexpr uint32_t STREAM_SINK_TAG = 0x5eed1e55u;

template <int U>
__global__ void __launch_bounds__(1024) stream_read_kernel(StreamArgs a)
{
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const int64_t step = B * U;
    const int64_t vbeg = a.interleave ? (int64_t)blockIdx.x * step : (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = a.interleave ? a.nvec : min(vbeg + a.chunk, a.nvec);
    const int64_t stride = a.interleave ? (int64_t)gridDim.x * step : step;
    u32x4 acc = {0u, 0u, 0u, 0u};
    int64_t base = vbeg;
    for (; base + step <= vend; base += stride) {
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = load_stream<16>(a.x, base + t + k * B);
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k)
            acc ^= v[k];
    }
    if (base < vend) {
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = load_stream<16>(a.x, min(base + t + k * B, vend - 1));
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (base + t + k * B < vend)
                acc ^= v[k];
    }
    const uint32_t f = (acc[0] ^ acc[1]) ^ (acc[2] ^ acc[3]);
    if (f == STREAM_SINK_TAG)
        *reinterpret_cast<uint32_t *>(a.out) = f;
}

template <int U>
__global__ void __launch_bounds__(1024) stream_copy_kernel(StreamArgs a)
{
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const int64_t step = B * U;
    const int64_t vbeg = a.interleave ? (int64_t)blockIdx.x * step : (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = a.interleave ? a.nvec : min(vbeg + a.chunk, a.nvec);
    const int64_t stride = a.interleave ? (int64_t)gridDim.x * step : step;
    int64_t base = vbeg;
    for (; base + step <= vend; base += stride) {
        u32x4 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = load_stream<16>(a.x, base + t + k * B);
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k)
            store_stream<16>(a.out, base + t + k * B, v[k]);
    }
    for (int64_t i = base + t; i < vend; i += B)
        store_stream<16>(a.out, i, load_stream<16>(a.x, i));
}

const void *stream_kernel(bool copy, int unroll)
{
    switch (unroll) {
    case 1: return copy ? (const void *)&stream_copy_kernel<1> : (const void *)&stream_read_kernel<1>;
    case 2: return copy ? (const void *)&stream_copy_kernel<2> : (const void *)&stream_read_kernel<2>;
    case 4: return copy ? (const void *)&stream_copy_kernel<4> : (const void *)&stream_read_kernel<4>;
    case 8: return copy ? (const void *)&stream_copy_kernel<8> : (const void *)&stream_read_kernel<8>;
    default: return nullptr;
    }
}

}  // namespace lift
