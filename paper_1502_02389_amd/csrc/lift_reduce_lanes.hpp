// asum and dot in the other lane forms of the derivation space.
//
// Section 6.2 lowers the work-group's share of a reduction in either of two
// ways at each of two places: the lanes take the chunk through
// reorder-stride (lane t: vectors t, t + B, ...; coalesced, the library's
// default kernel) or through a plain split (lane t: the t-th contiguous run
// of C / B vectors), and the B lane partials meet in the iterate tree or in
// one reduce-seq (Fig. 9c's expression is the last with a single lane).
// This kernel executes the three forms besides the default, so every
// expression the derivation search reaches has a launch:
//
//   RUNS = false, SEQ = true   reorder-stride lanes, lanes folded in order
//   RUNS = true,  SEQ = false  contiguous runs, tree over the lanes
//   RUNS = true,  SEQ = true   contiguous runs, lanes folded in order
//
// Work-group b takes vectors [b C, (b + 1) C) (the chunk partition); a lane
// folds its vectors in increasing order with U loads in flight (for runs: U
// consecutive vectors of its run per step).  The scalar head elements go to
// lanes i mod B of work-group 0 and the tail elements to lanes i mod B of
// the last one, in order.  With B >= 64 the work-group partials meet in the
// default kernel's combine (one wavefront: lane t folds partials t, t + 64,
// ..., then the butterfly); with B < 64 (sequential forms only) lane t of
// the last work-group folds partials t, t + B, ... and the B lane values
// meet in a pairwise tree.  binary32 accumulation only.
#pragma once

#include "lift_reduce.hpp"

namespace lift {

template <class T, int OP, int VB, int U, bool RUNS, bool SEQ>
__global__ void __launch_bounds__(1024) reduce_lanes_kernel(ReduceArgs a)
{
    constexpr int ACC = ACC_F32;
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    __shared__ float lds_block[16];
    __shared__ float lds_lane[SEQ ? 1024 : 64];
    __shared__ int s_last;

    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const char *xv = reinterpret_cast<const char *>(a.x) + a.head * T::bytes;
    const char *yv = OP == OP_DOT ? reinterpret_cast<const char *>(a.y) + a.head * T::bytes : nullptr;
    const int64_t vbeg = (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = min(vbeg + a.chunk, a.nvec);

    // the lane's vectors: [lo, hi) with stride ls, in steps of U loads
    int64_t lo, hi, ls, step;
    if constexpr (RUNS) {
        const int64_t per = a.chunk / B;   // the host keeps chunk a multiple of B * U
        lo = vbeg + t * per;
        hi = min(lo + per, vend);
        ls = 1;
        step = U;
    } else {
        lo = vbeg + t;
        hi = vend;
        ls = B;
        step = B * U;
    }

    LaneAcc<ACC, E> acc;
    int64_t base = lo;
    for (; base + (U - 1) * ls < hi; base += step) {
        V vx[U], vy[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            vx[k] = load_stream<VB>(xv, base + k * ls);
            if constexpr (OP == OP_DOT)
                vy[k] = load_stream<VB>(yv, base + k * ls);
        }
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k) {
            float fx[E], fy[E];
            decode<T, VB>(vx[k], fx);
            if constexpr (OP == OP_DOT)
                decode<T, VB>(vy[k], fy);
            accumulate<T, OP, ACC, E>(acc, fx, fy);
        }
    }
    if (base < hi) {
        // the last, partial step: loads at clamped indices, zeros past the end
        V vx[U], vy[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = min(base + k * ls, hi - 1);
            vx[k] = load_stream<VB>(xv, i);
            if constexpr (OP == OP_DOT)
                vy[k] = load_stream<VB>(yv, i);
        }
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool in = base + k * ls < hi;
            float fx[E], fy[E];
            decode<T, VB>(vx[k], fx);
            if constexpr (OP == OP_DOT)
                decode<T, VB>(vy[k], fy);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                fx[e] = in ? fx[e] : 0.f;
                if constexpr (OP == OP_DOT)
                    fy[e] = in ? fy[e] : 0.f;
            }
            accumulate<T, OP, ACC, E>(acc, fx, fy);
        }
    }
    if (blockIdx.x == 0)
        for (int64_t i = t; i < a.head; i += B) {
            const float fy = OP == OP_DOT ? load_elem<T>(a.y, i) : 0.f;
            accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(a.x, i), fy);
        }
    const int64_t tail0 = a.head + a.nvec * E;
    if (blockIdx.x == gridDim.x - 1)
        for (int64_t i = t; i < a.n - tail0; i += B) {
            const float fy = OP == OP_DOT ? load_elem<T>(a.y, tail0 + i) : 0.f;
            accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(a.x, tail0 + i), fy);
        }

    // the lane partials meet: in lane order (one thread), or in the tree
    float wg;
    if constexpr (SEQ) {
        lds_lane[t] = acc.value();
        __syncthreads();
        wg = lds_lane[0];
        if (t == 0)
            for (int64_t i = 1; i < B; ++i)
                wg = wg + lds_lane[i];
        __syncthreads();  // lds_lane is free again (the small combine reuses it)
    } else {
        wg = block_sum<float>(acc.value(), lds_block);
    }
    if (!SEQ || B >= 64) {   // tree forms run 64 or more lanes (the host checks)
        combine_partials<ACC, false>(a, wg);
        return;
    }

    // B < 64 (sequential forms): the combine over B lanes
    if (gridDim.x == 1) {
        if (t == 0)
            write_result(a.result, a.result_f64, wg);
        return;
    }
    char *slots = reinterpret_cast<char *>(a.ws) + WS_HEADER;
    if (t == 0) {
        store_coherent(slots + (int64_t)blockIdx.x * WS_SLOT, wg);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);  // the partial's store has completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        s_last = arrive(reinterpret_cast<unsigned *>(a.ws), reinterpret_cast<char *>(a.ws) + WS_GROUPS) ? 1 : 0;
    }
    __syncthreads();
    if (!s_last)
        return;
    const int64_t G = gridDim.x;
    float v = 0.f;
    for (int64_t i = t; i < G; i += B)
        v = v + load_coherent<float>(slots + i * WS_SLOT);
    lds_lane[t] = v;
    __syncthreads();
    if (t == 0) {
        // pairwise over the B (a power of two) lane values, adjacent pairs
        // at each level
        for (int64_t w = 1; w < B; w <<= 1)
            for (int64_t e = 0; e + w < B; e += 2 * w)
                lds_lane[e] = lds_lane[e] + lds_lane[e + w];
        write_result(a.result, a.result_f64, lds_lane[0]);
        __hip_atomic_store(reinterpret_cast<unsigned *>(a.ws), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <class T, int OP, int VB, int U>
const void *pick_lanes_form(int form)
{
    switch (form) {
    case 1: return reinterpret_cast<const void *>(&reduce_lanes_kernel<T, OP, VB, U, false, true>);
    case 2: return reinterpret_cast<const void *>(&reduce_lanes_kernel<T, OP, VB, U, true, false>);
    case 3: return reinterpret_cast<const void *>(&reduce_lanes_kernel<T, OP, VB, U, true, true>);
    default: return nullptr;
    }
}

template <class T, int OP, int VB>
const void *pick_lanes_unroll(int unroll, int form)
{
    switch (unroll) {
    case 1: return pick_lanes_form<T, OP, VB, 1>(form);
    case 2: return pick_lanes_form<T, OP, VB, 2>(form);
    case 4: return pick_lanes_form<T, OP, VB, 4>(form);
    case 8: return pick_lanes_form<T, OP, VB, 8>(form);
    default: return nullptr;
    }
}

template <class T, int OP>
const void *pick_lanes_vec(int vec_bytes, int unroll, int form)
{
    switch (vec_bytes) {
    case 2:
        if constexpr (T::bytes == 2)
            return pick_lanes_unroll<T, OP, 2>(unroll, form);
        else
            return nullptr;
    case 4: return pick_lanes_unroll<T, OP, 4>(unroll, form);
    case 8: return pick_lanes_unroll<T, OP, 8>(unroll, form);
    case 16: return pick_lanes_unroll<T, OP, 16>(unroll, form);
    default: return nullptr;
    }
}

template <class T>
const void *pick_lanes(int op, int vec_bytes, int unroll, int form)
{
    return op == OP_DOT ? pick_lanes_vec<T, OP_DOT>(vec_bytes, unroll, form)
                        : pick_lanes_vec<T, OP_ASUM>(vec_bytes, unroll, form);
}

}  // namespace lift
