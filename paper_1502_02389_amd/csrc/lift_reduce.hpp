// asum and dot: one streaming pass, one launch.
//
// The kernel is the paper's fused reduction (the asum derivation of Fig. 8,
// eq. 8, and the GPU expressions of Fig. 9) laid out for CDNA4:
//
//   reduce-seq o join o map-workgroup(
//       toGlobal(...)                              partial -> workspace slot
//     o iterate(part-red) with toLocal             DPP wave butterfly + LDS
//     o map-local(reduce-seq(lambda acc, a: acc + term(a), 0))
//     o split o reorder-stride                     lane t reads vector t, t+B, ..
//   ) o asVector o split^chunk                      dwordx4 loads, chunk per WG
//
// term(a) = |a| (asum) or a_x * a_y (dot, zip fused into the load).  The
// final reduce-seq o join runs in the same launch: every work-group stores
// its partial, then counts in on agent-scope arrival counters (two levels,
// see arrive()); in the one that arrives last, one wavefront folds all
// partials (lane t: partials t, t + 64, ...; then the wave butterfly) and
// writes the result, then resets the counter for the next call.  No float
// atomics
// and no inter-work-group waiting, so the result is deterministic and the
// grid always drains.
//
// Cross-XCD visibility without cache maintenance: the partials are written
// and read with agent-scope atomic stores / loads, which gfx950 performs
// device-coherently (write-through / miss in the per-XCD L2), and a
// work-group counts in only once its partial's store has completed.  An agent-scope
// release/acquire fence would instead write back and invalidate the whole
// L2 of the XCD in every work-group.
#pragma once

#include "lift_device.hpp"
#include "lift_internal.hpp"

namespace lift {

// Per-lane accumulator of the streaming phase.
template <int ACC, int E>
struct LaneAcc;

// binary32: E independent sums (one per vector component), folded pairwise
// at the end.
template <int E>
struct LaneAcc<ACC_F32, E> {
    float s[E];
    __device__ __forceinline__ LaneAcc()
    {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] = 0.f;
    }
    // asum / dot-with-product-given
    __device__ __forceinline__ void add_terms(const float *t)
    {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] += t[e];
    }
    __device__ __forceinline__ void add_products(const float *a, const float *b)
    {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] = fmaf(a[e], b[e], s[e]);
    }
    __device__ __forceinline__ void add_scalar(float v) { s[0] += v; }
    __device__ __forceinline__ void add_scalar_product(float a, float b) { s[0] = fmaf(a, b, s[0]); }
    __device__ __forceinline__ float value() const
    {
        float t[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            t[e] = s[e];
#pragma unroll
        for (int w = 1; w < E; w <<= 1)
#pragma unroll
            for (int e = 0; e + w < E; e += 2 * w)
                t[e] = t[e] + t[e + w];
        return t[0];
    }
};

// binary32 with a binary64 cross-work-group combine: same lane arithmetic.
template <int E>
struct LaneAcc<ACC_F64, E> : LaneAcc<ACC_F32, E> {};

// Compensated: the E terms of one load are summed pairwise, then added to
// the lane's (sum, error) pair with TwoSum; binary32 products contribute
// their exact rounding error (fma(a, b, -a*b), the TwoProduct of Ogita,
// Rump and Oishi) to the error term.
template <int E>
struct LaneAcc<ACC_COMP, E> {
    Pair p{0.f, 0.f};
    __device__ __forceinline__ static float tree(float *t)
    {
#pragma unroll
        for (int w = 1; w < E; w <<= 1)
#pragma unroll
            for (int e = 0; e + w < E; e += 2 * w)
                t[e] = t[e] + t[e + w];
        return t[0];
    }
    __device__ __forceinline__ void add_terms(const float *t)
    {
        float u[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            u[e] = t[e];
        p = pair_add(p, tree(u));
    }
    template <bool EXACT_PRODUCTS>
    __device__ __forceinline__ void add_products_c(const float *a, const float *b)
    {
        float q[E], r[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            q[e] = a[e] * b[e];
            r[e] = EXACT_PRODUCTS ? 0.f : fmaf(a[e], b[e], -q[e]);
        }
        p = pair_add(p, tree(q));
        if (!EXACT_PRODUCTS)
            p.c += tree(r);
    }
    __device__ __forceinline__ void add_scalar(float v) { p = pair_add(p, v); }
    template <bool EXACT_PRODUCTS>
    __device__ __forceinline__ void add_scalar_product_c(float a, float b)
    {
        float q = a * b;
        p = pair_add(p, q);
        if (!EXACT_PRODUCTS)
            p.c += fmaf(a, b, -q);
    }
    __device__ __forceinline__ Pair value() const { return p; }
};

// Partial slot type written by each work-group.
template <int ACC> struct SlotT { using type = float; };
template <> struct SlotT<ACC_COMP> { using type = Pair; };
template <> struct SlotT<ACC_F64> { using type = double; };

template <int ACC> struct BlockT { using type = float; };
template <> struct BlockT<ACC_COMP> { using type = Pair; };

__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(Pair p) { return (double)p.s + (double)p.c; }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(double v) { return (float)v; }
__device__ __forceinline__ float to_f32(Pair p) { return p.s + p.c; }

template <int ACC>
__device__ __forceinline__ typename SlotT<ACC>::type to_slot(typename BlockT<ACC>::type v)
{
    return typename SlotT<ACC>::type(v);
}
template <>
__device__ __forceinline__ Pair to_slot<ACC_COMP>(Pair v)
{
    return v;
}

template <class S>
__device__ __forceinline__ S zero_of();
template <> __device__ __forceinline__ float zero_of<float>() { return 0.f; }
template <> __device__ __forceinline__ double zero_of<double>() { return 0.0; }
template <> __device__ __forceinline__ Pair zero_of<Pair>() { return Pair{0.f, 0.f}; }

// Agent-coherent (all XCDs) store / load of a partial slot.
__device__ __forceinline__ void store_coherent(char *p, float v)
{
    __hip_atomic_store(reinterpret_cast<uint32_t *>(p), __builtin_bit_cast(uint32_t, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(char *p, double v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(char *p, Pair v)
{
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}
template <class S>
__device__ __forceinline__ S load_coherent(const char *p);
template <>
__device__ __forceinline__ float load_coherent<float>(const char *p)
{
    return __builtin_bit_cast(float, __hip_atomic_load(reinterpret_cast<const uint32_t *>(p), __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT));
}
template <>
__device__ __forceinline__ double load_coherent<double>(const char *p)
{
    return __builtin_bit_cast(double, __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT));
}
template <>
__device__ __forceinline__ Pair load_coherent<Pair>(const char *p)
{
    return __builtin_bit_cast(Pair, __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
}

// Two-level arrival of this work-group (called by one thread, after its
// partial's store has completed).  Work-group b counts in on the group
// counter at group_base + (b / ARRIVAL_GROUP) * WS_GROUP_STRIDE; the last of
// a group resets that counter and counts the group in on `global`.  Returns
// true in the one work-group that arrives last overall; by then every
// partial is stored.  The caller resets `global`.
__device__ __forceinline__ bool arrive(unsigned *global, char *group_base)
{
    const unsigned g = blockIdx.x / ARRIVAL_GROUP;
    const unsigned groups = (gridDim.x + ARRIVAL_GROUP - 1) / ARRIVAL_GROUP;
    const unsigned size = min((unsigned)ARRIVAL_GROUP, gridDim.x - g * ARRIVAL_GROUP);
    unsigned *gc = reinterpret_cast<unsigned *>(group_base + g * WS_GROUP_STRIDE);
    unsigned prev = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev != size - 1)
        return false;
    __hip_atomic_store(gc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    prev = __hip_atomic_fetch_add(global, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return prev == groups - 1;
}

template <class S>
__device__ __forceinline__ void write_result(void *result, int f64, S v)
{
    if (f64)
        *reinterpret_cast<double *>(result) = to_f64(v);
    else
        *reinterpret_cast<float *>(result) = to_f32(v);
}

// 16-bit products are exact in binary32 (8- or 11-bit significands).
template <class T> struct ExactProducts { static constexpr bool value = T::bytes == 2; };

template <class T, int OP, int ACC, int E>
__device__ __forceinline__ void accumulate(LaneAcc<ACC, E> &acc, const float *a, const float *b)
{
    if constexpr (OP == OP_ASUM) {
        float t[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            t[e] = fabsf(a[e]);
        acc.add_terms(t);
    } else if constexpr (ACC == ACC_COMP) {
        acc.template add_products_c<ExactProducts<T>::value>(a, b);
    } else {
        acc.add_products(a, b);
    }
}

template <class T, int OP, int ACC, int E>
__device__ __forceinline__ void accumulate_scalar(LaneAcc<ACC, E> &acc, float a, float b)
{
    if constexpr (OP == OP_ASUM) {
        acc.add_scalar(fabsf(a));
    } else if constexpr (ACC == ACC_COMP) {
        acc.template add_scalar_product_c<ExactProducts<T>::value>(a, b);
    } else {
        acc.add_scalar_product(a, b);
    }
}

// Clock reading for the stamped instances (s_memrealtime: 100 MHz, shared
// by all XCDs), written by thread 0 with an ordinary vector store.
template <bool STAMP>
__device__ __forceinline__ void stamp(const ReduceArgs &a, int k)
{
    if constexpr (STAMP) {
        if (threadIdx.x == 0)
            a.stamps[(int64_t)blockIdx.x * STAMPS_PER_WG + k] = (uint64_t)wall_clock64();
    }
}

// Stamped instances, thread 0 of a work-group whose arrival is counted:
// the arrival time (also its end, unless it combines), its ids and whether
// it combines.  A single work-group stamps its partial's store here too.
template <bool STAMP>
__device__ __forceinline__ void stamp_arrival(const ReduceArgs &a, int last)
{
    if constexpr (STAMP) {
        __builtin_amdgcn_sched_barrier(0);
        uint64_t *w = a.stamps + (int64_t)blockIdx.x * STAMPS_PER_WG;
        const uint64_t now = (uint64_t)wall_clock64();
        if (gridDim.x == 1)
            w[3] = now;
        w[4] = now;
        w[5] = now;
        const uint32_t xcc = __builtin_amdgcn_s_getreg((20 << 0) | (0 << 6) | (3 << 11));  // XCC_ID[3:0]
        const uint32_t hw = __builtin_amdgcn_s_getreg((4 << 0) | (8 << 6) | (7 << 11));    // HW_ID[15:8]: CU, SH, SE
        w[6] = ((uint64_t)(unsigned)last << 32) | ((uint64_t)xcc << 16) | hw;
    }
}

// The work-group's partial wg (valid in thread 0; every thread calls this
// after the work-group tree) goes to the combine: with one work-group it is
// the result; else it is stored to its slot and counted in, and in the
// work-group that arrives last one wavefront folds all partials -- lane t
// folds partials t, t + 64, t + 128, ... in that order (COMBINE_LOADS loads
// in flight), then the wave butterfly -- and writes the result.  No barrier
// on this path.
template <int ACC, bool STAMP>
__device__ __forceinline__ void combine_partials(const ReduceArgs &a, typename BlockT<ACC>::type wg)
{
    using ST = typename SlotT<ACC>::type;
    const int t = threadIdx.x;
    if (gridDim.x == 1) {
        if (t == 0) {
            write_result(a.result, a.result_f64, wg);
            stamp_arrival<STAMP>(a, 1);  // the only work-group combines: stored, arrived and done at once
        }
        return;
    }

    // The rest is wave 0's: the other waves are done once the tree has their
    // values (block_sum ends with a barrier).
    if (t >= 64)
        return;
    char *slots = reinterpret_cast<char *>(a.ws) + WS_HEADER;  // 16-byte slots
    int last = 0;
    if (t == 0) {
        store_coherent(slots + (int64_t)blockIdx.x * WS_SLOT, to_slot<ACC>(wg));
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);  // the partial's store has completed
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if constexpr (STAMP) {
            __builtin_amdgcn_sched_barrier(0);
            stamp<STAMP>(a, 3);
            __builtin_amdgcn_sched_barrier(0);
        }
        last = arrive(reinterpret_cast<unsigned *>(a.ws), reinterpret_cast<char *>(a.ws) + WS_GROUPS) ? 1 : 0;
        stamp_arrival<STAMP>(a, last);  // after the arrival's atomics have returned (last depends on them)
    }
    last = __builtin_amdgcn_readfirstlane(last);  // lane 0's decision, for the whole wave
    if (!last)
        return;

    // the final reduce-seq o join, by this wavefront
    constexpr int COMBINE_LOADS = 8;
    const int64_t G = gridDim.x;
    ST v = zero_of<ST>();
    for (int64_t base = 0; base < G; base += 64 * COMBINE_LOADS) {
        ST p[COMBINE_LOADS];
#pragma unroll
        for (int k = 0; k < COMBINE_LOADS; ++k)
            p[k] = load_coherent<ST>(slots + min(base + t + 64 * k, G - 1) * WS_SLOT);
#pragma unroll
        for (int k = 0; k < COMBINE_LOADS; ++k)
            if (base + t + 64 * k < G)
                v = merge(v, p[k]);
    }
    v = wave_sum(v);
    if (t == 0) {
        write_result(a.result, a.result_f64, v);
        __hip_atomic_store(reinterpret_cast<unsigned *>(a.ws), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if constexpr (STAMP) {
        __builtin_amdgcn_sched_barrier(0);
        stamp<STAMP>(a, 5);
    }
}

template <class T, int OP, int ACC, int VB, int U, bool STAMP = false>
__global__ void __launch_bounds__(1024) reduce_kernel(ReduceArgs a)
{
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    using BT = typename BlockT<ACC>::type;
    __shared__ BT lds_block[16];

    stamp<STAMP>(a, 0);
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const char *xv = reinterpret_cast<const char *>(a.x) + a.head * T::bytes;
    const char *yv = OP == OP_DOT ? reinterpret_cast<const char *>(a.y) + a.head * T::bytes : nullptr;

    // The work-group's steps of B * U vectors: one contiguous chunk
    // (split^chunk), or every G-th step starting at its own (the chunking of
    // a reorder-stride-G over steps: all work-groups then stream neighbouring
    // steps at the same time).
    const int64_t step = B * U;
    const int64_t vbeg = a.interleave ? (int64_t)blockIdx.x * step : (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = a.interleave ? a.nvec : min(vbeg + a.chunk, a.nvec);
    const int64_t stride = a.interleave ? (int64_t)gridDim.x * step : step;

    LaneAcc<ACC, E> acc;
    int64_t base = vbeg;
    // full steps: U independent loads per lane (per operand) in flight
    for (; base + step <= vend; base += stride) {
        V vx[U], vy[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            vx[k] = load_stream<VB>(xv, base + t + k * B);
            if constexpr (OP == OP_DOT)
                vy[k] = load_stream<VB>(yv, base + t + k * B);
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
    // the last, partial step of this work-group
    if (base < vend) {
        // Final partial step: fewer than U vectors per lane.  Every lane loads
        // U vectors at clamped (in-range) indices so all loads are in flight
        // without branches; the ones past the end are replaced by zeros, which
        // leave every sum unchanged.
        V vx[U], vy[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = min(base + t + k * B, vend - 1);
            vx[k] = load_stream<VB>(xv, i);
            if constexpr (OP == OP_DOT)
                vy[k] = load_stream<VB>(yv, i);
        }
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool in = base + t + k * B < vend;
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
    // scalar head (work-group 0) and tail (last work-group), fewer than E each
    if (blockIdx.x == 0 && t < a.head) {
        float fy = OP == OP_DOT ? load_elem<T>(a.y, t) : 0.f;
        accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(a.x, t), fy);
    }
    const int64_t tail0 = a.head + a.nvec * E;
    if (blockIdx.x == gridDim.x - 1 && t < a.n - tail0) {
        float fy = OP == OP_DOT ? load_elem<T>(a.y, tail0 + t) : 0.f;
        accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(a.x, tail0 + t), fy);
    }

    if constexpr (STAMP) {  // every load of the streaming loop has been consumed
        __builtin_amdgcn_sched_barrier(0);
        stamp<STAMP>(a, 1);
        __builtin_amdgcn_sched_barrier(0);
    }
    BT wg = block_sum<BT>(acc.value(), lds_block);
    stamp<STAMP>(a, 2);
    combine_partials<ACC, STAMP>(a, wg);
}

// Table of instantiated reduce kernels for storage T.
template <class T, int OP, int ACC, int VB>
const void *pick_unroll(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&reduce_kernel<T, OP, ACC, VB, 1>);
    case 2: return reinterpret_cast<const void *>(&reduce_kernel<T, OP, ACC, VB, 2>);
    case 4: return reinterpret_cast<const void *>(&reduce_kernel<T, OP, ACC, VB, 4>);
    case 8: return reinterpret_cast<const void *>(&reduce_kernel<T, OP, ACC, VB, 8>);
    default: return nullptr;
    }
}

template <class T, int OP, int ACC>
const void *pick_vec(int vec_bytes, int unroll)
{
    switch (vec_bytes) {
    case 2:
        if constexpr (T::bytes == 2)
            return pick_unroll<T, OP, ACC, 2>(unroll);
        return nullptr;
    case 4: return pick_unroll<T, OP, ACC, 4>(unroll);
    case 8: return pick_unroll<T, OP, ACC, 8>(unroll);
    case 16: return pick_unroll<T, OP, ACC, 16>(unroll);
    default: return nullptr;
    }
}

template <class T, int OP>
const void *pick_acc(int acc, int vec_bytes, int unroll)
{
    switch (acc) {
    case ACC_F32: return pick_vec<T, OP, ACC_F32>(vec_bytes, unroll);
    case ACC_COMP: return pick_vec<T, OP, ACC_COMP>(vec_bytes, unroll);
    case ACC_F64: return pick_vec<T, OP, ACC_F64>(vec_bytes, unroll);
    default: return nullptr;
    }
}

template <class T>
const void *pick_reduce(int op, int acc, int vec_bytes, int unroll)
{
    if (op == OP_ASUM)
        return pick_acc<T, OP_ASUM>(acc, vec_bytes, unroll);
    if (op == OP_DOT)
        return pick_acc<T, OP_DOT>(acc, vec_bytes, unroll);
    return nullptr;
}

// The stamped instances (binary32 storage and accumulation, 16-byte loads).
template <int OP>
const void *pick_stamped(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&reduce_kernel<F32, OP, ACC_F32, 16, 1, true>);
    case 2: return reinterpret_cast<const void *>(&reduce_kernel<F32, OP, ACC_F32, 16, 2, true>);
    case 4: return reinterpret_cast<const void *>(&reduce_kernel<F32, OP, ACC_F32, 16, 4, true>);
    case 8: return reinterpret_cast<const void *>(&reduce_kernel<F32, OP, ACC_F32, 16, 8, true>);
    default: return nullptr;
    }
}

}  // namespace lift
