// gemv: y = alpha * A x + beta * y, row-major A.
//
// The paper's program maps scal(alpha) o dot(x) over the rows of A and then
// zips the result with scal(beta, y) (Fig. 5).  Here one wavefront owns R
// rows at a time (map over rows -> map-wavefront); inside a row the 64 lanes
// read consecutive VB-byte vectors (reorder-stride: lane l takes vectors
// l, l+64, ...), each lane folds its products with reduce-seq, and a DPP
// butterfly (iterate of part-red) yields the row's dot.  The R rows of a
// wavefront share every x load, which divides x traffic by R.  A is read
// once with nontemporal loads; x stays cache-resident.  alpha scales
// the finished dot once, and the zip with beta*y is fused into the store.
#pragma once

#include "lift_device.hpp"
#include "lift_internal.hpp"
#include "lift_reduce.hpp"

#include <type_traits>

namespace lift {

// E consecutive binary32 values of x starting at element E * v.
template <int E>
__device__ __forceinline__ void load_x(const float *x, int64_t v, float *o)
{
    if constexpr (E == 1) {
        o[0] = x[v];
    } else if constexpr (E == 2) {
        u32x2 w = load_vec<8>(x, v);
        o[0] = bits_to_float(w[0]);
        o[1] = bits_to_float(w[1]);
    } else {
#pragma unroll
        for (int h = 0; h < E / 4; ++h) {
            u32x4 w = load_vec<16>(x, v * (E / 4) + h);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                o[4 * h + i] = bits_to_float(w[i]);
        }
    }
}

template <int ACC, int E>
struct RowAcc;

template <int E>
struct RowAcc<ACC_F32, E> {
    float s[E];
    __device__ __forceinline__ RowAcc()
    {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] = 0.f;
    }
    __device__ __forceinline__ void add(const float *a, const float *x)
    {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] = fmaf(a[e], x[e], s[e]);
    }
    __device__ __forceinline__ void add_scalar(float a, float x) { s[0] = fmaf(a, x, s[0]); }
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

template <int E>
struct RowAcc<ACC_F64, E> : RowAcc<ACC_F32, E> {};

// Compensated: products split exactly into a*x = q + r (TwoProduct via fma),
// q summed pairwise per load and added with TwoSum, r into the error term.
template <int E>
struct RowAcc<ACC_COMP, E> {
    Pair p{0.f, 0.f};
    __device__ __forceinline__ void add(const float *a, const float *x)
    {
        float q[E], r[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            q[e] = a[e] * x[e];
            r[e] = fmaf(a[e], x[e], -q[e]);
        }
#pragma unroll
        for (int w = 1; w < E; w <<= 1)
#pragma unroll
            for (int e = 0; e + w < E; e += 2 * w) {
                q[e] = q[e] + q[e + w];
                r[e] = r[e] + r[e + w];
            }
        p = pair_add(p, q[0]);
        p.c += r[0];
    }
    __device__ __forceinline__ void add_scalar(float a, float x)
    {
        float q = a * x;
        p = pair_add(p, q);
        p.c += fmaf(a, x, -q);
    }
    __device__ __forceinline__ Pair value() const { return p; }
};

// Largest work-group an instance is compiled for.  R x U vector loads,
// U x E values of x and the R values of y read ahead are live at once; the
// register estimate below keeps
// every instance within the budget its launch bound grants (1024 threads:
// 128 registers per lane, 512: 256, 256: 512) so none spills.  The host
// reads the bound back from the kernel and lowers the work-group size to it.
template <class T, int ACC, int VB, int R, int U>
constexpr int gemv_bound()
{
    constexpr int E = Elems<T, VB>::value;
    constexpr int load_regs = R * U * (VB < 4 ? 2 : VB / 4);  // sub-dword loads: value + address
    constexpr int acc_regs = ACC == ACC_COMP ? R * 2 + 2 * E : R * E;
    constexpr int regs = load_regs + U * E + acc_regs + R;
    return regs <= 64 ? 1024 : regs <= 200 ? 512 : 256;
}

template <int ACC>
__device__ __forceinline__ void store_row(float *y, int64_t i, float alpha, float beta, float dotv)
{
    float by = beta == 0.f ? 0.f : beta * y[i];
    y[i] = fmaf(alpha, dotv, by);
}

// The same epilogue with y_i already read (`yold`, ignored when beta is 0).
template <int ACC>
__device__ __forceinline__ void store_row_y(float *y, int64_t i, float alpha, float beta, float dotv, float yold)
{
    float by = beta == 0.f ? 0.f : beta * yold;
    y[i] = fmaf(alpha, dotv, by);
}

// y_i of a row about to be reduced, read before the row's loads so that the
// epilogue does not wait a dependent round trip (0 when beta is 0: y is not
// read, as BLAS specifies, or when the row is past the end).
__device__ __forceinline__ float prefetch_y(const float *y, int64_t i, int64_t m, float beta)
{
    return beta != 0.f && i < m ? y[i] : 0.f;
}

// Rows r0 .. r0 + R - 1 (clamped to m) of y = alpha * A x + beta * y, by one
// wavefront; `lane` is the lane index.  nvec = whole VB-byte vectors per row.
template <class T, int ACC, int VB, int R, int U>
__device__ __forceinline__ void gemv_row_group(const void *A, const float *x, float *y, int64_t m, int64_t n,
                                               int64_t lda, int64_t nvec, float alpha, float beta, int64_t r0,
                                               int lane)
{
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    const int64_t row_bytes = lda * T::bytes;
    const int64_t tail0 = nvec * E;
    const char *rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        rows[r] = reinterpret_cast<const char *>(A) + min(r0 + r, m - 1) * row_bytes;
    float yold[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        yold[r] = prefetch_y(y, r0 + r, m, beta);

    RowAcc<ACC, E> acc[R];
    int64_t base = 0;
    for (; base + 64 * U <= nvec; base += 64 * U) {
        float xf[U][E];
        V va[R][U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            load_x<E>(x, base + lane + 64 * k, xf[k]);
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < U; ++k)
                va[r][k] = load_stream<VB>(rows[r], base + lane + 64 * k);
        loads_in_flight();
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < U; ++k) {
                float af[E];
                decode<T, VB>(va[r][k], af);
                acc[r].add(af, xf[k]);
            }
    }
    if (base < nvec) {
        // Final partial step: fewer than U vectors per lane, loaded at clamped
        // indices so all are in flight; those past the row end become zeros.
        float xf[U][E];
        V va[R][U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t v = min(base + lane + 64 * k, nvec - 1);
            load_x<E>(x, v, xf[k]);
#pragma unroll
            for (int r = 0; r < R; ++r)
                va[r][k] = load_stream<VB>(rows[r], v);
        }
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool in = base + lane + 64 * k < nvec;
#pragma unroll
            for (int e = 0; e < E; ++e)
                xf[k][e] = in ? xf[k][e] : 0.f;
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool in = base + lane + 64 * k < nvec;
                float af[E];
                decode<T, VB>(va[r][k], af);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    af[e] = in ? af[e] : 0.f;
                acc[r].add(af, xf[k]);
            }
    }
    if (tail0 + lane < n) {  // fewer than E trailing columns
        float xs = x[tail0 + lane];
#pragma unroll
        for (int r = 0; r < R; ++r)
            acc[r].add_scalar(load_elem<T>(rows[r], tail0 + lane), xs);
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        if constexpr (ACC == ACC_F64) {
            double d = wave_sum((double)acc[r].value());
            if (lane == 0 && r0 + r < m) {
                double by = beta == 0.f ? 0.0 : (double)beta * (double)yold[r];
                y[r0 + r] = (float)((double)alpha * d + by);
            }
        } else if constexpr (ACC == ACC_COMP) {
            Pair p = wave_sum(acc[r].value());
            if (lane == 0 && r0 + r < m)
                store_row_y<ACC>(y, r0 + r, alpha, beta, p.s + p.c, yold[r]);
        } else {
            float d = wave_sum(acc[r].value());
            if (lane == 0 && r0 + r < m)
                store_row_y<ACC>(y, r0 + r, alpha, beta, d, yold[r]);
        }
    }
}

// Row-split form: one work-group computes R rows at a time, its B threads
// reading each row like the dot kernel reads a vector (thread t takes vectors
// t, t+B, ...: the whole work-group streams one contiguous row), then a
// work-group reduction per row.  This is map-workgroup over the rows with
// the row's dot lowered to map-local + the in-work-group tree, and it keeps
// HBM accesses as contiguous as a flat stream.
template <class T, int ACC, int VB, int R, int U>
__global__ void __launch_bounds__((gemv_bound<T, ACC, VB, R, U>())) gemv_split_kernel(GemvArgs a)
{
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    // LDS staging of the work-group reduction: binary64 for the binary64
    // combine, the lane type otherwise (16 waves at most).
    using LT = std::conditional_t<ACC == ACC_F64, double, typename BlockT<ACC>::type>;
    __shared__ LT lds[R][16];
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const int64_t row_bytes = a.lda * T::bytes;
    const int64_t tail0 = a.nvec * E;
    const int64_t step = B * U;

    for (int64_t r0 = (int64_t)blockIdx.x * R; r0 < a.m; r0 += (int64_t)gridDim.x * R) {  // uniform
        const char *rows[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            rows[r] = reinterpret_cast<const char *>(a.A) + min(r0 + r, a.m - 1) * row_bytes;
        float yold[R];  // read by wave 0, whose thread 0 stores the rows
#pragma unroll
        for (int r = 0; r < R; ++r)
            yold[r] = t < 64 ? prefetch_y(a.y, r0 + r, a.m, a.beta) : 0.f;
        RowAcc<ACC, E> acc[R];
        int64_t base = 0;
        for (; base + step <= a.nvec; base += step) {
            float xf[U][E];
            V va[R][U];
#pragma unroll
            for (int k = 0; k < U; ++k)
                load_x<E>(a.x, base + t + k * B, xf[k]);
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < U; ++k)
                    va[r][k] = load_stream<VB>(rows[r], base + t + k * B);
            loads_in_flight();
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    float af[E];
                    decode<T, VB>(va[r][k], af);
                    acc[r].add(af, xf[k]);
                }
        }
        if (base < a.nvec) {  // final partial step, clamped loads, zeros past the end
            float xf[U][E];
            V va[R][U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int64_t v = min(base + t + k * B, a.nvec - 1);
                load_x<E>(a.x, v, xf[k]);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    va[r][k] = load_stream<VB>(rows[r], v);
            }
            loads_in_flight();
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const bool in = base + t + k * B < a.nvec;
#pragma unroll
                for (int e = 0; e < E; ++e)
                    xf[k][e] = in ? xf[k][e] : 0.f;
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const bool in = base + t + k * B < a.nvec;
                    float af[E];
                    decode<T, VB>(va[r][k], af);
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        af[e] = in ? af[e] : 0.f;
                    acc[r].add(af, xf[k]);
                }
        }
        if (tail0 + t < a.n) {  // fewer than E trailing columns
            const float xs = a.x[tail0 + t];
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r].add_scalar(load_elem<T>(rows[r], tail0 + t), xs);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (ACC == ACC_F64) {
                double d = block_sum<double>((double)acc[r].value(), lds[r]);
                if (t == 0 && r0 + r < a.m) {
                    double by = a.beta == 0.f ? 0.0 : (double)a.beta * (double)yold[r];
                    a.y[r0 + r] = (float)((double)a.alpha * d + by);
                }
            } else if constexpr (ACC == ACC_COMP) {
                Pair p = block_sum<Pair>(acc[r].value(), lds[r]);
                if (t == 0 && r0 + r < a.m)
                    store_row_y<ACC>(a.y, r0 + r, a.alpha, a.beta, p.s + p.c, yold[r]);
            } else {
                float d = block_sum<float>(acc[r].value(), lds[r]);
                if (t == 0 && r0 + r < a.m)
                    store_row_y<ACC>(a.y, r0 + r, a.alpha, a.beta, d, yold[r]);
            }
        }
    }
}

// The row's finished dot (a wave's partial, then the work-group's fold of
// the wave partials) in the LDS type of the accumulation variant.
template <int ACC>
using RowPartT = std::conditional_t<ACC == ACC_F64, double, typename BlockT<ACC>::type>;

template <int ACC, int E>
__device__ __forceinline__ RowPartT<ACC> wave_row_partial(const RowAcc<ACC, E> &acc)
{
    if constexpr (ACC == ACC_F64)
        return wave_sum((double)acc.value());
    else
        return wave_sum(acc.value());
}

template <int ACC>
__device__ __forceinline__ void store_row_part(const GemvArgs &a, int64_t i, RowPartT<ACC> d)
{
    if constexpr (ACC == ACC_F64) {
        double by = a.beta == 0.f ? 0.0 : (double)a.beta * (double)a.y[i];
        a.y[i] = (float)((double)a.alpha * d + by);
    } else if constexpr (ACC == ACC_COMP) {
        store_row<ACC>(a.y, i, a.alpha, a.beta, d.s + d.c);
    } else {
        store_row<ACC>(a.y, i, a.alpha, a.beta, d);
    }
}

// Row-split form with x held in registers, for rows that one step of the
// work-group covers (nvec <= B * U).  Thread t needs the same x vectors
// t, t+B, ..., t+(U-1)B for every row, so it loads them once and each row
// costs only its A loads; x is read once per call instead of once per row.
// The work-group visits row groups [r0, r0 + R) for r0 = first, first + step,
// ... below `end` (rows from `end` on are read at a clamped index and never
// written).  Every wave folds its row partial with the butterfly and parks it
// in LDS; after 16 rows one barrier lets 16 threads fold those rows' wave
// partials in wave order and store y.  Two LDS banks alternate, so one
// barrier per 16 rows is enough (a bank is rewritten only after the next
// barrier, which every thread reaches after its reads of that bank).  Lanes,
// waves and wave partials are folded in the same orders as in
// gemv_split_kernel.  All threads of the work-group must call this with the
// same arguments (it has barriers).
template <class T, int ACC, int VB, int R, int U>
__device__ __forceinline__ void gemv_xs_rows(const GemvArgs &a, int64_t first, int64_t step, int64_t end,
                                             RowPartT<ACC> (*lds)[16][16])
{
    constexpr int E = Elems<T, VB>::value;
    constexpr int FL = 16 / R;  // row groups per flush
    using V = typename Vec<VB>::type;
    using LT = RowPartT<ACC>;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, waves = blockDim.x >> 6;
    const int64_t B = blockDim.x;
    const int64_t row_bytes = a.lda * T::bytes;
    const int64_t tail0 = a.nvec * E;
    const bool has_vec = a.nvec > 0;           // uniform
    const bool has_tail = tail0 + t < a.n;     // fewer than E trailing columns

    float xf[U][E];
#pragma unroll
    for (int k = 0; k < U; ++k)
#pragma unroll
        for (int e = 0; e < E; ++e)
            xf[k][e] = 0.f;
    if (has_vec) {
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t v = t + k * B;
            if (v < a.nvec)
                load_x<E>(a.x, v, xf[k]);
        }
    }
    const float xs = has_tail ? a.x[tail0 + t] : 0.f;

    int j = 0;
    for (int64_t r0 = first; r0 < end; r0 += step, ++j) {  // uniform
        const char *rows[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            rows[r] = reinterpret_cast<const char *>(a.A) + min(r0 + r, end - 1) * row_bytes;
        RowAcc<ACC, E> acc[R];
        if (has_vec) {
            V va[R][U];
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < U; ++k)
                    va[r][k] = load_stream<VB>(rows[r], min(t + k * B, a.nvec - 1));
            loads_in_flight();
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const bool in = t + k * B < a.nvec;
                    float af[E];
                    decode<T, VB>(va[r][k], af);
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        af[e] = in ? af[e] : 0.f;
                    acc[r].add(af, xf[k]);
                }
        }
        if (has_tail) {
#pragma unroll
            for (int r = 0; r < R; ++r)
                acc[r].add_scalar(load_elem<T>(rows[r], tail0 + t), xs);
        }
        const int slot = (j % FL) * R;
        const int bank = (j / FL) & 1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const LT w = wave_row_partial<ACC, E>(acc[r]);
            if (lane == 0)
                lds[bank][slot + r][wave] = w;
        }
        if (j % FL == FL - 1 || r0 + step >= end) {  // uniform: flush the parked rows
            __syncthreads();
            if (t < slot + R) {
                const int64_t row = first + (int64_t)(j - j % FL + t / R) * step + t % R;
                if (row < end) {
                    LT d = lds[bank][t][0];
                    for (int w = 1; w < waves; ++w)
                        d = merge(d, lds[bank][t][w]);
                    store_row_part<ACC>(a, row, d);
                }
            }
        }
    }
    __syncthreads();  // the caller may reuse the LDS banks
}

template <class T, int ACC, int VB, int R, int U>
__global__ void __launch_bounds__((gemv_bound<T, ACC, VB, R, U>())) gemv_xs_kernel(GemvArgs a)
{
    __shared__ RowPartT<ACC> lds[2][16][16];  // [bank][row slot][wave]
    gemv_xs_rows<T, ACC, VB, R, U>(a, (int64_t)blockIdx.x * R, (int64_t)gridDim.x * R, a.m, lds);
}

template <class T, int ACC, int VB, int R, int U>
__global__ void __launch_bounds__((gemv_bound<T, ACC, VB, R, U>())) gemv_kernel(GemvArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t wpb = blockDim.x >> 6;
    const int64_t gw = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * wpb;
    for (int64_t r0 = gw * R; r0 < a.m; r0 += nw * R)  // wave-uniform loop
        gemv_row_group<T, ACC, VB, R, U>(a.A, a.x, a.y, a.m, a.n, a.lda, a.nvec, a.alpha, a.beta, r0, lane);
}

template <class T, int ACC, int VB, int R>
const void *gemv_pick_unroll(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&gemv_kernel<T, ACC, VB, R, 1>);
    case 2: return reinterpret_cast<const void *>(&gemv_kernel<T, ACC, VB, R, 2>);
    case 4: return reinterpret_cast<const void *>(&gemv_kernel<T, ACC, VB, R, 4>);
    case 8: return reinterpret_cast<const void *>(&gemv_kernel<T, ACC, VB, R, 8>);
    default: return nullptr;
    }
}

template <class T, int ACC, int VB, int R, int U>
const void *gemv_split_variant(bool x_stationary)
{
    return x_stationary ? reinterpret_cast<const void *>(&gemv_xs_kernel<T, ACC, VB, R, U>)
                        : reinterpret_cast<const void *>(&gemv_split_kernel<T, ACC, VB, R, U>);
}

template <class T, int ACC, int VB, int R>
const void *gemv_split_pick_unroll(int unroll, bool x_stationary)
{
    switch (unroll) {
    case 2: return gemv_split_variant<T, ACC, VB, R, 2>(x_stationary);
    case 4: return gemv_split_variant<T, ACC, VB, R, 4>(x_stationary);
    case 8: return gemv_split_variant<T, ACC, VB, R, 8>(x_stationary);
    default: return nullptr;
    }
}

// Row-split instances: element loads (unaligned rows) or 16-byte loads,
// 1 or 2 rows per iteration, x streamed or held in registers.
template <class T, int ACC>
const void *gemv_split_pick(int vec_bytes, int rows, int unroll, bool xs)
{
    if (rows != 1 && rows != 2)
        return nullptr;
    if (vec_bytes == T::bytes)
        return rows == 1 ? gemv_split_pick_unroll<T, ACC, T::bytes, 1>(unroll, xs)
                         : gemv_split_pick_unroll<T, ACC, T::bytes, 2>(unroll, xs);
    if (vec_bytes == 16)
        return rows == 1 ? gemv_split_pick_unroll<T, ACC, 16, 1>(unroll, xs)
                         : gemv_split_pick_unroll<T, ACC, 16, 2>(unroll, xs);
    return nullptr;
}

template <class T>
const void *pick_gemv_split(int acc, int vec_bytes, int rows, int unroll, bool x_stationary)
{
    switch (acc) {
    case ACC_F32: return gemv_split_pick<T, ACC_F32>(vec_bytes, rows, unroll, x_stationary);
    case ACC_COMP: return gemv_split_pick<T, ACC_COMP>(vec_bytes, rows, unroll, x_stationary);
    case ACC_F64: return gemv_split_pick<T, ACC_F64>(vec_bytes, rows, unroll, x_stationary);
    default: return nullptr;
    }
}

template <class T, int ACC, int VB>
const void *gemv_pick_rows(int rows, int unroll)
{
    switch (rows) {
    case 1: return gemv_pick_unroll<T, ACC, VB, 1>(unroll);
    case 2: return gemv_pick_unroll<T, ACC, VB, 2>(unroll);
    case 4: return gemv_pick_unroll<T, ACC, VB, 4>(unroll);
    default: return nullptr;
    }
}

template <class T, int ACC>
const void *gemv_pick_vec(int vec_bytes, int rows, int unroll)
{
    switch (vec_bytes) {
    case 2:
        if constexpr (T::bytes == 2)
            return gemv_pick_rows<T, ACC, 2>(rows, unroll);
        return nullptr;
    case 4: return gemv_pick_rows<T, ACC, 4>(rows, unroll);
    case 8: return gemv_pick_rows<T, ACC, 8>(rows, unroll);
    case 16: return gemv_pick_rows<T, ACC, 16>(rows, unroll);
    default: return nullptr;
    }
}

template <class T>
const void *pick_gemv(int acc, int vec_bytes, int rows, int unroll)
{
    switch (acc) {
    case ACC_F32: return gemv_pick_vec<T, ACC_F32>(vec_bytes, rows, unroll);
    case ACC_COMP: return gemv_pick_vec<T, ACC_COMP>(vec_bytes, rows, unroll);
    case ACC_F64: return gemv_pick_vec<T, ACC_F64>(vec_bytes, rows, unroll);
    default: return nullptr;
    }
}

}  // namespace lift
