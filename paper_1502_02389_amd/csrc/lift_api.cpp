// C ABI of the library: argument checks, launch geometry, kernel dispatch.
//
// Every check runs before the first HIP call, so invalid calls fail the same
// way with or without a GPU.  Launch geometry follows the paper's knobs:
// the split factor decides how many vectors each work-group owns, the
// work-group size and vector width pick the kernel instance.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "lift.h"
#include "lift_internal.hpp"

using namespace lift;

namespace {

thread_local int g_last_hip_error = 0;
thread_local hipEvent_t g_time_start = nullptr;  // armed by lift_time_next_launch
thread_local hipEvent_t g_time_stop = nullptr;

constexpr int MAX_DEVICES = 64;
std::atomic<int> g_cu_count[MAX_DEVICES];

lift_status hip_fail(hipError_t e)
{
    g_last_hip_error = (int)e;
    return LIFT_EHIP;
}

// Compute units of the current device (cached per device).
lift_status cu_count(int *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e);
    if (dev < 0 || dev >= MAX_DEVICES)
        return LIFT_EUNSUPPORTED;
    int c = g_cu_count[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess)
            return hip_fail(e);
        if (c <= 0)
            c = 256;
        g_cu_count[dev].store(c, std::memory_order_relaxed);
    }
    *out = c;
    return LIFT_OK;
}

lift_status launch(const void *kernel, int64_t grid, int block, void *args, hipStream_t s)
{
    void *argv[] = {args};
    hipError_t e;
    if (g_time_start) {
        e = hipExtLaunchKernel(kernel, dim3((unsigned)grid), dim3((unsigned)block), argv, 0, s, g_time_start,
                               g_time_stop, 0);
        g_time_start = g_time_stop = nullptr;
    } else {
        e = hipLaunchKernel(kernel, dim3((unsigned)grid), dim3((unsigned)block), argv, 0, s);
    }
    if (e != hipSuccess)
        return hip_fail(e);
    return LIFT_OK;
}

int elem_bytes(int dt)
{
    switch (dt) {
    case LIFT_F32: return 4;
    case LIFT_BF16:
    case LIFT_F16: return 2;
    case LIFT_F64: return 8;
    default: return 0;
    }
}

bool aligned(const void *p, int64_t a) { return ((uintptr_t)p % (uintptr_t)a) == 0; }

// [p, p + bytes) and [q, q + qbytes) share a byte.
bool overlaps(const void *p, int64_t bytes, const void *q, int64_t qbytes)
{
    if (!p || !q || bytes <= 0 || qbytes <= 0)
        return false;
    uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return a < b + (uintptr_t)qbytes && b < a + (uintptr_t)bytes;
}

bool pow2_in(int64_t v, int64_t lo, int64_t hi)
{
    return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

// Resolved launch knobs.
struct Knobs {
    int block, vec_bytes, unroll, rows;
    int64_t split;
};

// Checks the caller's knobs (0 = default) and merges them with defaults.
lift_status resolve(const lift_knobs *k, Knobs def, int ebytes, Knobs *out)
{
    *out = def;
    if (!k)
        return LIFT_OK;
    if (k->block) {
        if (!pow2_in(k->block, 64, 1024))
            return LIFT_EINVAL;
        out->block = k->block;
    }
    if (k->vec_bytes) {
        if (!pow2_in(k->vec_bytes, 2, 16) || k->vec_bytes < ebytes)
            return LIFT_EINVAL;
        out->vec_bytes = k->vec_bytes;
    }
    if (k->unroll) {
        if (!pow2_in(k->unroll, 1, 8))
            return LIFT_EINVAL;
        out->unroll = k->unroll;
    }
    if (k->rows_per_wave) {
        if (!pow2_in(k->rows_per_wave, 1, 4))
            return LIFT_EINVAL;
        out->rows = k->rows_per_wave;
    }
    if (k->split < 0)
        return LIFT_EINVAL;
    if (k->split)
        out->split = k->split;
    return LIFT_OK;
}

// Defaults, from the knob search on MI355X (256 CUs): reductions run about
// one long-lived work-group per CU (fewer partials, shorter combine tail),
// scal many one-step work-groups, gemv small work-groups of row wavefronts.
constexpr Knobs DEF_SCAL = {256, 16, 2, 1, 0};
constexpr Knobs DEF_REDUCE = {256, 16, 8, 1, 0};
constexpr Knobs DEF_GEMV = {128, 16, 4, 1, 0};
constexpr int64_t WG_PER_CU_SCAL = 32;    // default grid for scal
constexpr int64_t WG_PER_CU_REDUCE = 1;   // default grid for asum / dot

// Split a range of n elements of `ebytes` bytes at base address p into a
// scalar head (up to the first vb-aligned address), whole vb-byte vectors,
// and a scalar tail.  Both p and q (if given) must share the head length.
struct Split3 {
    int64_t head, nvec;
};

bool split3(const void *p, const void *q, int64_t n, int ebytes, int vb, Split3 *out)
{
    const int64_t e = vb / ebytes;
    int64_t mis = (int64_t)((uintptr_t)p % (uintptr_t)vb);
    int64_t head = mis ? (vb - mis) / ebytes : 0;
    if (q) {
        int64_t mq = (int64_t)((uintptr_t)q % (uintptr_t)vb);
        if (mq != mis)
            return false;
    }
    head = std::min(head, n);
    out->head = head;
    out->nvec = (n - head) / e;
    return true;
}

// Vectors per work-group: the requested split (elements) or the default
// grid, rounded up to whole block * unroll steps, with the grid capped.
int64_t chunk_for(int64_t nvec, int64_t elems_per_vec, const Knobs &k, int cus, int64_t wg_per_cu,
                  int64_t max_wg)
{
    const int64_t step = (int64_t)k.block * k.unroll;
    int64_t chunk;
    if (k.split > 0) {
        chunk = (k.split + elems_per_vec - 1) / elems_per_vec;
    } else {
        int64_t target = (int64_t)cus * wg_per_cu;
        chunk = (nvec + target - 1) / std::max<int64_t>(target, 1);
    }
    chunk = std::max<int64_t>(step, (chunk + step - 1) / step * step);
    if ((nvec + chunk - 1) / chunk > max_wg) {
        chunk = (nvec + max_wg - 1) / max_wg;
        chunk = (chunk + step - 1) / step * step;
    }
    return chunk;
}

const void *reduce_table(int dt, int op, int acc, int vb, int unroll)
{
    switch (dt) {
    case LIFT_F32: return reduce_kernel_f32(op, acc, vb, unroll);
    case LIFT_BF16: return reduce_kernel_bf16(op, acc, vb, unroll);
    case LIFT_F16: return reduce_kernel_f16(op, acc, vb, unroll);
    default: return nullptr;
    }
}

const void *gemv_table(int dt, int acc, int vb, int rows, int unroll)
{
    switch (dt) {
    case LIFT_F32: return gemv_kernel_f32(acc, vb, rows, unroll);
    case LIFT_BF16: return gemv_kernel_bf16(acc, vb, rows, unroll);
    case LIFT_F16: return gemv_kernel_f16(acc, vb, rows, unroll);
    default: return nullptr;
    }
}

lift_status reduce_common(int op, int64_t n, int xt, const void *x, const void *y, int acc, int rt,
                          void *result, void *ws, size_t ws_bytes, const lift_knobs *knobs,
                          hipStream_t stream)
{
    if (n < 0)
        return LIFT_EINVAL;
    if (xt != LIFT_F32 && xt != LIFT_BF16 && xt != LIFT_F16)
        return LIFT_EINVAL;
    if (rt != LIFT_F32 && rt != LIFT_F64)
        return LIFT_EINVAL;
    if (acc != LIFT_ACC_F32 && acc != LIFT_ACC_F32_COMP && acc != LIFT_ACC_F32_F64COMBINE)
        return LIFT_EINVAL;
    const int eb = elem_bytes(xt), rb = elem_bytes(rt);
    if (!result || !aligned(result, rb))
        return LIFT_EINVAL;
    if (n > 0 && (!x || !aligned(x, eb)))
        return LIFT_EINVAL;
    if (op == OP_DOT && n > 0 && (!y || !aligned(y, eb)))
        return LIFT_EINVAL;
    if (!ws || ws_bytes < lift_workspace_bytes())
        return LIFT_EWORKSPACE;
    if (!aligned(ws, 16))
        return LIFT_EINVAL;
    const int64_t xbytes = n * eb;
    if (overlaps(result, rb, x, xbytes) || overlaps(result, rb, y, op == OP_DOT ? xbytes : 0) ||
        overlaps(result, rb, ws, (int64_t)ws_bytes))
        return LIFT_EINVAL;
    Knobs k;
    Knobs def = DEF_REDUCE;
    if (eb == 2)
        def.unroll = 4;  // 8 elements per 16-byte load already; more only adds registers
    lift_status st = resolve(knobs, def, eb, &k);
    if (st != LIFT_OK)
        return st;

    // Vector width: the requested one if x (and y) share its alignment
    // phase, else the element size (scalar loads).
    Split3 sp{0, 0};
    int vb = k.vec_bytes;
    if (n > 0 && !split3(x, op == OP_DOT ? y : nullptr, n, eb, vb, &sp)) {
        vb = eb;
        split3(x, nullptr, n, eb, vb, &sp);
    }
    const void *kern = reduce_table(xt, op, acc, vb, k.unroll);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t e = vb / eb;
    const int64_t chunk = chunk_for(sp.nvec, e, k, cus, WG_PER_CU_REDUCE, MAX_WORKGROUPS);
    const int64_t grid = std::max<int64_t>(1, (sp.nvec + chunk - 1) / chunk);

    ReduceArgs a;
    a.x = x;
    a.y = y;
    a.n = n;
    a.head = sp.head;
    a.nvec = sp.nvec;
    a.chunk = chunk;
    a.ws = ws;
    a.result = result;
    a.result_f64 = rt == LIFT_F64;
    return launch(kern, grid, k.block, &a, stream);
}

lift_status gemv_common(int64_t m, int64_t n, float alpha, int at, const void *A, int64_t lda,
                        const float *x, float beta, float *y, int acc, const lift_knobs *knobs,
                        hipStream_t stream)
{
    if (m < 0 || n < 0 || lda < std::max<int64_t>(1, n))
        return LIFT_EINVAL;
    if (at != LIFT_F32 && at != LIFT_BF16 && at != LIFT_F16)
        return LIFT_EINVAL;
    if (acc != LIFT_ACC_F32 && acc != LIFT_ACC_F32_COMP && acc != LIFT_ACC_F32_F64COMBINE)
        return LIFT_EINVAL;
    const int eb = elem_bytes(at);
    if (m > 0 && (!y || !aligned(y, 4)))
        return LIFT_EINVAL;
    if (m > 0 && n > 0 && (!A || !x || !aligned(A, eb) || !aligned(x, 4)))
        return LIFT_EINVAL;
    const int64_t abytes = m > 0 && n > 0 ? ((m - 1) * lda + n) * eb : 0;
    if (overlaps(y, m * 4, A, abytes) || overlaps(y, m * 4, x, m > 0 ? n * 4 : 0))
        return LIFT_EINVAL;
    Knobs k;
    lift_status st = resolve(knobs, DEF_GEMV, eb, &k);
    if (st != LIFT_OK)
        return st;
    if (m == 0)
        return LIFT_OK;

    if (!knobs || !knobs->rows_per_wave)
        k.rows = m * n > ((int64_t)1 << 25) ? 2 : 1;  // long matrices: share x loads over 2 rows
    // Vector path needs every row start and x aligned for the chosen width.
    int vb = k.vec_bytes;
    int64_t e = vb / eb;
    const int64_t xalign = std::min<int64_t>(e * 4, 16);
    if (n == 0 || !aligned(A, vb) || (lda * eb) % vb != 0 || !aligned(x, xalign)) {
        vb = eb;
        e = 1;
    }
    const void *kern = gemv_table(at, acc, vb, k.rows, std::min(k.unroll, 4));
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t waves = (m + k.rows - 1) / k.rows;
    const int64_t wpb = k.block / 64;
    int64_t grid = (waves + wpb - 1) / wpb;
    grid = std::min<int64_t>(grid, (int64_t)cus * 64);

    GemvArgs a;
    a.A = A;
    a.x = x;
    a.y = y;
    a.m = m;
    a.n = n;
    a.lda = lda;
    a.nvec = n / e;
    a.alpha = alpha;
    a.beta = beta;
    return launch(kern, grid, k.block, &a, stream);
}

}  // namespace

extern "C" {

size_t lift_workspace_bytes(void) { return (size_t)(WS_HEADER + (int64_t)MAX_WORKGROUPS * WS_SLOT); }

int32_t lift_max_workgroups(void) { return MAX_WORKGROUPS; }

lift_status lift_scal_ex(int64_t n, float alpha, const float *x, float *out, const lift_knobs *knobs,
                         hipStream_t stream)
{
    if (n < 0)
        return LIFT_EINVAL;
    if (n > 0 && (!x || !out || !aligned(x, 4) || !aligned(out, 4)))
        return LIFT_EINVAL;
    if (x != out && overlaps(x, n * 4, out, n * 4))
        return LIFT_EINVAL;
    Knobs k;
    lift_status st = resolve(knobs, DEF_SCAL, 4, &k);
    if (st != LIFT_OK)
        return st;
    if (k.vec_bytes < 4)
        return LIFT_EINVAL;
    if (n == 0)
        return LIFT_OK;
    Split3 sp;
    int vb = k.vec_bytes;
    if (!split3(x, out, n, 4, vb, &sp)) {
        vb = 4;
        split3(x, nullptr, n, 4, vb, &sp);
    }
    const void *kern = scal_kernel(vb, k.unroll);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t chunk = chunk_for(sp.nvec, vb / 4, k, cus, WG_PER_CU_SCAL, INT32_MAX);
    const int64_t grid = std::max<int64_t>(1, (sp.nvec + chunk - 1) / chunk);
    ScalArgs a;
    a.x = x;
    a.out = out;
    a.n = n;
    a.head = sp.head;
    a.nvec = sp.nvec;
    a.chunk = chunk;
    a.alpha = alpha;
    return launch(kern, grid, k.block, &a, stream);
}

lift_status lift_scal(int64_t n, float alpha, const float *x, float *out, hipStream_t stream)
{
    return lift_scal_ex(n, alpha, x, out, nullptr, stream);
}

lift_status lift_asum(int64_t n, const float *x, float *result, void *ws, size_t ws_bytes,
                      hipStream_t stream)
{
    return reduce_common(OP_ASUM, n, LIFT_F32, x, nullptr, LIFT_ACC_F32, LIFT_F32, result, ws,
                         ws_bytes, nullptr, stream);
}

lift_status lift_dot(int64_t n, const float *x, const float *y, float *result, void *ws,
                     size_t ws_bytes, hipStream_t stream)
{
    return reduce_common(OP_DOT, n, LIFT_F32, x, y, LIFT_ACC_F32, LIFT_F32, result, ws, ws_bytes,
                         nullptr, stream);
}

lift_status lift_asum_ex(int64_t n, lift_dtype xt, const void *x, lift_acc acc, lift_dtype rt,
                         void *result, void *ws, size_t ws_bytes, const lift_knobs *knobs,
                         hipStream_t stream)
{
    return reduce_common(OP_ASUM, n, xt, x, nullptr, acc, rt, result, ws, ws_bytes, knobs, stream);
}

lift_status lift_dot_ex(int64_t n, lift_dtype xt, const void *x, const void *y, lift_acc acc,
                        lift_dtype rt, void *result, void *ws, size_t ws_bytes,
                        const lift_knobs *knobs, hipStream_t stream)
{
    return reduce_common(OP_DOT, n, xt, x, y, acc, rt, result, ws, ws_bytes, knobs, stream);
}

lift_status lift_gemv(int64_t m, int64_t n, float alpha, const float *A, int64_t lda,
                      const float *x, float beta, float *y, hipStream_t stream)
{
    return gemv_common(m, n, alpha, LIFT_F32, A, lda, x, beta, y, LIFT_ACC_F32, nullptr, stream);
}

lift_status lift_gemv_ex(int64_t m, int64_t n, float alpha, lift_dtype at, const void *A,
                         int64_t lda, const float *x, float beta, float *y, lift_acc acc,
                         const lift_knobs *knobs, hipStream_t stream)
{
    return gemv_common(m, n, alpha, at, A, lda, x, beta, y, acc, knobs, stream);
}

const char *lift_status_string(lift_status s)
{
    switch (s) {
    case LIFT_OK: return "ok";
    case LIFT_EINVAL: return "invalid argument";
    case LIFT_EWORKSPACE: return "workspace missing or too small";
    case LIFT_EHIP: return "HIP runtime error";
    case LIFT_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown status";
    }
}

int lift_last_hip_error(void) { return g_last_hip_error; }

lift_status lift_time_next_launch(hipEvent_t start, hipEvent_t stop)
{
    if ((start == nullptr) != (stop == nullptr))
        return LIFT_EINVAL;
    g_time_start = start;
    g_time_stop = stop;
    return LIFT_OK;
}

const char *lift_version(void) { return "lift-mi355x 0.1 gfx950"; }

}  // extern "C"
