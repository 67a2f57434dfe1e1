// C ABI of the library: argument checks, launch geometry, kernel dispatch.
//
// Every check runs before the first HIP call, so invalid calls fail the same
// way with or without a GPU.  Launch geometry follows the paper's knobs:
// the split factor decides how many vectors each work-group owns, the
// work-group size and vector width pick the kernel instance.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <numeric>
#include <utility>
#include <vector>

#include "lift.h"
#include "lift_apps.hpp"
#include "lift_internal.hpp"

using namespace lift;

namespace {

thread_local int g_last_hip_error = 0;
thread_local hipEvent_t g_time_start = nullptr;  // armed by lift_time_next_launch
thread_local hipEvent_t g_time_stop = nullptr;
thread_local uint64_t *g_stamps = nullptr;       // armed by lift_stamp_next_launch
thread_local int64_t g_stamp_capacity = 0;

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

// The largest work-group a kernel was compiled for (its launch bound),
// cached per kernel.
lift_status max_block(const void *kernel, int *out)
{
    static std::mutex mu;
    static std::vector<std::pair<const void *, int>> cache;
    std::lock_guard<std::mutex> lock(mu);
    for (const auto &kv : cache)
        if (kv.first == kernel) {
            *out = kv.second;
            return LIFT_OK;
        }
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, kernel);
    if (e != hipSuccess)
        return hip_fail(e);
    cache.emplace_back(kernel, attr.maxThreadsPerBlock);
    *out = attr.maxThreadsPerBlock;
    return LIFT_OK;
}

// How many work-groups of `block` threads of a kernel fit on one compute
// unit at once (registers, LDS, wave slots), cached per kernel and size.
lift_status resident_per_cu(const void *kernel, int block, int *out)
{
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void *, int>, int>> cache;
    std::lock_guard<std::mutex> lock(mu);
    for (const auto &kv : cache)
        if (kv.first.first == kernel && kv.first.second == block) {
            *out = kv.second;
            return LIFT_OK;
        }
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, block, 0);
    if (e != hipSuccess)
        return hip_fail(e);
    n = std::max(n, 1);
    cache.emplace_back(std::make_pair(kernel, block), n);
    *out = n;
    return LIFT_OK;
}

// Work-items of one dispatch are counted in 32 bits (the dispatch packet's
// grid size).
constexpr int64_t MAX_DISPATCH_ITEMS = 0xFFFFFFFFLL;

lift_status launch(const void *kernel, int64_t grid, int block, void *args, hipStream_t s)
{
    if (grid <= 0 || block <= 0 || grid * block > MAX_DISPATCH_ITEMS)
        return LIFT_EUNSUPPORTED;
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
    int wg_per_cu;
    int row_split;  // 1: wavefront per row group, 2: work-group per row
    int lanes;      // MD: lanes per particle
    int interleave; // reductions: 1 = grid-stride steps, 0 = contiguous chunks
    int lane_form;  // reductions: a lift_lane_form value
};

// Checks the caller's knobs (0 = default) and merges them with defaults.
// `lanes`: the op takes lane forms (asum / dot), whose sequential forms
// allow work-groups of 1 to 32 lanes.
lift_status resolve(const lift_knobs *k, Knobs def, int ebytes, Knobs *out, bool lanes = false)
{
    *out = def;
    if (!k)
        return LIFT_OK;
    if (k->lane_form < LIFT_LANES_TREE || k->lane_form > LIFT_LANES_RUNS_SEQ)
        return LIFT_EINVAL;
    if (lanes)
        out->lane_form = k->lane_form;
    if (k->block) {
        if (!pow2_in(k->block, lanes && (k->lane_form & LIFT_LANES_SEQ) ? 1 : 64, 1024))
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
    if (k->wg_per_cu < 0 || k->wg_per_cu > 64 || k->row_split < 0 || k->row_split > 2)
        return LIFT_EINVAL;
    if (k->wg_per_cu)
        out->wg_per_cu = k->wg_per_cu;
    if (k->row_split)
        out->row_split = k->row_split;
    if (k->lanes_per_item) {
        if (!pow2_in(k->lanes_per_item, 1, 16))
            return LIFT_EINVAL;
        out->lanes = k->lanes_per_item;
    }
    if (k->interleave < LIFT_INTERLEAVE_DEFAULT || k->interleave > LIFT_INTERLEAVE_CHUNK)
        return LIFT_EINVAL;
    if (k->interleave)
        out->interleave = k->interleave == LIFT_INTERLEAVE_STRIDE;
    return LIFT_OK;
}

// Defaults, from the knob search on MI355X (256 CUs): reductions run about
// one long-lived work-group per CU (fewer partials, shorter combine tail),
// scal many one-step work-groups, gemv a work-group per row with x held in
// registers where one step covers a row (row_split 0 = chosen per shape).
constexpr Knobs DEF_SCAL = {256, 4, 8, 1, 0, 32, 1, 1, 0};
constexpr Knobs DEF_REDUCE = {256, 16, 8, 1, 0, 1, 1, 1, 0};
constexpr Knobs DEF_GEMV = {256, 16, 8, 1, 0, 0, 0, 1, 0};
constexpr Knobs DEF_BATCH = {256, 16, 4, 1, 65536, 2, 1, 1, 0};
constexpr Knobs DEF_BS = {256, 4, 4, 1, 0, 16, 1, 1, 0};
constexpr Knobs DEF_MD = {256, 16, 2, 1, 0, 0, 1, 16, 0};
constexpr Knobs DEF_STREAM = {256, 16, 8, 1, 0, 1, 1, 1, 0};

// ---- knobs for calls that pass none --------------------------------------
//
// A call with knobs == NULL runs with, in this order: the LIFT_FORCE_CONFIG
// override (read once from the environment), the autotuned entry for its
// op / storage / accumulation / log2 size bucket on a device of the same
// architecture and compute-unit count (generated at build time from the
// tuner's cache), or the defaults above.

enum TunedOp { TOP_SCAL = 0, TOP_ASUM, TOP_DOT, TOP_GEMV, TOP_BATCH, TOP_BS, TOP_MD, TOP_COUNT };

struct TunedEntry {
    const char *arch;  // e.g. "gfx950"; nullptr ends the table
    int cus, op, storage, acc, bucket;
    int row_bucket;    // gemv: floor(log2(n)); -1: any
    lift_knobs knobs;
};

const TunedEntry TUNED_TABLE[] = {
#include "lift_tuned_table.inc"
    {nullptr, 0, 0, 0, 0, 0, -1, {0, 0, 0, 0, 0, 0, 0, 0, 0}},
};

const char *const TUNED_OP_NAMES[TOP_COUNT] = {"scal", "asum", "dot", "gemv", "batch", "blackscholes", "md"};

int log2_bucket(int64_t elements)
{
    int b = 0;
    while (elements > 1) {
        elements >>= 1;
        ++b;
    }
    return b;
}

const TunedEntry *tuned_entry(const char *arch, int cus, int op, int storage, int acc, int64_t elements,
                              int64_t row_length)
{
    const int bucket = op == TOP_BATCH ? 0 : log2_bucket(elements);
    const int row_bucket = log2_bucket(row_length);
    for (const TunedEntry *e = TUNED_TABLE; e->arch; ++e)
        if (e->cus == cus && e->op == op && e->storage == storage && e->acc == acc && e->bucket == bucket &&
            (e->row_bucket < 0 || e->row_bucket == row_bucket) && std::strcmp(e->arch, arch) == 0)
            return e;
    return nullptr;
}

// LIFT_FORCE_CONFIG="key=value,...": keys block (or wg), vec, unroll, rpw,
// split, wgcu, rowsplit, lanes, interleave (stride | chunk), laneform; values are
// non-negative integers.  Parsed once; a malformed string makes every call
// without knobs fail with LIFT_EINVAL.
struct Forced {
    bool present = false, valid = true;
    lift_knobs knobs{};
};

bool parse_forced(const char *text, lift_knobs *k)
{
    std::memset(k, 0, sizeof *k);
    const char *p = text;
    while (*p) {
        const char *eq = std::strchr(p, '=');
        if (!eq)
            return false;
        std::string key(p, eq);
        const char *v = eq + 1;
        const char *end = std::strchr(v, ',');
        std::string val = end ? std::string(v, end) : std::string(v);
        p = end ? end + 1 : v + val.size();
        if (key == "interleave" && (val == "stride" || val == "chunk")) {
            k->interleave = val == "stride" ? LIFT_INTERLEAVE_STRIDE : LIFT_INTERLEAVE_CHUNK;
            continue;
        }
        if (val.empty() || val.size() > 12 || val.find_first_not_of("0123456789") != std::string::npos)
            return false;
        const long long x = std::stoll(val);
        if (key == "block" || key == "wg")
            k->block = (int32_t)x;
        else if (key == "vec")
            k->vec_bytes = (int32_t)x;
        else if (key == "unroll")
            k->unroll = (int32_t)x;
        else if (key == "rpw")
            k->rows_per_wave = (int32_t)x;
        else if (key == "split")
            k->split = (int64_t)x;
        else if (key == "wgcu")
            k->wg_per_cu = (int32_t)x;
        else if (key == "rowsplit")
            k->row_split = (int32_t)x;
        else if (key == "lanes")
            k->lanes_per_item = (int32_t)x;
        else if (key == "interleave")
            k->interleave = (int32_t)x;
        else if (key == "laneform")
            k->lane_form = (int32_t)x;
        else
            return false;
        if (x > INT32_MAX && key != "split")
            return false;
    }
    return true;
}

const Forced &forced_config()
{
    static Forced f;
    static std::once_flag once;
    std::call_once(once, [] {
        const char *env = std::getenv("LIFT_FORCE_CONFIG");
        if (env && *env) {
            f.present = true;
            f.valid = parse_forced(env, &f.knobs);
        }
    });
    return f;
}

// Architecture name (up to the first ':') and CU count of the current
// device, cached per device; false if the device cannot be queried.
bool device_identity(const char **arch, int *cus)
{
    static std::mutex mu;
    static char names[MAX_DEVICES][64];
    static int counts[MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES)
        return false;
    std::lock_guard<std::mutex> lock(mu);
    if (counts[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
            return false;
        size_t i = 0;
        for (; i + 1 < sizeof names[dev] && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
            names[dev][i] = prop.gcnArchName[i];
        names[dev][i] = 0;
        counts[dev] = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : -1;
    }
    *arch = names[dev];
    *cus = counts[dev];
    return true;
}

// The knobs a call runs with: the caller's, else forced, else tuned for this
// device, else nullptr (defaults).  *st is LIFT_EINVAL for a malformed
// LIFT_FORCE_CONFIG.
const lift_knobs *effective_knobs(const lift_knobs *given, int op, int storage, int acc, int64_t elements,
                                  lift_status *st, int64_t row_length = 0)
{
    *st = LIFT_OK;
    if (given)
        return given;
    const Forced &f = forced_config();
    if (f.present) {
        if (!f.valid)
            *st = LIFT_EINVAL;
        return &f.knobs;
    }
    const char *arch = nullptr;
    int cus = 0;
    if (!device_identity(&arch, &cus))  // no device: defaults (the launch reports the HIP error)
        return nullptr;
    const TunedEntry *e = tuned_entry(arch, cus, op, storage, acc, elements, row_length);
    return e ? &e->knobs : nullptr;
}

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
int64_t chunk_for(int64_t nvec, int64_t elems_per_vec, const Knobs &k, int cus, int64_t max_wg)
{
    const int64_t wg_per_cu = k.wg_per_cu;
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

const void *gemv_split_table(int dt, int acc, int vb, int rows, int unroll, bool xs)
{
    switch (dt) {
    case LIFT_F32: return gemv_split_kernel_f32(acc, vb, rows, unroll, xs);
    case LIFT_BF16: return gemv_split_kernel_bf16(acc, vb, rows, unroll, xs);
    case LIFT_F16: return gemv_split_kernel_f16(acc, vb, rows, unroll, xs);
    default: return nullptr;
    }
}

// Checks of a reduction's operands (everything but the workspace).
lift_status reduce_check(int op, int64_t n, int xt, const void *x, const void *y, int acc, int rt,
                         const void *result)
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
    const int64_t xbytes = n * eb;
    if (overlaps(result, rb, x, xbytes) || overlaps(result, rb, y, op == OP_DOT ? xbytes : 0))
        return LIFT_EINVAL;
    return LIFT_OK;
}

lift_status reduce_common(int op, int64_t n, int xt, const void *x, const void *y, int acc, int rt,
                          void *result, void *ws, size_t ws_bytes, const lift_knobs *knobs,
                          hipStream_t stream)
{
    lift_status st0 = reduce_check(op, n, xt, x, y, acc, rt, result);
    if (st0 != LIFT_OK)
        return st0;
    const int eb = elem_bytes(xt), rb = elem_bytes(rt);
    if (!ws || ws_bytes < lift_workspace_bytes())
        return LIFT_EWORKSPACE;
    if (!aligned(ws, 16))
        return LIFT_EINVAL;
    if (overlaps(result, rb, ws, (int64_t)ws_bytes))
        return LIFT_EINVAL;
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, op == OP_DOT ? TOP_DOT : TOP_ASUM, xt, acc, n, &st);
    if (st != LIFT_OK)
        return st;
    Knobs k;
    Knobs def = DEF_REDUCE;
    if (op == OP_DOT) {
        def.unroll = 4;  // two streams: grid-stride steps of 4 loads of each in flight
        def.interleave = 1;
    }
    st = resolve(knobs, def, eb, &k, true);
    if (st != LIFT_OK)
        return st;
    if (k.lane_form) {
        // the other lane forms: binary32 accumulation, the chunk partition
        if (acc != LIFT_ACC_F32 || (xt != LIFT_F32 && xt != LIFT_BF16))
            return LIFT_EUNSUPPORTED;
        if (knobs->interleave == LIFT_INTERLEAVE_STRIDE)
            return LIFT_EINVAL;
        k.interleave = 0;
    }

    // Vector width: the requested one if x (and y) share its alignment
    // phase, else the element size (scalar loads).
    Split3 sp{0, 0};
    int vb = k.vec_bytes;
    if (n > 0 && !split3(x, op == OP_DOT ? y : nullptr, n, eb, vb, &sp)) {
        vb = eb;
        split3(x, nullptr, n, eb, vb, &sp);
    }
    const void *kern = !k.lane_form ? reduce_table(xt, op, acc, vb, k.unroll)
                       : xt == LIFT_F32 ? reduce_lanes_kernel_f32(op, vb, k.unroll, k.lane_form)
                                        : reduce_lanes_kernel_bf16(op, vb, k.unroll, k.lane_form);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t e = vb / eb;
    const int64_t chunk = chunk_for(sp.nvec, e, k, cus, MAX_WORKGROUPS);
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
    a.interleave = k.interleave;
    a.stamps = nullptr;
    if (g_stamps) {  // the stamped instance of the same kernel (one-shot)
        uint64_t *buf = g_stamps;
        const int64_t cap = g_stamp_capacity;
        g_stamps = nullptr;
        if (xt != LIFT_F32 || acc != LIFT_ACC_F32 || vb != 16 || k.lane_form)
            return LIFT_EUNSUPPORTED;
        if (grid > cap)
            return LIFT_EINVAL;
        kern = reduce_kernel_stamped_f32(op, k.unroll);
        if (!kern)
            return LIFT_EUNSUPPORTED;
        a.stamps = buf;
    }
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
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, TOP_GEMV, at, acc, m * n, &st, n);
    if (st != LIFT_OK)
        return st;
    Knobs k;
    st = resolve(knobs, DEF_GEMV, eb, &k);
    if (st != LIFT_OK)
        return st;
    if (m == 0)
        return LIFT_OK;

    // Vector path needs every row start and x aligned for the chosen width.
    int vb = k.vec_bytes;
    int64_t e = vb / eb;
    const int64_t xalign = std::min<int64_t>(e * 4, 16);
    if (n == 0 || !aligned(A, vb) || (lda * eb) % vb != 0 || !aligned(x, xalign)) {
        vb = eb;
        e = 1;
    }
    if (k.row_split == 0) {
        // library choice: a work-group per row where one step of at most 512
        // threads covers the row (x then stays in registers), sized to the row
        // unless the caller fixed the work-group size
        const int64_t nvec = n / e;
        const bool fits = (vb == 16 || vb == eb) && nvec <= (int64_t)512 * k.unroll;
        k.row_split = fits ? 2 : 1;
        if (fits && (!knobs || !knobs->block)) {
            k.block = 64;
            while ((int64_t)k.block * k.unroll < nvec && k.block < 512)
                k.block *= 2;
        }
    }
    if (!knobs || !knobs->rows_per_wave)  // wavefront form on long matrices: share x loads over 2 rows
        k.rows = k.row_split == 1 && m * n > ((int64_t)1 << 25) ? 2 : 1;
    int cus = 0;
    const void *kern;
    int64_t grid;
    int bound = 0;
    if (k.row_split == 2) {
        // the work-group streams whole rows: 16-byte loads or element loads
        if (vb != eb && vb != 16) {
            vb = eb;
            e = 1;
        }
        kern = gemv_split_table(at, acc, vb, k.rows, k.unroll, false);
        if (!kern)
            return LIFT_EUNSUPPORTED;
        st = cu_count(&cus);
        if (st == LIFT_OK)
            st = max_block(kern, &bound);  // the x-stationary instance has the same bound
        if (st != LIFT_OK)
            return st;
        k.block = std::min(k.block, bound);
        // rows that one step of the work-group covers: x stays in registers
        const bool xs = n / e <= (int64_t)k.block * k.unroll;
        if (xs)
            kern = gemv_split_table(at, acc, vb, k.rows, k.unroll, true);
        const int64_t per_cu = k.wg_per_cu ? k.wg_per_cu : (xs ? 8 : 16);
        grid = std::min<int64_t>((m + k.rows - 1) / k.rows, (int64_t)cus * per_cu);
    } else {
        kern = gemv_table(at, acc, vb, k.rows, k.unroll);
        if (!kern)
            return LIFT_EUNSUPPORTED;
        st = cu_count(&cus);
        if (st == LIFT_OK)
            st = max_block(kern, &bound);
        if (st != LIFT_OK)
            return st;
        k.block = std::min(k.block, bound);
        const int64_t waves = (m + k.rows - 1) / k.rows;
        const int64_t wpb = k.block / 64;
        grid = std::min<int64_t>((waves + wpb - 1) / wpb, (int64_t)cus * 64);
    }

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

const void *batch_table(int dt, int acc, int vb, int unroll, bool gemv)
{
    switch (dt) {
    case LIFT_F32: return batch_kernel_f32(acc, vb, unroll, gemv);
    case LIFT_BF16: return batch_kernel_bf16(acc, vb, unroll, gemv);
    case LIFT_F16: return batch_kernel_f16(acc, vb, unroll, gemv);
    default: return nullptr;
    }
}

// True if any interval of `outs` shares a byte with another interval of
// `outs` or with any interval of `ins` ([begin, end) byte ranges).
bool any_overlap(std::vector<std::pair<uintptr_t, uintptr_t>> outs,
                 std::vector<std::pair<uintptr_t, uintptr_t>> ins)
{
    std::sort(outs.begin(), outs.end());
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].first < outs[i - 1].second)
            return true;
    std::sort(ins.begin(), ins.end());
    // prefix maximum of input ends, to test each output against every input
    std::vector<uintptr_t> maxend(ins.size());
    uintptr_t m = 0;
    for (size_t i = 0; i < ins.size(); ++i)
        maxend[i] = m = std::max(m, ins[i].second);
    for (const auto &o : outs) {
        // inputs starting before o.second; overlap if any of them ends after o.first
        size_t k = std::lower_bound(ins.begin(), ins.end(), std::make_pair(o.second, (uintptr_t)0)) - ins.begin();
        if (k > 0 && maxend[k - 1] > o.first)
            return true;
    }
    return false;
}

// The bandwidth reference kernels: checks, then the reductions' partition
// (chunk_for) over 16-byte vectors.
lift_status stream_common(bool copy, int64_t n, const float *x, float *out, const lift_knobs *knobs,
                          hipStream_t stream)
{
    if (n < 0 || n % 4 != 0)
        return LIFT_EINVAL;
    if (n > 0 && (!x || !out || !aligned(x, 16) || !aligned(out, copy ? 16 : 4)))
        return LIFT_EINVAL;
    if (overlaps(x, n * 4, out, copy ? n * 4 : 4))
        return LIFT_EINVAL;
    Knobs k;
    lift_status st = resolve(knobs, DEF_STREAM, 4, &k);
    if (st != LIFT_OK)
        return st;
    if (k.vec_bytes != 16)
        return LIFT_EUNSUPPORTED;
    if (n == 0)
        return LIFT_OK;
    const void *kern = stream_kernel(copy, k.unroll);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t nvec = n / 4;
    const int64_t chunk = chunk_for(nvec, 4, k, cus, MAX_DISPATCH_ITEMS / k.block);
    StreamArgs a;
    a.x = x;
    a.out = out;
    a.nvec = nvec;
    a.chunk = chunk;
    a.interleave = k.interleave;
    return launch(kern, std::max<int64_t>(1, (nvec + chunk - 1) / chunk), k.block, &a, stream);
}

// ---- allocation-free reductions --------------------------------------------
//
// lift_dot_ex_noalloc keeps its arrival counters and partial slots in this
// file-scope device array instead of a caller workspace: one copy per device,
// zero-filled when the library's code object is loaded on it, and left with
// its counters zeroed by every call that completes (the last work-group
// resets them), so nothing is cleared per call.  In host code `scratch` names
// a host-side stand-in; the device address of each device's copy comes from
// hipGetSymbolAddress with that device current, once, and only that address
// is handed to kernels.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)(WS_HEADER + (int64_t)MAX_WORKGROUPS * WS_SLOT);
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

lift_status static_scratch(void **out)
{
    static std::mutex mu;
    static void *addr[MAX_DEVICES];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e);
    if (dev < 0 || dev >= MAX_DEVICES)
        return LIFT_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e);
        if (!p)
            return LIFT_EHIP;
        addr[dev] = p;
    }
    *out = addr[dev];
    return LIFT_OK;
}

}  // namespace

// A planned batch: one launch over the reduction tiles ([0]) and one over
// the gemv tiles ([1]), each with its own tile table and counters.
struct lift_batch {
    int device = 0;
    int64_t nprobs = 0;
    int64_t bytes = 0;
    int block = 0;
    void *dmem = nullptr;
    int64_t ntiles[2] = {0, 0};
    int64_t grid[2] = {0, 0};
    const void *kern[2] = {nullptr, nullptr};
    BatchArgs args[2]{};
    hipEvent_t ev[2] = {nullptr, nullptr};  // inner ends of a timed two-launch run
    int storage = 0, acc = 0, vb = 0, unroll = 0;  // for the stamped gemv instance
};

namespace {

lift_status batch_plan(const lift_problem *probs, int32_t count, int storage, int acc, int rt,
                       const lift_knobs *knobs, lift_batch *b)
{
    if (count < 0 || (count > 0 && !probs))
        return LIFT_EINVAL;
    if (storage != LIFT_F32 && storage != LIFT_BF16 && storage != LIFT_F16)
        return LIFT_EINVAL;
    if (acc != LIFT_ACC_F32 && acc != LIFT_ACC_F32_COMP && acc != LIFT_ACC_F32_F64COMBINE)
        return LIFT_EINVAL;
    if (rt != LIFT_F32 && rt != LIFT_F64)
        return LIFT_EINVAL;
    const int eb = elem_bytes(storage), rb = elem_bytes(rt);
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, TOP_BATCH, storage, acc, 0, &st);
    if (st != LIFT_OK)
        return st;
    Knobs k;
    st = resolve(knobs, DEF_BATCH, eb, &k);
    if (st != LIFT_OK)
        return st;
    if (k.vec_bytes < 4)
        return LIFT_EUNSUPPORTED;  // the batched kernels load at least a dword per lane
    if (k.block > 512)
        return LIFT_EUNSUPPORTED;  // built for at most 512 threads (no register spills at 8 loads in flight)
    if (k.row_split == 2)
        return LIFT_EUNSUPPORTED;  // batch gemv tiles use one wavefront per row pair
    const int vb = k.vec_bytes;
    const int64_t e = vb / eb;

    std::vector<std::pair<uintptr_t, uintptr_t>> outs, ins;
    std::vector<BatchProblem> hp((size_t)count);
    std::vector<BatchTile> tiles[2];   // reduction tiles, gemv tiles
    std::vector<int64_t> cost[2];
    int64_t slots = 0, bytes = 0;
    const int64_t step = (int64_t)k.block * k.unroll;
    const int64_t waves = k.block / 64;
    for (int32_t i = 0; i < count; ++i) {
        const lift_problem &q = probs[i];
        BatchProblem &p = hp[(size_t)i];
        std::memset(&p, 0, sizeof p);
        if (q.reserved != 0)
            return LIFT_EINVAL;
        p.kind = q.kind;
        p.n = q.n;
        p.a = q.a;
        p.b = q.b;
        p.out = q.out;
        p.alpha = q.alpha;
        p.beta = q.beta;
        if (q.kind == LIFT_KIND_ASUM || q.kind == LIFT_KIND_DOT) {
            const bool dot = q.kind == LIFT_KIND_DOT;
            if (q.n < 0 || !q.out || !aligned(q.out, rb))
                return LIFT_EINVAL;
            if (q.n > 0 && (!q.a || !aligned(q.a, eb) || (dot && (!q.b || !aligned(q.b, eb)))))
                return LIFT_EINVAL;
            outs.push_back({(uintptr_t)q.out, (uintptr_t)q.out + rb});
            if (q.n > 0) {
                ins.push_back({(uintptr_t)q.a, (uintptr_t)q.a + q.n * eb});
                if (dot)
                    ins.push_back({(uintptr_t)q.b, (uintptr_t)q.b + q.n * eb});
            }
            Split3 sp{0, 0};
            int64_t unit_e = e;
            p.vec = 1;
            if (q.n > 0 && !split3(q.a, dot ? q.b : nullptr, q.n, eb, vb, &sp)) {
                p.vec = 0;
                unit_e = 1;
                sp.head = 0;
                sp.nvec = q.n;
            }
            p.head = sp.head;
            p.nvec = sp.nvec;
            // tile length in units (vectors or elements), whole steps
            int64_t len = std::max<int64_t>(1, (k.split + unit_e - 1) / unit_e);
            len = (len + step - 1) / step * step;
            const int64_t nt = std::max<int64_t>(1, (p.nvec + len - 1) / len);
            if (nt > INT32_MAX)
                return LIFT_EUNSUPPORTED;
            p.ntiles = (int32_t)nt;
            p.slot_base = slots;
            slots += nt;
            for (int64_t t = 0; t < nt; ++t) {
                BatchTile tl{i, (int32_t)t, t * len, std::min(len, p.nvec - t * len)};
                if (tl.len < 0)
                    tl.len = 0;
                tiles[0].push_back(tl);
                cost[0].push_back(tl.len * unit_e * eb * (dot ? 2 : 1));
            }
            bytes += q.n * eb * (dot ? 2 : 1) + rb;
        } else if (q.kind == LIFT_KIND_GEMV) {
            if (q.m < 0 || q.n < 0 || q.lda < std::max<int64_t>(1, q.n))
                return LIFT_EINVAL;
            p.m = q.m;
            p.lda = q.lda;
            if (q.m > 0 && (!q.out || !aligned(q.out, 4)))
                return LIFT_EINVAL;
            if (q.m > 0 && q.n > 0 && (!q.a || !q.b || !aligned(q.a, eb) || !aligned(q.b, 4)))
                return LIFT_EINVAL;
            if (q.m == 0)
                continue;
            outs.push_back({(uintptr_t)q.out, (uintptr_t)q.out + q.m * 4});
            if (q.n > 0) {
                ins.push_back({(uintptr_t)q.a, (uintptr_t)q.a + ((q.m - 1) * q.lda + q.n) * eb});
                ins.push_back({(uintptr_t)q.b, (uintptr_t)q.b + q.n * 4});
            }
            const int64_t xalign = std::min<int64_t>(e * 4, 16);
            p.vec = q.n > 0 && aligned(q.a, vb) && (q.lda * eb) % vb == 0 && aligned(q.b, xalign);
            // rows with heads against shifted copies of x in LDS, for rows with
            // at least one vector per lane (shorter ones keep element loads,
            // two rows per wavefront)
            if (!p.vec && e > 1 && vb <= 8 && q.n >= 64 * e && e * ((q.n + 3) / 4 * 4) <= BATCH_LDS_X)
                p.vec = 2;
            p.nvec = p.vec == 1 ? q.n / e : q.n;
            int64_t rows = std::max<int64_t>(1, k.split / std::max<int64_t>(1, q.n));
            // a wavefront pays a memory round trip per row pair whatever the
            // rows' length: at most 16 row pairs per wavefront in a tile, so
            // short rows spread over many work-groups
            rows = std::min<int64_t>(rows, waves * 2 * 16);
            rows = (rows + waves - 1) / waves * waves;
            const int64_t nt = (q.m + rows - 1) / rows;
            if (nt > INT32_MAX)
                return LIFT_EUNSUPPORTED;
            p.ntiles = (int32_t)nt;
            for (int64_t t = 0; t < nt; ++t) {
                BatchTile tl{i, (int32_t)t, t * rows, std::min(rows, q.m - t * rows)};
                tiles[1].push_back(tl);
                // a row shorter than one step of loads costs about a whole step
                cost[1].push_back(tl.len * std::max<int64_t>(q.n, 64 * k.unroll * e) * eb);
            }
            bytes += q.m * q.n * eb + q.n * 4 + q.m * 4 + (q.beta != 0.f ? q.m * 4 : 0);
        } else {
            return LIFT_EINVAL;
        }
    }
    if (any_overlap(outs, ins))
        return LIFT_EINVAL;
    if ((int64_t)tiles[0].size() > INT32_MAX || (int64_t)tiles[1].size() > INT32_MAX || count > 0x7fffffff)
        return LIFT_EUNSUPPORTED;

    // each kind's tiles largest first, so its dynamic schedule ends on small ones
    std::vector<BatchTile> sorted[2];
    for (int kd = 0; kd < 2; ++kd) {
        std::vector<int64_t> order(tiles[kd].size());
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t x, int64_t y) { return cost[kd][x] > cost[kd][y]; });
        sorted[kd].resize(tiles[kd].size());
        for (size_t i = 0; i < order.size(); ++i)
            sorted[kd][i] = tiles[kd][(size_t)order[i]];
    }

    // Each launch's grid: at most wg_per_cu work-groups per CU, and no more
    // than fit on one at once.  (A persistent grid larger than what the CUs
    // hold would park the excess work-groups until resident ones drain the
    // tile counter; each would then run its first tile, taken by index and
    // among the largest, at the end of the launch.)
    const void *kern[2] = {batch_table(storage, acc, vb, k.unroll, false),
                           batch_table(storage, acc, vb, k.unroll, true)};
    if (!kern[0] || !kern[1])
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    int64_t resident[2];
    for (int kd = 0; kd < 2; ++kd) {
        int fit = 1;
        st = resident_per_cu(kern[kd], k.block, &fit);
        if (st != LIFT_OK)
            return st;
        resident[kd] = (int64_t)cus * std::min<int64_t>(k.wg_per_cu, fit);
    }
    // The gemv launch's last round of tiles (one per work-group) is cut in
    // quarters of whole row groups: the launch then ends on short tiles, so
    // its work-groups finish within a fraction of a tile of one another.
    // (A gemv row's result does not depend on its tile; the reduction tiles
    // are the problems' work-group chunks and stay as planned.)
    {
        std::vector<BatchTile> &g = sorted[1];
        const size_t cut = g.size() - (size_t)std::min<int64_t>((int64_t)g.size(), resident[1]);
        std::vector<std::pair<int64_t, BatchTile>> pieces;
        for (size_t i = cut; i < g.size(); ++i) {
            const BatchTile tl = g[i];
            const int64_t n = hp[tl.problem].n;
            const int64_t group = 2 * e;   // a row pair, or a heads tile's pairs of every phase
            const int64_t sub = std::max<int64_t>(group, ((tl.len + 3) / 4 + group - 1) / group * group);
            for (int64_t r = 0; r < tl.len; r += sub) {
                BatchTile pc{tl.problem, tl.index, tl.begin + r, std::min(sub, tl.len - r)};
                pieces.push_back({pc.len * std::max<int64_t>(n, 64 * k.unroll * e) * eb, pc});
            }
        }
        std::stable_sort(pieces.begin(), pieces.end(),
                         [](const auto &x, const auto &y) { return x.first > y.first; });
        g.resize(cut);
        for (const auto &pc : pieces)
            g.push_back(pc.second);
    }
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess)
        return hip_fail(he);

    // one allocation: per launch (reductions, gemv) counters | group
    // counters, then per-problem counters | problems | reduction tiles | gemv
    // tiles | slots
    auto up = [](int64_t v) { return (v + 255) / 256 * 256; };
    int64_t grid[2], off_ct[2], off_gc[2], off = 0;
    for (int kd = 0; kd < 2; ++kd) {
        grid[kd] = std::max<int64_t>(1, std::min<int64_t>(resident[kd], (int64_t)sorted[kd].size()));
        off_ct[kd] = off;
        off_gc[kd] = off + 256;
        off = off_gc[kd] + up((grid[kd] + ARRIVAL_GROUP - 1) / ARRIVAL_GROUP * WS_GROUP_STRIDE);
    }
    const int64_t off_pc = off;
    const int64_t off_pr = off_pc + up(std::max<int64_t>(count, 1) * 4);
    const int64_t off_ti0 = off_pr + up(std::max<int64_t>(count, 1) * (int64_t)sizeof(BatchProblem));
    const int64_t off_ti1 = off_ti0 + up(std::max<int64_t>((int64_t)sorted[0].size(), 1) * (int64_t)sizeof(BatchTile));
    const int64_t off_sl = off_ti1 + up(std::max<int64_t>((int64_t)sorted[1].size(), 1) * (int64_t)sizeof(BatchTile));
    const int64_t total = off_sl + std::max<int64_t>(slots, 1) * WS_SLOT;
    void *mem = nullptr;
    he = hipMalloc(&mem, (size_t)total);
    if (he != hipSuccess)
        return hip_fail(he);
    char *base = (char *)mem;
    if ((he = hipMemset(base, 0, (size_t)off_pr)) != hipSuccess ||
        (count > 0 && (he = hipMemcpy(base + off_pr, hp.data(), hp.size() * sizeof(BatchProblem),
                                      hipMemcpyHostToDevice)) != hipSuccess) ||
        (!sorted[0].empty() && (he = hipMemcpy(base + off_ti0, sorted[0].data(), sorted[0].size() * sizeof(BatchTile),
                                               hipMemcpyHostToDevice)) != hipSuccess) ||
        (!sorted[1].empty() && (he = hipMemcpy(base + off_ti1, sorted[1].data(), sorted[1].size() * sizeof(BatchTile),
                                               hipMemcpyHostToDevice)) != hipSuccess)) {
        hipFree(mem);
        return hip_fail(he);
    }
    for (hipEvent_t &ev : b->ev) {
        if ((he = hipEventCreate(&ev)) != hipSuccess) {
            for (hipEvent_t &e2 : b->ev)
                if (e2) {
                    hipEventDestroy(e2);
                    e2 = nullptr;
                }
            hipFree(mem);
            return hip_fail(he);
        }
    }
    b->device = dev;
    b->storage = storage;
    b->acc = acc;
    b->vb = vb;
    b->unroll = k.unroll;
    b->nprobs = count;
    b->bytes = bytes;
    b->block = k.block;
    b->dmem = mem;
    for (int kd = 0; kd < 2; ++kd) {
        b->ntiles[kd] = (int64_t)sorted[kd].size();
        b->grid[kd] = grid[kd];
        b->kern[kd] = kern[kd];
        BatchArgs &a = b->args[kd];
        a.probs = (const BatchProblem *)(base + off_pr);
        a.tiles = (const BatchTile *)(base + (kd == 0 ? off_ti0 : off_ti1));
        a.counters = (unsigned *)(base + off_ct[kd]);
        a.groups = base + off_gc[kd];
        a.pcount = (unsigned *)(base + off_pc);
        a.slots = base + off_sl;
        a.ntiles = b->ntiles[kd];
        a.result_f64 = rt == LIFT_F64;
    }
    return LIFT_OK;
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
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, TOP_SCAL, LIFT_F32, LIFT_ACC_F32, n, &st);
    if (st != LIFT_OK)
        return st;
    Knobs k;
    st = resolve(knobs, DEF_SCAL, 4, &k);
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
    const int64_t chunk = chunk_for(sp.nvec, vb / 4, k, cus, MAX_DISPATCH_ITEMS / k.block);
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

lift_status lift_dot_ex_noalloc(int64_t n, lift_dtype xt, const void *x, const void *y, lift_acc acc,
                                lift_dtype rt, void *result, const lift_knobs *knobs, hipStream_t stream)
{
    lift_status st = reduce_check(OP_DOT, n, xt, x, y, acc, rt, result);
    if (st != LIFT_OK)
        return st;
    Knobs checked;  // explicit knobs and the override are checked before the first HIP call
    if (knobs && (st = resolve(knobs, DEF_REDUCE, elem_bytes(xt), &checked, true)) != LIFT_OK)
        return st;
    if (!knobs && forced_config().present && !forced_config().valid)
        return LIFT_EINVAL;
    static_assert(STATIC_SCRATCH_BYTES >= (size_t)(WS_HEADER + (int64_t)MAX_WORKGROUPS * WS_SLOT),
                  "the array holds a partial for the largest grid a reduction launches");
    void *ws = nullptr;
    st = static_scratch(&ws);
    if (st != LIFT_OK)
        return st;
    return reduce_common(OP_DOT, n, xt, x, y, acc, rt, result, ws, STATIC_SCRATCH_BYTES, knobs, stream);
}

lift_status lift_blackscholes_ex(int64_t n, const float *s, float strike, float rate, float volatility,
                                 float years, float *call_put, const lift_knobs *knobs, hipStream_t stream)
{
    if (n < 0)
        return LIFT_EINVAL;
    if (n > 0 && (!s || !call_put || !aligned(s, 4) || !aligned(call_put, 8)))
        return LIFT_EINVAL;
    if (overlaps(s, n * 4, call_put, n * 8))
        return LIFT_EINVAL;
    if (!(strike > 0.f) || !std::isfinite(strike) || !(volatility > 0.f) || !std::isfinite(volatility) ||
        !(years > 0.f) || !std::isfinite(years) || !std::isfinite(rate))
        return LIFT_EINVAL;
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, TOP_BS, LIFT_F32, LIFT_ACC_F32, n, &st);
    if (st != LIFT_OK)
        return st;
    Knobs k;
    st = resolve(knobs, DEF_BS, 4, &k);
    if (st != LIFT_OK)
        return st;
    if (k.vec_bytes < 4)
        return LIFT_EINVAL;
    if (n == 0)
        return LIFT_OK;
    // vector path: prices vb-aligned after the head, and the head's pairs
    // aligned for the pair stores (2 vb bytes, at most 16 per store)
    int vb = k.vec_bytes;
    Split3 sp;
    split3(s, nullptr, n, 4, vb, &sp);
    const uintptr_t out_head = reinterpret_cast<uintptr_t>(call_put) + (uintptr_t)sp.head * 8;
    if (out_head % (uintptr_t)std::min(2 * vb, 16) != 0) {
        vb = 4;
        split3(s, nullptr, n, 4, vb, &sp);
    }
    const void *kern = blackscholes_kernel_table(vb, k.unroll);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    int cus = 0;
    st = cu_count(&cus);
    if (st != LIFT_OK)
        return st;
    const int64_t chunk = chunk_for(sp.nvec, vb / 4, k, cus, MAX_DISPATCH_ITEMS / k.block);
    BsArgs a;
    a.s = s;
    a.call_put = call_put;
    a.n = n;
    a.head = sp.head;
    a.nvec = sp.nvec;
    a.chunk = chunk;
    const double K = strike, r = rate, v = volatility, T = years;
    const double vst = v * std::sqrt(T);
    a.ln2_over_vst = (float)(std::log(2.0) / vst);
    a.d1_offset = (float)(((r + 0.5 * v * v) * T - std::log(K)) / vst);
    a.vol_sqrt_t = (float)vst;
    a.strike_disc = (float)(K * std::exp(-r * T));
    const int64_t grid = std::max<int64_t>(1, (sp.nvec + chunk - 1) / chunk);
    return launch(kern, grid, k.block, &a, stream);
}

lift_status lift_blackscholes(int64_t n, const float *s, float strike, float rate, float volatility,
                              float years, float *call_put, hipStream_t stream)
{
    return lift_blackscholes_ex(n, s, strike, rate, volatility, years, call_put, nullptr, stream);
}

lift_status lift_md_ex(int64_t n, const float *pos, int64_t k, const int32_t *nbr, float cutoff,
                       float epsilon, float sigma, float *force, const lift_knobs *knobs,
                       hipStream_t stream)
{
    if (n < 0 || k < 0 || n > INT32_MAX)
        return LIFT_EINVAL;
    if (n > 0 && (!pos || !force || !aligned(pos, 16) || !aligned(force, 16)))
        return LIFT_EINVAL;
    if (n > 0 && k > 0 && (!nbr || !aligned(nbr, 4)))
        return LIFT_EINVAL;
    if (n > 0 && k > INT64_MAX / 4 / n)
        return LIFT_EINVAL;
    if (overlaps(force, n * 16, pos, n * 16) || overlaps(force, n * 16, nbr, n > 0 ? n * k * 4 : 0))
        return LIFT_EINVAL;
    if (!(cutoff >= 0.f) || !std::isfinite(cutoff) || !(sigma > 0.f) || !std::isfinite(sigma) ||
        !std::isfinite(epsilon))
        return LIFT_EINVAL;
    lift_status st = LIFT_OK;
    knobs = effective_knobs(knobs, TOP_MD, LIFT_F32, LIFT_ACC_F32, n * k, &st);
    if (st != LIFT_OK)
        return st;
    Knobs kn;
    st = resolve(knobs, DEF_MD, 4, &kn);
    if (st != LIFT_OK)
        return st;
    if (kn.vec_bytes < 4 || kn.unroll > 4)
        return LIFT_EINVAL;
    if (n * kn.lanes > MAX_DISPATCH_ITEMS - kn.block)  // one thread per lane of each particle
        return LIFT_EINVAL;
    if (n == 0)
        return LIFT_OK;
    // V indices per load when every row starts V-aligned
    int v = kn.vec_bytes / 4;
    while (v > 1 && (k % v != 0 || !aligned(nbr, (size_t)v * 4)))
        v /= 2;
    const void *kern = md_kernel_table(kn.lanes, v, kn.unroll);
    if (!kern)
        return LIFT_EUNSUPPORTED;
    MdArgs a;
    a.pos = pos;
    a.nbr = nbr;
    a.force = force;
    a.n = n;
    a.k = k;
    a.t2 = (float)((double)cutoff * (double)cutoff);
    a.sigma2 = (float)((double)sigma * (double)sigma);
    a.eps24 = (float)(24.0 * (double)epsilon);
    const int64_t threads = n * kn.lanes;
    const int64_t grid = (threads + kn.block - 1) / kn.block;
    return launch(kern, grid, kn.block, &a, stream);
}

lift_status lift_md(int64_t n, const float *pos, int64_t k, const int32_t *nbr, float cutoff, float epsilon,
                    float sigma, float *force, hipStream_t stream)
{
    return lift_md_ex(n, pos, k, nbr, cutoff, epsilon, sigma, force, nullptr, stream);
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

lift_status lift_batch_create(const lift_problem *probs, int32_t count, lift_dtype storage, lift_acc acc,
                              lift_dtype rt, const lift_knobs *knobs, lift_batch **out)
{
    if (!out)
        return LIFT_EINVAL;
    *out = nullptr;
    lift_batch *b = new (std::nothrow) lift_batch();
    if (!b)
        return LIFT_EUNSUPPORTED;
    lift_status st = batch_plan(probs, count, storage, acc, rt, knobs, b);
    if (st != LIFT_OK) {
        delete b;
        return st;
    }
    *out = b;
    return LIFT_OK;
}

lift_status lift_batch_run(lift_batch *b, hipStream_t stream)
{
    if (!b)
        return LIFT_EINVAL;
    if (b->ntiles[0] + b->ntiles[1] == 0)
        return LIFT_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e);
    if (dev != b->device)
        return LIFT_EINVAL;
    // An armed timing hook covers the whole run: its start event goes with
    // the first launch and its stop event with the last (the batch's own
    // pair of events fills the other ends when there are two launches).
    const hipEvent_t t0 = g_time_start, t1 = g_time_stop;
    g_time_start = g_time_stop = nullptr;
    // an armed stamp hook takes both launches' stamped instances (one-shot)
    const void *kern[2] = {b->kern[0], b->kern[1]};
    int64_t grid[2] = {b->grid[0], b->grid[1]};
    uint64_t *stamps = nullptr;
    if (g_stamps) {
        stamps = g_stamps;
        const int64_t cap = g_stamp_capacity;
        g_stamps = nullptr;
        if (b->acc != LIFT_ACC_F32 || (b->storage != LIFT_F32 && b->storage != LIFT_BF16))
            return LIFT_EUNSUPPORTED;
        if (b->ntiles[0] + b->ntiles[1] > cap)
            return LIFT_EINVAL;
        int cus = 0;
        lift_status st = cu_count(&cus);
        if (st != LIFT_OK)
            return st;
        for (int kd = 0; kd < 2; ++kd) {
            kern[kd] = b->storage == LIFT_F32 ? batch_stamped_f32(b->vb, b->unroll, kd == 1)
                                              : batch_stamped_bf16(b->vb, b->unroll, kd == 1);
            if (!kern[kd])
                return LIFT_EUNSUPPORTED;
            int fit = 1;
            if ((st = resident_per_cu(kern[kd], b->block, &fit)) != LIFT_OK)
                return st;
            grid[kd] = std::min<int64_t>(grid[kd], (int64_t)cus * fit);
        }
    }
    const int first = b->ntiles[0] > 0 ? 0 : 1, last = b->ntiles[1] > 0 ? 1 : 0;
    for (int kd = first; kd <= last; ++kd) {
        if (b->ntiles[kd] == 0)
            continue;
        if (t0) {
            g_time_start = kd == first ? t0 : b->ev[1];
            g_time_stop = kd == last ? t1 : b->ev[0];
        }
        BatchArgs a = b->args[kd];
        if (stamps)  // the reduction tiles' words first, then the gemv tiles'
            a.stamps = stamps + (kd == 1 ? b->ntiles[0] : 0) * STAMPS_PER_TILE;
        lift_status st = launch(kern[kd], grid[kd], b->block, &a, stream);
        if (st != LIFT_OK) {
            g_time_start = g_time_stop = nullptr;
            return st;
        }
    }
    return LIFT_OK;
}

lift_status lift_batch_capture(lift_batch *b, hipStream_t stream, hipGraphExec_t *exec)
{
    if (!b || !exec || !stream)
        return LIFT_EINVAL;
    *exec = nullptr;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
        return hip_fail(e);
    lift_status st = lift_batch_run(b, stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(stream, &graph);
    if (st != LIFT_OK) {
        if (graph)
            hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess)
        return hip_fail(e);
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
        *exec = nullptr;
        return hip_fail(e);
    }
    return LIFT_OK;
}

lift_status lift_batch_info(const lift_batch *b, int64_t *tiles, int64_t *grid, int64_t *bytes)
{
    if (!b)
        return LIFT_EINVAL;
    if (tiles)
        *tiles = b->ntiles[0] + b->ntiles[1];
    if (grid)
        *grid = (b->ntiles[0] ? b->grid[0] : 0) + (b->ntiles[1] ? b->grid[1] : 0);
    if (bytes)
        *bytes = b->bytes;
    return LIFT_OK;
}

void lift_batch_destroy(lift_batch *b)
{
    if (!b)
        return;
    if (b->dmem)
        hipFree(b->dmem);
    for (hipEvent_t ev : b->ev)
        if (ev)
            hipEventDestroy(ev);
    delete b;
}

lift_status lift_stream_read(int64_t n, const float *x, float *sink, const lift_knobs *knobs,
                             hipStream_t stream)
{
    return stream_common(false, n, x, sink, knobs, stream);
}

lift_status lift_stream_copy(int64_t n, const float *x, float *out, const lift_knobs *knobs,
                             hipStream_t stream)
{
    return stream_common(true, n, x, out, knobs, stream);
}

int32_t lift_default_knobs(const char *op, lift_dtype storage, lift_acc acc, int64_t elements, int64_t row_length,
                           const char *arch, int32_t cus, lift_knobs *out)
{
    if (!op || !out || elements < 0 || row_length < 0)
        return LIFT_EINVAL;
    if (storage != LIFT_F32 && storage != LIFT_BF16 && storage != LIFT_F16)
        return LIFT_EINVAL;
    if (acc != LIFT_ACC_F32 && acc != LIFT_ACC_F32_COMP && acc != LIFT_ACC_F32_F64COMBINE)
        return LIFT_EINVAL;
    int top = -1;
    for (int i = 0; i < TOP_COUNT; ++i)
        if (std::strcmp(op, TUNED_OP_NAMES[i]) == 0)
            top = i;
    if (top < 0)
        return LIFT_EINVAL;
    std::memset(out, 0, sizeof *out);
    const Forced &f = forced_config();
    if (f.present) {
        if (!f.valid)
            return LIFT_EINVAL;
        *out = f.knobs;
        return 2;
    }
    if (!arch && !device_identity(&arch, &cus))
        return LIFT_EHIP;
    const TunedEntry *e = tuned_entry(arch, cus, top, storage, acc, elements, row_length);
    if (!e)
        return 0;
    *out = e->knobs;
    return 1;
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

lift_status lift_stamp_next_launch(uint64_t *stamps, int64_t capacity, int32_t *clock_khz)
{
    if (!stamps) {
        g_stamps = nullptr;
        g_stamp_capacity = 0;
        return LIFT_OK;
    }
    if (capacity <= 0 || !aligned(stamps, 8) || !clock_khz)
        return LIFT_EINVAL;
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess)
        return hip_fail(e);
    *clock_khz = khz;
    g_stamps = stamps;
    g_stamp_capacity = capacity;
    return LIFT_OK;
}

const char *lift_version(void) { return "lift-mi355x 0.1 gfx950"; }

}  // extern "C"
