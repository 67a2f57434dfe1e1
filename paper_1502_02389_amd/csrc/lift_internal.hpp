// Launch descriptors and kernel tables shared by the host library and the
// kernel translation units.  Host code fills one descriptor per call and
// launches the table entry chosen by the knobs.
#pragma once

#include <stdint.h>

namespace lift {

enum Dtype { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2, DT_F64 = 3 };
enum Op { OP_ASUM = 0, OP_DOT = 1 };
enum Acc { ACC_F32 = 0, ACC_COMP = 1, ACC_F64 = 2 };

// Workspace layout: the global arrival counter in the first 256 bytes; one
// group arrival counter per ARRIVAL_GROUP work-groups, each in its own
// 64-byte line; then one 16-byte partial slot per work-group.  Arrivals are
// counted in two levels because agent-scope atomics on a single address
// serialize (about 10 ns each on MI355X) when every work-group finishes at
// once.
constexpr int32_t MAX_WORKGROUPS = 8192;
constexpr int32_t ARRIVAL_GROUP = 16;
constexpr int64_t WS_GROUPS = 256;                      // offset of the group counters
constexpr int64_t WS_GROUP_STRIDE = 64;
constexpr int64_t WS_HEADER = WS_GROUPS + (MAX_WORKGROUPS / ARRIVAL_GROUP) * WS_GROUP_STRIDE;
constexpr int64_t WS_SLOT = 16;

// reduce(add, 0) . map(abs) over x, or reduce(add, 0) . map(mult) . zip(x, y).
// Elements [0, head) are scalars before the first VB-aligned address; then
// nvec aligned vectors; then the scalar tail [head + nvec * E, n).  Work-group
// b owns vectors [b * chunk, min((b + 1) * chunk, nvec)).
struct ReduceArgs {
    const void *x;
    const void *y;
    int64_t n;
    int64_t head;
    int64_t nvec;
    int64_t chunk;
    void *ws;          // header + partial slots (unused when the grid is 1)
    void *result;
    int32_t result_f64;
    int32_t interleave;  // 1: work-group b takes steps b, b + G, ... (grid-stride)
    uint64_t *stamps;    // stamped instances only: STAMPS_PER_WG clock readings per work-group
};

// Clock readings of a stamped reduction launch, per work-group (the device's
// constant wall clock): [0] entry, [1] streaming loop done, [2] work-group
// tree done, [3] partial stored, [4] arrival counted, [5] end (the last
// work-group: after the combine; the others: = [4]); [6] ids: bit 32 set in
// the work-group that combined, bits 16-19 its XCC, bits 0-7 HW_ID[15:8]
// (CU, shader array, shader engine); [7] unused.
constexpr int STAMPS_PER_WG = 8;
const void *reduce_kernel_stamped_f32(int op, int unroll);
// The other lane forms (lift_lane_form 1-3) of asum / dot, binary32
// accumulation, chunk partition.
const void *reduce_lanes_kernel_f32(int op, int vec_bytes, int unroll, int form);
const void *reduce_lanes_kernel_bf16(int op, int vec_bytes, int unroll, int form);

// map(mult(alpha), x) with the same head / vector / tail split.
struct ScalArgs {
    const float *x;
    float *out;
    int64_t n;
    int64_t head;
    int64_t nvec;
    int64_t chunk;
    float alpha;
};

// Bandwidth reference kernels: nvec 16-byte vectors of x read (and copied to
// out), work-group b owning vectors [b * chunk, (b + 1) * chunk) or, with
// interleave, steps b, b + G, ... of block * unroll vectors.  The read kernel
// writes one word to out only if the XOR fold of its loads hits a fixed tag.
struct StreamArgs {
    const void *x;
    void *out;
    int64_t nvec;
    int64_t chunk;
    int32_t interleave;
};

// y = alpha * A x + beta * y; rows are handled R at a time by one wavefront;
// each row has nvec aligned vectors followed by n - nvec * E scalar columns.
struct GemvArgs {
    const void *A;
    const float *x;
    float *y;
    int64_t m;
    int64_t n;
    int64_t lda;
    int64_t nvec;
    float alpha;
    float beta;
};

// ---- batched form ----------------------------------------------------------

enum Kind { KIND_ASUM = 0, KIND_DOT = 1, KIND_GEMV = 2 };

// One problem of a batch, as the kernel reads it.  Reductions: the element
// range is head scalars, nvec vectors of the batch's vector width (or, when
// vec == 0, nvec = n single elements), then the scalar tail.  gemv: rows of
// lda elements, nvec vectors per row when vec == 1; vec == 2: rows whose
// starts fall inside a vector, each read as a scalar head, whole vectors and
// a scalar tail, against copies of x in LDS shifted by the head.
struct BatchProblem {
    int32_t kind;
    int32_t vec;        // 1: vector loads; 0: element loads; 2: gemv rows with heads
    int32_t ntiles;
    int32_t pad;
    int64_t n;          // elements (reductions) or columns (gemv)
    int64_t m;          // gemv rows
    int64_t lda;
    int64_t head;
    int64_t nvec;
    int64_t slot_base;  // first partial slot of this problem
    const void *a;
    const void *b;
    void *out;
    float alpha;
    float beta;
};

// Floats of x that a batch gemv work-group holds in LDS: one copy (rows of at
// most this many columns), or, for rows with heads, E = vector width / element
// size copies shifted by 0 .. E - 1 elements, each padded to a multiple of 4
// floats.  64 KiB with the work-group's other LDS.
constexpr int64_t BATCH_LDS_X = 16320;

// One tile: vectors (or elements) [begin, begin + len) of a reduction, or
// rows [begin, begin + len) of a gemv.
struct BatchTile {
    int32_t problem;
    int32_t index;      // tile number within its problem
    int64_t begin;
    int64_t len;
};

// Device state of a batch: [next tile | finished work-groups] counters, the
// group counters of the two-level arrival of finished work-groups, one
// arrival counter per problem, and 16-byte partial slots.  Work-group b
// starts with tile b; the next-tile counter hands out tiles from the grid
// size on.
struct BatchArgs {
    const BatchProblem *probs;
    const BatchTile *tiles;
    unsigned *counters;   // [0] next tile (minus grid size), [1] work-groups done
    char *groups;         // ceil(grid / ARRIVAL_GROUP) counters, WS_GROUP_STRIDE apart
    unsigned *pcount;     // per problem: tiles finished
    char *slots;
    int64_t ntiles;
    int32_t result_f64;
    uint64_t *stamps;     // stamped instances only: STAMPS_PER_TILE words per tile
};

// Clock readings of a stamped batch launch, per tile (indexed by its place
// in that launch's tile table): [0] the work-group starts the tile, [1] it
// is done with it, [2] the tile's problem (high 32 bits) and length (low
// 32: units of a reduction tile -- vectors, or elements where its problem
// is read element-wise -- rows of a gemv tile), [3] ids (high 32
// bits: bits 16-19 XCC, bits 0-7 HW_ID[15:8]) and the work-group (low 32).
constexpr int STAMPS_PER_TILE = 4;
const void *batch_stamped_f32(int vec_bytes, int unroll, bool gemv);
const void *batch_stamped_bf16(int vec_bytes, int unroll, bool gemv);

const void *batch_kernel_f32(int acc, int vec_bytes, int unroll, bool gemv);
const void *batch_kernel_bf16(int acc, int vec_bytes, int unroll, bool gemv);
const void *batch_kernel_f16(int acc, int vec_bytes, int unroll, bool gemv);

// Kernel tables (nullptr where a combination is not built).
const void *reduce_kernel(int dtype, int op, int acc, int vec_bytes, int unroll);
const void *scal_kernel(int vec_bytes, int unroll);
const void *stream_kernel(bool copy, int unroll);
const void *gemv_kernel(int dtype, int acc, int vec_bytes, int rows, int unroll);

// Per-dtype tables, one per translation unit.
const void *reduce_kernel_f32(int op, int acc, int vec_bytes, int unroll);
const void *reduce_kernel_bf16(int op, int acc, int vec_bytes, int unroll);
const void *reduce_kernel_f16(int op, int acc, int vec_bytes, int unroll);
const void *gemv_kernel_f32(int acc, int vec_bytes, int rows, int unroll);
const void *gemv_kernel_bf16(int acc, int vec_bytes, int rows, int unroll);
const void *gemv_kernel_f16(int acc, int vec_bytes, int rows, int unroll);
const void *gemv_split_kernel_f32(int acc, int vec_bytes, int rows, int unroll, bool x_stationary);
const void *gemv_split_kernel_bf16(int acc, int vec_bytes, int rows, int unroll, bool x_stationary);
const void *gemv_split_kernel_f16(int acc, int vec_bytes, int rows, int unroll, bool x_stationary);

}  // namespace lift
