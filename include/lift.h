/*
 * lift.h -- C ABI of the MI355X (gfx950) map/reduce BLAS library.
 *
 * The operations are the linear-algebra programs of Steuwer, Fensch and
 * Dubach, "Patterns and Rewrite Rules for Systematic Code Generation"
 * (arXiv 1502.02389), Section 5.1 and its BLAS figure (Fig. 5):
 *
 *   scal(a, x)          = map(mult(a), x)
 *   asum(x)             = reduce(add, 0) . map(abs, x)
 *   dot(x, y)           = reduce(add, 0) . map(mult) . zip(x, y)
 *   gemv(A, x, y, a, b) : z = map(scal(a) . dot(x), A);
 *                         y' = map(add) . zip(z, scal(b, y))      (y = aAx + by)
 *
 * Each call runs hand-written HIP kernels for gfx950; nothing runs on the
 * host but argument checks and launch set-up.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Pointers.   Every array pointer is a DEVICE pointer (hipMalloc'd or any
 *             allocation the device can address), aligned to its element
 *             size.  Other alignment is not required: misaligned heads and
 *             tails are handled inside the kernels.  The caller owns every
 *             buffer; the library keeps no pointer after a call returns.
 * Sizes.      int64_t element counts; negative sizes are rejected.  An empty
 *             reduction (n == 0) writes 0, as reduce of the empty array is
 *             [z] (Table 1); scal with n == 0 and gemv with m == 0 do nothing;
 *             gemv with n == 0 computes y = b*y.
 * Streams.    Work is enqueued on `stream` (0 = the null stream) and the call
 *             returns without synchronising.  Results are valid once the
 *             stream has reached the call.  No call allocates memory, copies
 *             to or from the host, or records a memset, so every call can be
 *             captured into a HIP graph.
 * Results.    A reduction writes its scalar to DEVICE memory (`result`): the
 *             paper's reduce returns a one-element array, T[] -> T[1].
 * Workspace.  asum and dot take a device workspace `ws` of `ws_bytes` bytes,
 *             at least lift_workspace_bytes().  It must be zero-filled ONCE
 *             before its first use; every call leaves it zeroed again (the
 *             last work-group resets the counter it uses), so replays need
 *             no memset.  Calls that may run concurrently (different streams)
 *             need different workspaces.
 * Errors.     Arguments are checked before any HIP call.  LIFT_EINVAL: bad
 *             size, null pointer with a non-empty extent, pointer not aligned
 *             to its element size, partial overlap of an output with an
 *             input, unknown enum or knob value.  LIFT_EWORKSPACE: ws too
 *             small or null.  LIFT_EUNSUPPORTED: a knob combination with no
 *             kernel instance, or a launch that would exceed the 2^32
 *             work-items one dispatch can count (the library sizes its own
 *             grids below that).  LIFT_EHIP: a HIP runtime call failed; its
 *             code is in lift_last_hip_error().  Nothing is enqueued on error.
 * Determinism. For a given size, pointer alignment and knob set, the work
 *             partition and every summation order are fixed, so results are
 *             bitwise reproducible run to run.  Different knobs associate the
 *             floating-point sums differently (the paper's reduction rule,
 *             Fig. 3d, allows any partition); integer-valued inputs whose
 *             partial sums stay below 2^24 in magnitude give identical
 *             results under every knob set.  The cross-work-group combine
 *             relies on gfx950's memory behaviour rather than on fences:
 *             partials are written with agent-scope atomic stores (which the
 *             hardware writes through past the XCD-private L2), a work-group
 *             counts in on the arrival counters only after its store has
 *             completed (a wait on the store, not a release fence, which
 *             would write back the whole L2), and the combining work-group
 *             reads the partials with agent-scope atomic loads (which miss
 *             the L2).  Built and tested for gfx950 only.
 */
#ifndef LIFT_H
#define LIFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lift_status {
    LIFT_OK = 0,
    LIFT_EINVAL = -1,
    LIFT_EWORKSPACE = -2,
    LIFT_EHIP = -3,
    LIFT_EUNSUPPORTED = -4
} lift_status;

/* Storage / result types.  The two bound enumerators of lift_dtype and
 * lift_acc are not values: they make every 32-bit integer a representable
 * value of the type, so an out-of-range argument from any caller is read
 * as such and rejected (LIFT_EINVAL) instead of being undefined in C++. */
typedef enum lift_dtype {
    LIFT_F32 = 0,   /* IEEE binary32 */
    LIFT_BF16 = 1,  /* bfloat16: the upper 16 bits of a binary32 */
    LIFT_F16 = 2,   /* IEEE binary16 */
    LIFT_F64 = 3,   /* IEEE binary64 (reduction results only) */
    LIFT_DTYPE_BOUND_LO_ = -0x7fffffff - 1,
    LIFT_DTYPE_BOUND_HI_ = 0x7fffffff
} lift_dtype;

/* Accumulation variants for 16-bit and 32-bit storage. */
typedef enum lift_acc {
    LIFT_ACC_F32 = 0,           /* binary32 accumulation everywhere */
    LIFT_ACC_F32_COMP = 1,      /* compensated binary32: every partial sum is
                                   a (sum, error) pair propagated with the
                                   error-free TwoSum transformation */
    LIFT_ACC_F32_F64COMBINE = 2, /* binary32 within a work-group, binary64 for
                                   the final cross-work-group combine (gemv:
                                   for the cross-lane combine of each row) */
    LIFT_ACC_BOUND_LO_ = -0x7fffffff - 1,
    LIFT_ACC_BOUND_HI_ = 0x7fffffff
} lift_acc;

/* Values of lift_knobs.interleave: how the work-groups of asum and dot
 * divide the vectors among themselves (the work-group level of the paper's
 * reorder, Section 3.3 and Fig. 9). */
typedef enum lift_interleave {
    LIFT_INTERLEAVE_DEFAULT = 0, /* library choice: STRIDE for dot, CHUNK
                                    for asum */
    LIFT_INTERLEAVE_STRIDE = 1,  /* work-group b takes steps of block * unroll
                                    vectors b, b + G, b + 2G, ... (G
                                    work-groups, as many as split gives) */
    LIFT_INTERLEAVE_CHUNK = 2    /* work-group b reduces one contiguous chunk
                                    of split elements */
} lift_interleave;

/* How the lanes of a work-group take and combine their share of its chunk
 * in asum / dot (Section 6.2's choices between reorder-stride and plain
 * split, and between the iterate tree and reduce-seq; Fig. 9c is the last
 * form with one lane).  Bit 0: the lane partials are folded in lane order
 * by one thread instead of the tree; bit 1: lane t reduces the t-th
 * contiguous run of chunk / block vectors instead of vectors t, t + block,
 * ....  Forms other than the default take binary32 accumulation (LIFT_ACC_F32)
 * and F32 or BF16 storage, and the chunk partition (LIFT_INTERLEAVE_STRIDE
 * is LIFT_EINVAL); the sequential forms also take a block of 1 to 32 lanes
 * (a power of two), their final combine then folding the work-group partials
 * over that many lanes. */
typedef enum lift_lane_form {
    LIFT_LANES_TREE = 0,        /* reorder-stride lanes, tree (the default) */
    LIFT_LANES_SEQ = 1,         /* reorder-stride lanes, folded in lane order */
    LIFT_LANES_RUNS_TREE = 2,   /* contiguous runs, tree */
    LIFT_LANES_RUNS_SEQ = 3     /* contiguous runs, folded in lane order */
} lift_lane_form;

/* Launch knobs: the parameters the paper's low-level expressions expose
 * (split factor, work-group size, vector width; Fig. 9 and Section 6.2)
 * plus the rows handled together by one wavefront in gemv.  A zero field
 * selects the library default for that field.
 *
 * Calls that take no knobs, or are passed knobs == NULL, run with
 *   1. the environment override LIFT_FORCE_CONFIG="key=value,..." if set
 *      (read once per process; keys block (or wg), vec, unroll, rpw, split,
 *      wgcu, rowsplit, lanes, interleave = stride | chunk | 1 | 2, laneform; values
 *      non-negative integers; an unknown key or malformed value makes every
 *      such call return LIFT_EINVAL), applied as if the caller had passed
 *      those knobs (fields the op does not use are ignored);
 *   2. else the autotuned knobs for the call's op, storage, accumulation and
 *      size bucket floor(log2(elements)) (gemv: m n, and floor(log2(n)) of
 *      its rows; MD: n k; a batch: one bucket) -- a table built into the library from the autotuner's
 *      cache, used only on a device of the architecture and compute-unit
 *      count it was tuned on;
 *   3. else the library defaults.
 * lift_default_knobs reports which applies.  Explicit knobs are never
 * overridden. */
typedef struct lift_knobs {
    int32_t block;         /* work-group size: 64, 128, 256, 512 or 1024
                              (1 to 32 too for the sequential lane forms)
                              (batched form: at most 512; gemv lowers it to
                              what the instance's registers allow: with
                              many rows x loads in flight, 512 or 256) */
    int32_t vec_bytes;     /* bytes per lane per load: 2 (16-bit storage
                              only), 4, 8 or 16 -- asVector width times the
                              element size */
    int32_t unroll;        /* independent loads in flight per lane: 1, 2, 4, 8 */
    int32_t rows_per_wave; /* gemv only: 1, 2 or 4 rows per wavefront */
    int64_t split;         /* elements per work-group chunk (split^n); the
                              library rounds it up to a whole number of
                              block * unroll loads and caps the grid at
                              lift_max_workgroups().  Batched form: elements
                              per tile (gemv tiles: about this many matrix
                              elements, whole rows) */
    int32_t wg_per_cu;     /* grid size in work-groups per compute unit when
                              split is 0 (per-call forms), the grid cap of
                              the work-group-per-row gemv, and the cap of
                              the persistent grid per compute unit (batched
                              form: never more than fit on a unit at once) */
    int32_t row_split;     /* gemv only: 1 = each wavefront owns rows_per_wave
                              rows; 2 = all threads of a work-group split each
                              row (then rows_per_wave is 1 or 2 and unroll 2,
                              4 or 8; when one pass of block * unroll loads
                              covers a row, each thread keeps its part of x
                              in registers for all its rows); 0 = library
                              choice (2, with a work-group of up to 512
                              threads sized to the row, where x fits in
                              registers; else 1) */
    int32_t lanes_per_item; /* MD only: lanes that share one particle's
                              neighbour list: 1, 2, 4, 8 or 16 */
    int32_t interleave;    /* asum / dot only: a lift_interleave value */
    int32_t lane_form;     /* asum / dot only: a lift_lane_form value */
} lift_knobs;

/* ---- plain FP32 forms (Fig. 5) --------------------------------------- */

/* scal: out[i] = alpha * x[i], one binary32 multiply per element (rounded
 * to nearest even), i in [0, n).  `out` may equal `x` (in place); any other
 * overlap is LIFT_EINVAL. */
lift_status lift_scal(int64_t n, float alpha, const float *x, float *out, hipStream_t stream);

/* asum: *result = sum_i |x_i| in binary32 (binary32 accumulation). */
lift_status lift_asum(int64_t n, const float *x, float *result, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* dot: *result = sum_i x_i * y_i in binary32 (products fused into the
 * accumulation with fma). */
lift_status lift_dot(int64_t n, const float *x, const float *y, float *result, void *ws,
                     size_t ws_bytes, hipStream_t stream);

/* gemv: y[i] = alpha * (sum_j A[i*lda + j] * x[j]) + beta * y[i] for
 * i in [0, m), j in [0, n).  A is row-major (the paper maps the dot over the
 * rows of A) with leading dimension lda >= max(1, n).  alpha multiplies the
 * finished dot once.  beta == 0 follows the BLAS convention: y is written
 * but not read (NaN in y does not propagate).  y must not overlap A or x. */
lift_status lift_gemv(int64_t m, int64_t n, float alpha, const float *A, int64_t lda,
                      const float *x, float beta, float *y, hipStream_t stream);

/* Bytes of workspace any asum/dot call (plain or _ex) needs on this device. */
size_t lift_workspace_bytes(void);

/* Largest work-group count a reduction grid uses. */
int32_t lift_max_workgroups(void);

/* ---- storage / accumulation variants and explicit knobs -------------- */

/* scal with explicit knobs (NULL = defaults). */
lift_status lift_scal_ex(int64_t n, float alpha, const float *x, float *out,
                         const lift_knobs *knobs, hipStream_t stream);

/* asum of x stored as xt (F32, BF16 or F16) with accumulation `acc`; the
 * result is written as rt (F32 or F64) to device memory. */
lift_status lift_asum_ex(int64_t n, lift_dtype xt, const void *x, lift_acc acc, lift_dtype rt,
                         void *result, void *ws, size_t ws_bytes, const lift_knobs *knobs,
                         hipStream_t stream);

/* dot of x and y, both stored as xt (F32, BF16 or F16); 16-bit products
 * are exact in binary32. */
lift_status lift_dot_ex(int64_t n, lift_dtype xt, const void *x, const void *y, lift_acc acc,
                        lift_dtype rt, void *result, void *ws, size_t ws_bytes,
                        const lift_knobs *knobs, hipStream_t stream);

/* lift_dot_ex without a workspace argument, for callers that cannot
 * allocate device memory or pass one (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  The call allocates
 * nothing: its arrival counters and per-work-group partials live in a
 * static device array of 164,096 bytes inside the library (the workspace
 * size of lift_workspace_bytes(), enough for the largest grid any reduction
 * launches, so every n is accepted), one copy per device, held until the
 * process ends.  Same arguments, results (bit for bit, for the same knobs)
 * and errors as lift_dot_ex; the first call on a device also looks up that
 * device's copy (LIFT_EHIP if that fails).  Every call on a device shares
 * its copy: calls that may overlap on one device (different streams, or
 * host threads racing on one stream) race on it and must be serialised by
 * the caller; lift_dot_ex with distinct workspaces is the concurrent form. */
lift_status lift_dot_ex_noalloc(int64_t n, lift_dtype xt, const void *x, const void *y, lift_acc acc,
                                lift_dtype rt, void *result, const lift_knobs *knobs, hipStream_t stream);

/* gemv with A stored as at (F32, BF16 or F16); x and y are binary32. */
lift_status lift_gemv_ex(int64_t m, int64_t n, float alpha, lift_dtype at, const void *A,
                         int64_t lda, const float *x, float beta, float *y, lift_acc acc,
                         const lift_knobs *knobs, hipStream_t stream);

/* ---- BlackScholes (Section 5.2) ----------------------------------------- */

/* BlackScholes: map(BSComputation) over n stock prices s[i] (binary32, > 0).
 * For each price the pair {call, put} of the closed-form model of a European
 * option with the given strike (> 0), risk-free rate, volatility (> 0) and
 * time to expiry in years (> 0), the same for every element:
 *   d1 = (ln(s/K) + (r + v^2/2) T) / (v sqrt T),   d2 = d1 - v sqrt T,
 *   call = s N(d1) - K e^{-rT} N(d2),   put = K e^{-rT} N(-d2) - s N(-d1),
 * N the standard normal distribution function.  call_put[2i] is the call and
 * call_put[2i + 1] the put of s[i] (2n floats, 8-byte aligned, not
 * overlapping s).  Evaluated in binary32: the per-call constants in binary64,
 * rounded once; ln s from the hardware log2; N through a fitted polynomial
 * for the normal tail (absolute error about 2e-7).  Prices must be positive
 * normal binary32 numbers.  LIFT_EINVAL: n < 0, null or misaligned pointers
 * with n > 0, overlap, or a parameter out of its range or not finite. */
lift_status lift_blackscholes(int64_t n, const float *s, float strike, float rate, float volatility,
                              float years, float *call_put, hipStream_t stream);

/* lift_blackscholes with explicit knobs (block, vec_bytes 4/8/16 prices
 * per lane, unroll, split, wg_per_cu; NULL = defaults). */
lift_status lift_blackscholes_ex(int64_t n, const float *s, float strike, float rate, float volatility,
                                 float years, float *call_put, const lift_knobs *knobs,
                                 hipStream_t stream);

/* ---- MD (Fig. 7) ------------------------------------------------------- */

/* MD: the force on every particle from its neighbour list,
 *   md(ps, N, t) = map(lambda (p, ns): reduce(lambda (f, nId):
 *                      updateF(f, nId, p, ps, t), 0, ns)) . zip(ps, N),
 * where updateF adds the pair force of ps[nId] on p when |p - ps[nId]| < t.
 * The pair force (not given in the paper) is Lennard-Jones:
 *   F = 24 eps / r^2 * (2 (sigma^2/r^2)^6 - (sigma^2/r^2)^3) * (p - q).
 * pos:   n particles, 4 floats each (x, y, z, unused), 16-byte aligned.
 * nbr:   n x k int32, row-major (nbr[i*k + j] = j-th neighbour of i); an index
 *        outside [0, n) is an empty slot (lists of uneven length are padded,
 *        e.g. with -1).  A particle must not list itself.
 * force: n x 4 floats (fx, fy, fz, 0), 16-byte aligned, not overlapping pos
 *        or nbr.
 * cutoff >= 0: the test is r^2 < binary32(cutoff^2), taken in binary32 on
 * ((dx dx + dy dy) + dz dz) without contraction, which agrees with the exact
 * |p - q| < cutoff for every pair whose squared distance is more than 6
 * binary32 ulps (relative 6 * 2^-24) from cutoff^2; nearer pairs may fall
 * either way, the same way on every call.  epsilon finite, sigma > 0.
 * Binary32 throughout;
 * the sum over a list is split over the lanes given by lanes_per_item, in a
 * fixed order (deterministic).  LIFT_EINVAL for bad sizes, pointers or
 * parameters; n must be below 2^31, and n * lanes_per_item (one thread per
 * lane of each particle) below 2^32: with the default 16 lanes, n below
 * about 2^28. */
lift_status lift_md(int64_t n, const float *pos, int64_t k, const int32_t *nbr, float cutoff, float epsilon,
                    float sigma, float *force, hipStream_t stream);

/* lift_md with explicit knobs (block, vec_bytes 4/8/16 = indices per load,
 * unroll 1/2/4, lanes_per_item; NULL = defaults). */
lift_status lift_md_ex(int64_t n, const float *pos, int64_t k, const int32_t *nbr, float cutoff,
                       float epsilon, float sigma, float *force, const lift_knobs *knobs,
                       hipStream_t stream);

/* ---- batched form ------------------------------------------------------ */

/* Many asum / dot / gemv problems of uneven size in one run: one persistent
 * launch over the reduction tiles and one over the gemv tiles, enqueued
 * together (each kernel compiled for its own kind of tile).  The paper's
 * split and map-workgroup applied to a list of problems: every problem is
 * cut into tiles (split^n), and a persistent grid of work-groups takes tiles
 * from a shared counter until none are left.  The partials of a reduction
 * are combined by whichever work-group finishes its last tile, in tile
 * order, so results do not depend on which work-group ran which tile.  Each
 * gemv row is reduced by one wavefront (its dot over 64 lanes, as in the
 * per-call form with one row per wavefront): with vector loads where A's
 * rows start on vec_bytes boundaries and x is aligned to
 * min(vec_bytes / element size * 4, 16) bytes; else, for vec_bytes of at
 * most 8, rows of at least 64 * E columns (E = vec_bytes / element size)
 * and E copies of x, each padded to a multiple of 4 floats, fitting in
 * 16320 floats of LDS, each row from its own start: scalars up to its first
 * vec_bytes boundary, then vectors, then the scalar tail (a wavefront takes
 * two rows E apart, which start alike); else with element loads. */
typedef enum lift_kind {
    LIFT_KIND_ASUM = 0,
    LIFT_KIND_DOT = 1,
    LIFT_KIND_GEMV = 2
} lift_kind;

/* One problem; all pointers are device pointers, owned by the caller. */
typedef struct lift_problem {
    int32_t kind;      /* lift_kind */
    int32_t reserved;  /* must be 0 */
    int64_t m;         /* gemv: rows of A (ignored otherwise) */
    int64_t n;         /* asum / dot: elements; gemv: columns of A */
    int64_t lda;       /* gemv: leading dimension, >= max(1, n) */
    const void *a;     /* asum / dot: x (batch storage type); gemv: A (batch storage type) */
    const void *b;     /* dot: y (batch storage type); gemv: x (binary32); asum: unused */
    void *out;         /* asum / dot: result (batch result type); gemv: y (binary32, in/out) */
    float alpha;       /* gemv only */
    float beta;        /* gemv only; 0 means y is not read */
} lift_problem;

typedef struct lift_batch lift_batch;

/* Plan a batch on the current device: checks every problem as the per-call
 * entry points do, builds the tile table (tiles sorted largest first; the
 * gemv launch's last round of tiles, one per work-group, cut in quarters of
 * whole row groups; each launch's grid at most knobs.wg_per_cu work-groups
 * per compute unit and no more than the kernel keeps resident), and
 * allocates and fills one device buffer for descriptors, tiles, partial
 * slots and counters (this call allocates and synchronises; lift_batch_run
 * does neither).  storage: F32, BF16 or F16 for every x, y and A; rt: F32 or
 * F64 for reduction results.  The pointers inside `probs` are recorded: the
 * batch computes on whatever those buffers hold at run time.  On error
 * *out is NULL; LIFT_EINVAL names a bad problem or argument. */
lift_status lift_batch_create(const lift_problem *probs, int32_t count, lift_dtype storage,
                              lift_acc acc, lift_dtype rt, const lift_knobs *knobs,
                              lift_batch **out);

/* Enqueue the whole batch on `stream`: the reduction launch, then the gemv
 * launch (either is skipped when the batch has no tiles of its kind).
 * Allocation-free and memset-free: each kernel leaves its counters reset, so
 * the call can be captured into a HIP graph and replayed.  Runs of one batch
 * must not overlap (they share the counters).  An armed timing hook
 * (lift_time_next_launch) spans the whole run: start with the first launch,
 * stop with the last; an armed stamp hook (lift_stamp_next_launch) makes
 * both launches stamped. */
lift_status lift_batch_run(lift_batch *batch, hipStream_t stream);

/* Capture lift_batch_run on `stream` (which must not be the null stream)
 * into a HIP graph and instantiate it; the caller replays *exec with
 * hipGraphLaunch and destroys it with hipGraphExecDestroy. */
lift_status lift_batch_capture(lift_batch *batch, hipStream_t stream, hipGraphExec_t *exec);

/* Tiles in the plan, work-groups of the run's launches together, and
 * algorithmic HBM bytes of one run (each x, y, A element read once, y of
 * gemv read (beta != 0) and written, results written).  Any pointer may be
 * NULL. */
lift_status lift_batch_info(const lift_batch *batch, int64_t *tiles, int64_t *grid, int64_t *bytes);

/* Free the batch's device memory (synchronises its device).  NULL is a no-op. */
void lift_batch_destroy(lift_batch *batch);

/* ---- diagnostics ------------------------------------------------------ */

/* Bandwidth reference kernels (measurement only; no operation of the paper).
 * They move bytes the way the library's streaming kernels do -- 16-byte
 * nontemporal loads, `unroll` in flight per lane, the reductions' partition
 * into work-group chunks (split / wg_per_cu) or interleaved steps -- with no
 * arithmetic and no cross-work-group combine, so a timed launch gives the
 * achievable rate of one launch of that many bytes, the ceiling a reduction
 * or a map of the same size is measured against.
 * lift_stream_read reads x[0, n) and writes one word to *sink only if the
 *   XOR fold of a lane's loads equals a fixed tag (sink: 4-byte aligned
 *   device word owned by the caller; its contents are unspecified after the
 *   call).
 * lift_stream_copy writes out[i] = x[i] bit for bit (no overlap allowed).
 * n must be a multiple of 4 and x (and out for the copy) 16-byte aligned;
 * knobs: block, unroll, split, wg_per_cu, interleave (vec_bytes 0 or 16);
 * NULL = 256 threads, 8 loads in flight, one work-group per compute unit.
 * LIFT_EINVAL on a bad size, pointer, alignment or overlap. */
lift_status lift_stream_read(int64_t n, const float *x, float *sink, const lift_knobs *knobs,
                             hipStream_t stream);
lift_status lift_stream_copy(int64_t n, const float *x, float *out, const lift_knobs *knobs,
                             hipStream_t stream);

/* Profiling hook.  The NEXT kernel launched by a lift_* call on the calling
 * thread is dispatched with `start` and `stop` recorded inside its own
 * dispatch packet (hipExtLaunchKernel), so hipEventElapsedTime(start, stop)
 * is that kernel's execution time on its stream, with no extra marker
 * packets between kernels.  The caller creates both events (hipEventCreate)
 * on the device of the launch and owns them.  One-shot: the launch clears
 * it; a call rejected before launching leaves it armed; (NULL, NULL)
 * disarms it.  Exactly one NULL is LIFT_EINVAL. */
lift_status lift_time_next_launch(hipEvent_t start, hipEvent_t stop);

/* Diagnostic hook: the NEXT asum or dot launch on the calling thread (binary32
 * storage and accumulation, 16-byte loads) runs the stamped instance of its
 * kernel, identical in arithmetic, which writes 8 words per work-group into
 * `stamps` (device memory owned by the caller, `capacity` work-groups):
 * readings of the device's constant wall clock at entry, when its streaming
 * loop is done, after its work-group tree, once its partial is stored, once
 * its arrival is counted, and at its end (the combining work-group: after
 * the combine), then ids (bit 32: the work-group that combined; bits 16-19:
 * its XCC; bits 0-7: HW_ID[15:8], CU / shader array / shader engine), then
 * one unused word (a launch of one work-group, which writes the result
 * itself, takes the store, arrival and end readings together).  If the next call is lift_batch_run instead (binary32
 * accumulation, F32 or BF16 storage), both of its launches run the stamped
 * instances of their kernels, which write 4 words per tile (`capacity`
 * counts tiles): the reduction tiles in the order of that launch's tile
 * table, then the gemv tiles in theirs.  Per tile: the clock when a
 * work-group takes the tile and when it is done with it, the tile's problem
 * index (high 32 bits) and length (low 32: rows of a gemv tile; vectors, or
 * elements where the problem is read element-wise, of a reduction tile),
 * and ids (high 32 bits, as above) with the work-group (low 32).
 * *clock_khz receives the clock's rate.  One-shot; that run fails with
 * LIFT_EUNSUPPORTED for another storage, accumulation or vector width and
 * LIFT_EINVAL if its tile count exceeds `capacity` (the hook is cleared
 * either way).  stamps == NULL disarms it.
 * LIFT_EINVAL: capacity <= 0, stamps not 8-byte aligned or clock_khz NULL. */
lift_status lift_stamp_next_launch(uint64_t *stamps, int64_t capacity, int32_t *clock_khz);

/* The knobs a call with knobs == NULL would run with on a device of
 * architecture `arch` (e.g. "gfx950"; NULL = the current device, a HIP
 * query) with `cus` compute units (ignored when arch is NULL): op is one of
 * "scal", "asum", "dot", "gemv", "batch", "blackscholes", "md"; elements is
 * the size the bucket is taken of (see lift_knobs); row_length is gemv's n
 * (its entries are also keyed by floor(log2(n)); ignored for other ops).
 * Fills *out (all zero = the library defaults) and returns 2 if
 * LIFT_FORCE_CONFIG applies, 1 for a tuned entry, 0 for the defaults;
 * LIFT_EINVAL for an unknown op, storage or accumulation, a null pointer,
 * negative sizes or a malformed LIFT_FORCE_CONFIG; LIFT_EHIP if the current
 * device cannot be queried. */
int32_t lift_default_knobs(const char *op, lift_dtype storage, lift_acc acc, int64_t elements, int64_t row_length,
                           const char *arch, int32_t cus, lift_knobs *out);

/* Static description of a status code. */
const char *lift_status_string(lift_status status);

/* hipError_t of the last failed HIP call on this thread (0 if none). */
int lift_last_hip_error(void);

/* Library version, e.g. "lift-mi355x 0.1 gfx950". */
const char *lift_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LIFT_H */
