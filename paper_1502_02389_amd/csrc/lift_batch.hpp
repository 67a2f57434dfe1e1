// Batched form: every asum / dot / gemv of a problem list in one run.
//
// The paper's split and map-workgroup over a list of problems.  The host cuts
// every problem into tiles (reductions: runs of vectors; gemv: runs of rows)
// and sorts each kind's tiles largest first (the gemv launch's last round
// of tiles cut in quarters).  A run is two persistent launches on one
// stream, one per kind, so that each kernel is compiled for its own work
// (its register peak sets how many work-groups a CU holds, and the
// reductions' need not limit the gemv's); each grid holds no more
// work-groups than the CUs keep resident.  In each, work-groups take the
// next tile from an agent-scope counter until the table is exhausted:
//   reduction tile -> the per-call streaming body (lane reduce-seq, DPP wave
//                     butterfly, LDS across waves) -> partial slot of the tile;
//                     the work-group that finishes a problem's last tile folds
//                     that problem's partials in tile order and writes its
//                     result (a one-tile problem writes its partial directly);
//   gemv tile      -> each wavefront takes pairs of the tile's rows; where x
//                     fits, the work-group first copies it into LDS (for rows
//                     with heads, E copies shifted by one element each) and
//                     the rows read it there.
// Tile-to-work-group assignment is dynamic, but every tile's arithmetic and
// every combine order are fixed by the plan, so results are deterministic.
// The last work-group to leave a launch resets that launch's counters, so a
// run can be replayed from a HIP graph without a memset node.
#pragma once

#include "lift_gemv.hpp"
#include "lift_reduce.hpp"

namespace lift {

// Streaming phase of one reduction tile: the calling lane's partial.
template <class T, int OP, int ACC, int VB, int U>
__device__ __forceinline__ typename BlockT<ACC>::type tile_lane_value(const BatchProblem &p, const BatchTile &tl)
{
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const char *xv = reinterpret_cast<const char *>(p.a) + p.head * T::bytes;
    const char *yv = OP == OP_DOT ? reinterpret_cast<const char *>(p.b) + p.head * T::bytes : nullptr;
    const int64_t vbeg = tl.begin, vend = tl.begin + tl.len, step = B * U;

    LaneAcc<ACC, E> acc;
    int64_t base = vbeg;
    for (; base + step <= vend; base += step) {
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
    if (tl.index == 0 && t < p.head) {
        float fy = OP == OP_DOT ? load_elem<T>(p.b, t) : 0.f;
        accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(p.a, t), fy);
    }
    const int64_t tail0 = p.head + p.nvec * E;
    if (tl.index == p.ntiles - 1 && t < p.n - tail0) {
        float fy = OP == OP_DOT ? load_elem<T>(p.b, tail0 + t) : 0.f;
        accumulate_scalar<T, OP, ACC, E>(acc, load_elem<T>(p.a, tail0 + t), fy);
    }
    return acc.value();
}

// Rows [begin, begin + len) of a gemv problem, two rows per wavefront at a
// time so the pair shares every x load (x is re-read from cache for each row
// group; with 16-bit A that is otherwise twice A's own bytes): wavefront w
// takes rows begin + 2w, begin + 2w + 2W, ... (W wavefronts per work-group).
// The tile's end stands in for the row count, so a second row past it is
// read at a clamped index and never written: no row of another tile is
// touched.
template <class T, int ACC, int VB, int U>
__device__ __forceinline__ void gemv_tile(const BatchProblem &p, const BatchTile &tl)
{
    constexpr int R = 2;
    const int lane = threadIdx.x & 63;
    const int64_t waves = blockDim.x >> 6;
    const float *x = reinterpret_cast<const float *>(p.b);
    float *y = reinterpret_cast<float *>(p.out);
    const int64_t end = tl.begin + tl.len;
    for (int64_t r = tl.begin + (threadIdx.x >> 6) * R; r < end; r += waves * R)
        gemv_row_group<T, ACC, VB, R, U>(p.a, x, y, end, p.n, p.lda, p.nvec, p.alpha, p.beta, r, lane);
}

// x (n >= 1 floats) into LDS: E copies, copy h at h * stride holding
// x[j + h] at j (one plain copy when E is 1).  Each thread issues its K
// loads of a round (at clamped, in-range indices) before it stores any of
// them, so staging costs one memory round trip per K * blockDim.x floats,
// not one per blockDim.x.  The caller places the barrier.
template <int E>
__device__ __forceinline__ void stage_x(const float *x, int64_t n, float *xl, int64_t stride)
{
    constexpr int K = 8;
    const int64_t B = blockDim.x;
    for (int64_t j0 = threadIdx.x; j0 < n; j0 += K * B) {
        float v[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            v[k] = x[min(j0 + k * B, n - 1)];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t j = j0 + k * B;
            if (j < n) {
#pragma unroll
                for (int h = 0; h < E; ++h)
                    if (j >= h)
                        xl[h * stride + j - h] = v[k];
            }
        }
    }
}

// Rows r0, r0 + rstep, ..., r0 + (R - 1) rstep of a gemv problem, by one
// wavefront, with x in LDS.  The R rows must start at the same offset
// inside a VB-byte vector: rows of a pitch that is a multiple of VB (any
// rstep; then every head is empty), or rstep a multiple of E = VB / element
// size; so they share one head length, one vector count and one copy of x,
// and each x read serves all R rows.  A row from `end` on is replaced by row
// r0 (computed, not written).  Each row: a head of fewer than E columns up
// to its first vector boundary, whole vectors from there (the x vectors they
// meet are read from the copy of x shifted by the head, xl + head * stride,
// which holds x[j + head] at j), and its scalar tail.  Lane t folds vectors
// t, t + 64, ... as in gemv_row_group, then adds its head column (t < head)
// and its tail column to component 0: the order of the low-level dot
// expression with a misaligned start (gemv_row_group's order when there is
// no head), row by row.
template <class T, int ACC, int VB, int R, int UR>
__device__ __forceinline__ void gemv_rows_phase(const BatchProblem &p, int64_t r0, int64_t rstep, int64_t end,
                                                const float *xl, int64_t stride, int lane)
{
    constexpr int E = Elems<T, VB>::value;
    using V = typename Vec<VB>::type;
    float *y = reinterpret_cast<float *>(p.out);
    const char *row[R], *body[R];
    float yold[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t ri = r0 + r * rstep;
        yold[r] = prefetch_y(y, ri, end, p.beta);
        row[r] = reinterpret_cast<const char *>(p.a) + (ri < end ? ri : r0) * p.lda * T::bytes;
    }
    const int64_t head = min((int64_t)__builtin_amdgcn_readfirstlane(
                                 (int)(((VB - (uintptr_t)row[0] % VB) % VB) / T::bytes)), p.n);
    const int64_t nvec = (p.n - head) / E;
#pragma unroll
    for (int r = 0; r < R; ++r)
        body[r] = row[r] + head * T::bytes;
    const float *xs = xl + head * stride;
    // the head and tail columns are read now, so their loads overlap the
    // vectors' instead of costing a dependent round trip at the end; they
    // are added after the vectors, as the expression orders them
    // (loaded at clamped, in-range columns without a branch, so no load
    // waits on its own; decoded and selected at the end)
    const int64_t tail0 = head + nvec * E;
    const bool has_head = lane < head, has_tail = tail0 + lane < p.n;
    const int64_t hcol = min((int64_t)lane, p.n - 1), tcol = min(tail0 + lane, p.n - 1);
    using Raw = typename T::raw;
    Raw hraw[R], traw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        hraw[r] = reinterpret_cast<const Raw *>(row[r])[hcol];
        traw[r] = reinterpret_cast<const Raw *>(row[r])[tcol];
    }
    const float hx = xl[hcol], tx = xl[tcol];

    RowAcc<ACC, E> acc[R];
    int64_t base = 0;
    for (; base + 64 * UR <= nvec; base += 64 * UR) {
        // x from LDS is read together with the row loads, so its latency
        // hides behind theirs
        float xf[UR][E];
#pragma unroll
        for (int k = 0; k < UR; ++k)
            load_x<E>(xs, base + lane + 64 * k, xf[k]);
        V va[R][UR];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < UR; ++k)
                va[r][k] = load_stream<VB>(body[r], base + lane + 64 * k);
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < UR; ++k) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float af[E];
                decode<T, VB>(va[r][k], af);
                acc[r].add(af, xf[k]);
            }
        }
    }
    if (base < nvec) {
        // the last, partial step: clamped indices keep every load in its row;
        // the vectors past the row's end become zeros
        V va[R][UR];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < UR; ++k)
                va[r][k] = load_stream<VB>(body[r], min(base + lane + 64 * k, nvec - 1));
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < UR; ++k) {
            const int64_t v = min(base + lane + 64 * k, nvec - 1);
            const bool in = base + lane + 64 * k < nvec;
            float xf[E];
            load_x<E>(xs, v, xf);
#pragma unroll
            for (int e = 0; e < E; ++e)
                xf[e] = in ? xf[e] : 0.f;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float af[E];
                decode<T, VB>(va[r][k], af);
#pragma unroll
                for (int e = 0; e < E; ++e)
                    af[e] = in ? af[e] : 0.f;
                acc[r].add(af, xf);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (has_head)
            acc[r].add_scalar(decode_raw<T>(hraw[r]), hx);
        if (has_tail)
            acc[r].add_scalar(decode_raw<T>(traw[r]), tx);
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t ri = r0 + r * rstep;
        if constexpr (ACC == ACC_F64) {
            double d = wave_sum((double)acc[r].value());
            if (lane == 0 && ri < end) {
                double by = p.beta == 0.f ? 0.0 : (double)p.beta * (double)yold[r];
                y[ri] = (float)((double)p.alpha * d + by);
            }
        } else if constexpr (ACC == ACC_COMP) {
            Pair q = wave_sum(acc[r].value());
            if (lane == 0 && ri < end)
                store_row_y<ACC>(y, ri, p.alpha, p.beta, q.s + q.c, yold[r]);
        } else {
            float d = wave_sum(acc[r].value());
            if (lane == 0 && ri < end)
                store_row_y<ACC>(y, ri, p.alpha, p.beta, d, yold[r]);
        }
    }
}

// Rows [begin, begin + len) of a gemv problem whose rows start on vector
// boundaries (or are read element by element) and whose x fits in `xl`
// (LDS): the work-group copies x there once per tile, then each wavefront
// takes row pairs as in gemv_tile, reading x from LDS instead of the cache
// (re-reading x from the cache for every row pair limits the wavefront form;
// with 16-bit A, x is twice A's bytes).  The arithmetic is gemv_row_group's,
// so both forms give the same bits.  All threads of the work-group must call
// this (it has barriers).
template <class T, int ACC, int VB, int U>
__device__ __forceinline__ void gemv_tile_lx(const BatchProblem &p, const BatchTile &tl, float *xl)
{
    constexpr int R = 2;
    if (p.n > 0)
        stage_x<1>(reinterpret_cast<const float *>(p.b), p.n, xl, 0);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t waves = blockDim.x >> 6;
    const int64_t end = tl.begin + tl.len;
    // rows start on a vector boundary (or VB is the element size): no heads,
    // the plain copy of x serves every row
    for (int64_t r = tl.begin + (threadIdx.x >> 6) * R; r < end; r += waves * R)
        gemv_rows_phase<T, ACC, VB, R, U>(p, r, 1, end, xl, 0, lane);
    // the caller's draw of the next tile ends with barriers: every wave is
    // done with xl before the next tile rewrites it
}

// Rows [begin, begin + len) of a gemv problem with row heads (vec == 2): the
// work-group writes the E shifted copies of x into `xl` (copy h at h *
// stride holds x[j + h] for j < n - h), then each wavefront takes pairs of
// rows E apart, which start at the same offset inside a vector: pair q is
// rows begin + 2E (q / E) + q % E and E rows further, wavefront w taking
// pairs w, w + W, ....  All threads of the work-group must call this (it
// has barriers).
template <class T, int ACC, int VB, int U>
__device__ __forceinline__ void gemv_tile_skew(const BatchProblem &p, const BatchTile &tl, float *xl)
{
    constexpr int E = Elems<T, VB>::value;
    const int64_t stride = (p.n + 3) & ~(int64_t)3;   // E * stride <= BATCH_LDS_X (planner)
    stage_x<E>(reinterpret_cast<const float *>(p.b), p.n, xl, stride);   // n >= 64 E (planner)
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t waves = blockDim.x >> 6;
    const int64_t end = tl.begin + tl.len;
    const int64_t pairs = (tl.len + 2 * E - 1) / (2 * E) * E;
    for (int64_t q = threadIdx.x >> 6; q < pairs; q += waves) {
        const int64_t r0 = tl.begin + 2 * E * (q / E) + q % E;
        if (r0 < end)   // wave-uniform
            gemv_rows_phase<T, ACC, VB, 2, U>(p, r0, E, end, xl, stride, lane);
    }
    // the caller's draw of the next tile ends with barriers (as gemv_tile_lx)
}

// Stamped instances: thread 0 records when its work-group takes a tile and
// what the tile is, then (after a barrier, every wave done) when it is done.
template <bool STAMP>
__device__ __forceinline__ void stamp_tile_start(const BatchArgs &a, int ti, const BatchTile &tl)
{
    if constexpr (STAMP) {
        if (threadIdx.x == 0) {
            const uint32_t xcc = __builtin_amdgcn_s_getreg((20 << 0) | (0 << 6) | (3 << 11));  // XCC_ID[3:0]
            const uint32_t hw = __builtin_amdgcn_s_getreg((4 << 0) | (8 << 6) | (7 << 11));    // HW_ID[15:8]
            uint64_t *w = a.stamps + (int64_t)ti * STAMPS_PER_TILE;
            w[0] = (uint64_t)wall_clock64();
            w[2] = ((uint64_t)(uint32_t)tl.problem << 32) | (uint32_t)tl.len;
            w[3] = ((uint64_t)((xcc << 16) | hw) << 32) | (uint32_t)blockIdx.x;
        }
    }
}

template <bool STAMP>
__device__ __forceinline__ void stamp_tile_end(const BatchArgs &a, int ti)
{
    if constexpr (STAMP) {
        __syncthreads();
        if (threadIdx.x == 0)
            a.stamps[(int64_t)ti * STAMPS_PER_TILE + 1] = (uint64_t)wall_clock64();
    }
}

// Next tile for the work-group: thread 0 draws it from the shared counter
// (offset by the grid size: work-group b's first tile is b, taken without
// an atomic, so the launch does not start with every work-group contending
// for one address); everyone reads it after a barrier.  Wave-uniform result.
__device__ __forceinline__ int fetch_tile(unsigned *counter, int *s_tile)
{
    if (threadIdx.x == 0)
        *s_tile = (int)gridDim.x +
                  (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int ti = __builtin_amdgcn_readfirstlane(*s_tile);
    __syncthreads();  // every wave has read s_tile before thread 0 may write it again
    return ti;
}

// At most 512 threads per work-group: the widest instance (dot, 16-byte
// loads, 8 in flight) needs about 160 VGPRs, more than a 1024-thread
// work-group leaves each wave.
// The loop is written so that its only back edge passes through the tile's
// draw of the next one (thread 0's atomic, then a barrier every thread
// reaches): no continue / break, and every branch inside it is on a
// work-group-uniform scalar.  (A loop whose head is thread 0's conditional
// fetch, re-entered from several places, can be restructured by the
// compiler into a back edge that reaches the barrier without the fetch,
// splitting wave 0 around it.)
template <class T, int ACC, int VB, int U, bool STAMP = false>
__global__ void __launch_bounds__(512) batch_kernel(BatchArgs a)
{
    using BT = typename BlockT<ACC>::type;
    using ST = typename SlotT<ACC>::type;
    constexpr int EB = T::bytes;  // element-wise loads for unaligned problems
    __shared__ BT lds_block[16];
    __shared__ ST lds_final[16];
    __shared__ int s_tile;
    __shared__ int s_last;
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;

    int ti = blockIdx.x;  // the grid never exceeds the tile count
    while (ti < a.ntiles) {
        const BatchTile tl = a.tiles[ti];
        stamp_tile_start<STAMP>(a, ti, tl);
        const BatchProblem p = a.probs[tl.problem];
        const int kind = __builtin_amdgcn_readfirstlane(p.kind);
        int next;
        const int vec = __builtin_amdgcn_readfirstlane(p.vec);

        {
            BT v;
            if (kind == KIND_ASUM)
                v = vec ? tile_lane_value<T, OP_ASUM, ACC, VB, U>(p, tl) : tile_lane_value<T, OP_ASUM, ACC, EB, U>(p, tl);
            else
                v = vec ? tile_lane_value<T, OP_DOT, ACC, VB, U>(p, tl) : tile_lane_value<T, OP_DOT, ACC, EB, U>(p, tl);
            const BT wg = block_sum<BT>(v, lds_block);

            if (t == 0) {
                unsigned ticket;
                if (p.ntiles == 1) {
                    // a problem of one tile: the combine of a single partial
                    // returns it unchanged (it adds zeros to a sum that is
                    // never -0), so the partial is the result, written
                    // without the slot, the count and the combine
                    write_result(p.out, a.result_f64, to_slot<ACC>(wg));
                    ticket = __hip_atomic_fetch_add(&a.counters[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_last = 0;
                } else {
                    store_coherent(a.slots + (p.slot_base + tl.index) * WS_SLOT, to_slot<ACC>(wg));
                    // the next tile is drawn here, its round trip overlapping the
                    // partial's store (the work-group is all but done with this one)
                    ticket = __hip_atomic_fetch_add(&a.counters[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    __builtin_amdgcn_s_waitcnt(0);  // the partial's store has completed
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    unsigned prev = __hip_atomic_fetch_add(&a.pcount[tl.problem], 1u, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                    s_last = prev == (unsigned)(p.ntiles - 1);
                }
                s_tile = (int)gridDim.x + (int)ticket;
            }
            __syncthreads();
            const int last = __builtin_amdgcn_readfirstlane(s_last);
            next = __builtin_amdgcn_readfirstlane(s_tile);
            if (last) {
                ST acc = zero_of<ST>();
                for (int64_t i = t; i < p.ntiles; i += B)
                    acc = merge(acc, load_coherent<ST>(a.slots + (p.slot_base + i) * WS_SLOT));
                acc = block_sum<ST>(acc, lds_final);
                if (t == 0) {
                    write_result(p.out, a.result_f64, acc);
                    __hip_atomic_store(&a.pcount[tl.problem], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        stamp_tile_end<STAMP>(a, ti);
        // thread 0 writes s_tile and s_last again only after the next tile's
        // tree, whose barrier every thread reaches after reading them here
        ti = next;
    }

    // The last work-group out (two-level arrival) resets the counters for the
    // next launch; by then no work-group will read the tile counter again.
    if (t == 0 && arrive(&a.counters[1], a.groups)) {
        __hip_atomic_store(&a.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The gemv tiles of a batch: wavefronts take row pairs of each tile, reading
// x from a copy in LDS where it fits (up to BATCH_LDS_X columns), else from
// the cache; rows with heads (vec == 2, vectors of at most 8 bytes) go one
// per wavefront against shifted copies of x.  Same loop discipline as
// batch_kernel.
template <class T, int ACC, int VB, int U, bool STAMP = false>
__global__ void __launch_bounds__(512) batch_gemv_kernel(BatchArgs a)
{
    constexpr int EB = T::bytes;  // element-wise loads for unaligned problems
    __shared__ int s_tile;
    __shared__ __align__(16) float lds_x[BATCH_LDS_X];
    const int t = threadIdx.x;

    int ti = blockIdx.x;  // the grid never exceeds the tile count
    while (ti < a.ntiles) {
        const BatchTile tl = a.tiles[ti];
        stamp_tile_start<STAMP>(a, ti, tl);
        const BatchProblem p = a.probs[tl.problem];
        const int vec = __builtin_amdgcn_readfirstlane(p.vec);
        const int in_lds = __builtin_amdgcn_readfirstlane((int)(p.n <= BATCH_LDS_X));
        if (vec == 2) {
            if constexpr (VB <= 8)   // the planner sets vec 2 only for these widths
                gemv_tile_skew<T, ACC, VB, U>(p, tl, lds_x);
        } else if (in_lds) {
            if (vec)
                gemv_tile_lx<T, ACC, VB, U>(p, tl, lds_x);
            else
                gemv_tile_lx<T, ACC, EB, U>(p, tl, lds_x);
        } else {
            if (vec)
                gemv_tile<T, ACC, VB, U>(p, tl);
            else
                gemv_tile<T, ACC, EB, U>(p, tl);
        }
        stamp_tile_end<STAMP>(a, ti);
        ti = fetch_tile(&a.counters[0], &s_tile);
    }
    if (t == 0 && arrive(&a.counters[1], a.groups)) {
        __hip_atomic_store(&a.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&a.counters[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Kernel tables: `gemv` picks the gemv-tile kernel, else the reduction one.
template <class T, int ACC, int VB>
const void *batch_pick_unroll(int unroll, bool gemv)
{
    switch (unroll) {
    case 1: return gemv ? reinterpret_cast<const void *>(&batch_gemv_kernel<T, ACC, VB, 1>)
                        : reinterpret_cast<const void *>(&batch_kernel<T, ACC, VB, 1>);
    case 2: return gemv ? reinterpret_cast<const void *>(&batch_gemv_kernel<T, ACC, VB, 2>)
                        : reinterpret_cast<const void *>(&batch_kernel<T, ACC, VB, 2>);
    case 4: return gemv ? reinterpret_cast<const void *>(&batch_gemv_kernel<T, ACC, VB, 4>)
                        : reinterpret_cast<const void *>(&batch_kernel<T, ACC, VB, 4>);
    case 8: return gemv ? reinterpret_cast<const void *>(&batch_gemv_kernel<T, ACC, VB, 8>)
                        : reinterpret_cast<const void *>(&batch_kernel<T, ACC, VB, 8>);
    default: return nullptr;
    }
}

template <class T, int ACC>
const void *batch_pick_vec(int vec_bytes, int unroll, bool gemv)
{
    switch (vec_bytes) {
    case 4: return batch_pick_unroll<T, ACC, 4>(unroll, gemv);
    case 8: return batch_pick_unroll<T, ACC, 8>(unroll, gemv);
    case 16: return batch_pick_unroll<T, ACC, 16>(unroll, gemv);
    default: return nullptr;
    }
}

template <class T>
const void *pick_batch(int acc, int vec_bytes, int unroll, bool gemv)
{
    switch (acc) {
    case ACC_F32: return batch_pick_vec<T, ACC_F32>(vec_bytes, unroll, gemv);
    case ACC_COMP: return batch_pick_vec<T, ACC_COMP>(vec_bytes, unroll, gemv);
    case ACC_F64: return batch_pick_vec<T, ACC_F64>(vec_bytes, unroll, gemv);
    default: return nullptr;
    }
}

// The stamped instances (binary32 accumulation) of both kernels.
template <class T, int VB, int U>
const void *pick_batch_stamped_kind(bool gemv)
{
    return gemv ? reinterpret_cast<const void *>(&batch_gemv_kernel<T, ACC_F32, VB, U, true>)
                : reinterpret_cast<const void *>(&batch_kernel<T, ACC_F32, VB, U, true>);
}

template <class T, int VB>
const void *pick_batch_stamped_unroll(int unroll, bool gemv)
{
    switch (unroll) {
    case 1: return pick_batch_stamped_kind<T, VB, 1>(gemv);
    case 2: return pick_batch_stamped_kind<T, VB, 2>(gemv);
    case 4: return pick_batch_stamped_kind<T, VB, 4>(gemv);
    case 8: return pick_batch_stamped_kind<T, VB, 8>(gemv);
    default: return nullptr;
    }
}

template <class T>
const void *pick_batch_stamped(int vec_bytes, int unroll, bool gemv)
{
    switch (vec_bytes) {
    case 4: return pick_batch_stamped_unroll<T, 4>(unroll, gemv);
    case 8: return pick_batch_stamped_unroll<T, 8>(unroll, gemv);
    case 16: return pick_batch_stamped_unroll<T, 16>(unroll, gemv);
    default: return nullptr;
    }
}

}  // namespace lift
