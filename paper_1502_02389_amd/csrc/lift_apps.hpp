// Arguments and kernel tables of the two application kernels: BlackScholes
// (a map over stock prices, Section 5.2) and MD (a map over particles of a
// reduce over neighbour indices, Fig. 7).
#pragma once

#include <stdint.h>

namespace lift {

// BlackScholes over n prices: head scalars, nvec VB-byte vectors of prices,
// then the scalar tail; the per-call constants of the model in binary32.
struct BsArgs {
    const float *s;
    float *call_put;      // 2n floats: {call, put} per price
    int64_t n;
    int64_t head;
    int64_t nvec;
    int64_t chunk;        // vectors per work-group
    float ln2_over_vst;   // ln 2 / (v sqrt T): d1 = log2(s) ln2_over_vst + d1_offset
    float d1_offset;      // ((r + v^2 / 2) T - ln K) / (v sqrt T)
    float vol_sqrt_t;     // v sqrt T
    float strike_disc;    // K exp(-r T)
};

// MD forces: n particles (4 floats each), n x k neighbour indices.
struct MdArgs {
    const float *pos;
    const int32_t *nbr;
    float *force;
    int64_t n;
    int64_t k;
    float t2;      // binary32(cutoff^2)
    float sigma2;  // sigma^2
    float eps24;   // 24 epsilon
};

const void *blackscholes_kernel_table(int vec_bytes, int unroll);
const void *md_kernel_table(int lanes, int v, int unroll);

}  // namespace lift
