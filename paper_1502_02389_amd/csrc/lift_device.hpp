// Device-side building blocks shared by the gfx950 kernels.
//
// The paper's low-level patterns (Table 2) map onto CDNA4 as follows:
//   asVector^n / vect^n   -> one global_load_dwordx{1,2,4} per lane (Vec<VB>)
//   reorder-stride^s      -> lane t of a work-group reads vector t, t+B, ...
//   reduce-seq            -> a per-lane accumulator (Lane<...>)
//   iterate^k(part-red) + toLocal
//                         -> wave64 DPP butterfly, then one LDS slot per wave
//   toGlobal + final reduce-seq o join
//                         -> one partial per work-group in the workspace,
//                            summed in index order by the last work-group
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lift {

// ---------------------------------------------------------------- storage

struct F32 { using raw = uint32_t; static constexpr int bytes = 4; };
struct BF16 { using raw = uint16_t; static constexpr int bytes = 2; };
struct F16 { using raw = uint16_t; static constexpr int bytes = 2; };

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// VB bytes loaded by one lane in one instruction.
template <int VB> struct Vec;
template <> struct Vec<2> { using type = uint16_t; };
template <> struct Vec<4> { using type = uint32_t; };
template <> struct Vec<8> { using type = u32x2; };
template <> struct Vec<16> { using type = u32x4; };

template <int VB>
__device__ __forceinline__ typename Vec<VB>::type load_vec(const void *base, int64_t i)
{
    return reinterpret_cast<const typename Vec<VB>::type *>(base)[i];
}

// Streaming load of data read exactly once: the nontemporal hint keeps it
// from displacing reused lines and measurably raises sustained HBM read
// bandwidth on gfx950.
template <int VB>
__device__ __forceinline__ typename Vec<VB>::type load_stream(const void *base, int64_t i)
{
    return __builtin_nontemporal_load(reinterpret_cast<const typename Vec<VB>::type *>(base) + i);
}

// Scheduling fence after a group of independent loads: keeps the compiler
// from sinking each load next to its first use (which would leave one load
// in flight per wave and make the stream latency-bound).
__device__ __forceinline__ void loads_in_flight() { __builtin_amdgcn_sched_barrier(0); }

template <int VB>
__device__ __forceinline__ void store_stream(void *base, int64_t i, typename Vec<VB>::type v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<typename Vec<VB>::type *>(base) + i);
}

__device__ __forceinline__ float bits_to_float(uint32_t b) { return __builtin_bit_cast(float, b); }

// Exact decode of one 32-bit word holding two 16-bit values (lower address
// in the low half), or one binary32.
template <class T> struct Decode;
template <> struct Decode<F32> {
    static constexpr int per_word = 1;
    __device__ __forceinline__ static void word(uint32_t w, float *o) { o[0] = bits_to_float(w); }
    __device__ __forceinline__ static float half(uint16_t) { return 0.f; }
};
template <> struct Decode<BF16> {
    static constexpr int per_word = 2;
    // bfloat16 is the upper half of a binary32: shifting it into place is exact.
    __device__ __forceinline__ static void word(uint32_t w, float *o)
    {
        o[0] = bits_to_float(w << 16);
        o[1] = bits_to_float(w & 0xffff0000u);
    }
    __device__ __forceinline__ static float half(uint16_t h) { return bits_to_float((uint32_t)h << 16); }
};
template <> struct Decode<F16> {
    static constexpr int per_word = 2;
    // binary16 -> binary32 (v_cvt_f32_f16) is exact.
    __device__ __forceinline__ static void word(uint32_t w, float *o)
    {
        o[0] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
        o[1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
    }
    __device__ __forceinline__ static float half(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }
};

// Number of elements of storage T in VB bytes.
template <class T, int VB> struct Elems { static constexpr int value = VB / T::bytes; };

// Decode a VB-byte load of storage T into E = VB / sizeof(T) binary32 values.
template <class T, int VB>
__device__ __forceinline__ void decode(const typename Vec<VB>::type &v, float *o)
{
    if constexpr (VB == 2) {
        o[0] = Decode<T>::half(v);
    } else if constexpr (VB == 4) {
        Decode<T>::word(v, o);
    } else {
        constexpr int words = VB / 4;
#pragma unroll
        for (int w = 0; w < words; ++w)
            Decode<T>::word(v[w], o + w * Decode<T>::per_word);
    }
}

// One stored element of storage T (its raw bits), decoded.
template <class T>
__device__ __forceinline__ float decode_raw(typename T::raw v)
{
    if constexpr (T::bytes == 4)
        return bits_to_float(v);
    else
        return Decode<T>::half(v);
}

// Scalar element i of storage T, decoded.
template <class T>
__device__ __forceinline__ float load_elem(const void *base, int64_t i)
{
    return decode_raw<T>(reinterpret_cast<const typename T::raw *>(base)[i]);
}

// ---------------------------------------------------------------- error-free sums

// (s, c): value s + c with s the rounded sum and c an accumulated error term.
struct Pair {
    float s, c;
};

// TwoSum (Knuth): s = fl(a + b), e = (a + b) - s exactly, for any a, b.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ Pair pair_add(Pair p, float v)
{
    float s, e;
    two_sum(p.s, v, s, e);
    return {s, p.c + e};
}

// Symmetric merge: pair_merge(p, q) == pair_merge(q, p) bitwise.
__device__ __forceinline__ Pair pair_merge(Pair p, Pair q)
{
    float s, e;
    two_sum(p.s, q.s, s, e);
    return {s, (p.c + q.c) + e};
}

// ---------------------------------------------------------------- wave64 reduction

template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float readlane(float v, int lane)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// DPP controls of the butterfly inside each 16-lane row: swap neighbours,
// swap pairs (quad_perm), mirror each half-row, mirror the row.  Every step
// pairs a lane with one holding a disjoint partial sum, so after four steps
// every lane of a row holds the row total (a + b == b + a bitwise, so all
// lanes agree exactly).
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_ROW_MIRROR = 0x140;

// Sum over the 64 lanes; the result is wave-uniform.
__device__ __forceinline__ float wave_sum(float v)
{
    v += dpp<DPP_QUAD_XOR1>(v);
    v += dpp<DPP_QUAD_XOR2>(v);
    v += dpp<DPP_HALF_MIRROR>(v);
    v += dpp<DPP_ROW_MIRROR>(v);
    return (readlane(v, 0) + readlane(v, 16)) + (readlane(v, 32) + readlane(v, 48));
}

template <int CTRL>
__device__ __forceinline__ Pair dpp_pair(Pair p)
{
    return {dpp<CTRL>(p.s), dpp<CTRL>(p.c)};
}

__device__ __forceinline__ Pair wave_sum(Pair p)
{
    p = pair_merge(p, dpp_pair<DPP_QUAD_XOR1>(p));
    p = pair_merge(p, dpp_pair<DPP_QUAD_XOR2>(p));
    p = pair_merge(p, dpp_pair<DPP_HALF_MIRROR>(p));
    p = pair_merge(p, dpp_pair<DPP_ROW_MIRROR>(p));
    Pair r0{readlane(p.s, 0), readlane(p.c, 0)}, r1{readlane(p.s, 16), readlane(p.c, 16)};
    Pair r2{readlane(p.s, 32), readlane(p.c, 32)}, r3{readlane(p.s, 48), readlane(p.c, 48)};
    return pair_merge(pair_merge(r0, r1), pair_merge(r2, r3));
}

// binary64 butterfly over the wave (used only in the final combine).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1)
        v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float merge(float a, float b) { return a + b; }
__device__ __forceinline__ double merge(double a, double b) { return a + b; }
__device__ __forceinline__ Pair merge(Pair a, Pair b) { return pair_merge(a, b); }

// Work-group reduction: wave butterflies, one LDS slot per wave, then the
// wave totals folded in wave order by thread 0.  The value is valid in
// thread 0 only.  `lds` holds blockDim.x / 64 entries.  Ends with a barrier
// so `lds` can be reused.
template <class A>
__device__ __forceinline__ A block_sum(A v, A *lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    v = wave_sum(v);
    if (lane == 0)
        lds[wave] = v;
    __syncthreads();
    A r = lds[0];
    if (threadIdx.x == 0)
        for (int w = 1; w < waves; ++w)
            r = merge(r, lds[w]);
    __syncthreads();
    return r;
}

}  // namespace lift
