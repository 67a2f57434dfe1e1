// BlackScholes: map(BSComputation) over stock prices (Section 5.2).
//
// BSComputation(s) computes d1 and d2 from the price and returns the pair
// {call, put} of the closed-form model for a European option; strike K,
// rate r, volatility v and expiry T are the same for every element:
//   d1 = (ln(s/K) + (r + v^2/2) T) / (v sqrt T),  d2 = d1 - v sqrt T,
//   call = s N(d1) - K e^{-rT} N(d2),  put = K e^{-rT} N(-d2) - s N(-d1).
// The per-call constants are formed in binary64 on the host and rounded
// once, so d1 = log2(s) ln2/(v sqrt T) + (((r + v^2/2) T - ln K)/(v sqrt T))
// is one hardware log2 and one fma.  N is evaluated through the upper tail
// Q(z) = N(-z), z = |d| >= 0, as the density times a polynomial for the
// Mills ratio (below); the other side is 1 - Q (>= 1/2, so exact enough in
// absolute terms).  About 40 instructions per price instead of ~140 with
// the library's logf / erfcf, which leaves the kernel bound by HBM.
//
// Lowered like scal: join o map-workgroup(asScalar o map-local(vect(BS))
// o asVector) o split^chunk, VB-byte vectors of prices (E = VB / 4 per lane),
// U loads in flight, each lane storing its E pairs (2 VB bytes) right after
// the computation; a scalar head and tail cover any 4-byte-aligned input.
#include "lift_device.hpp"
#include "lift_apps.hpp"
#include "lift_internal.hpp"

namespace lift {

// Q(z) = phi(z) R(z): R(z) ~ sum_{k=1..7} c_k t^k, t = 1 / (1 + p z), fitted
// by least squares weighted by phi on [0, 12] (fit_normal_tail.py).  In exact
// arithmetic with these binary32 constants |Q error| < 2e-8 on [0, 40];
// evaluated in binary32 it stays within ~2e-7.
// worst |Q error| on [0, 40] of the fit: 7.288e-10
constexpr float TAIL_P = 0.315f;
constexpr float TAIL_C[7] = {3.227985905e-01f, 2.368258597e-01f, 6.157643717e-01f, -5.441662870e-01f,
                             1.140571062e+00f, -6.340257905e-01f, 1.155463295e-01f};
constexpr float INV_SQRT_2PI = 0.398942280401432678f;
constexpr float NEG_HALF_LOG2E = -0.721347520444481703f;  // -log2(e) / 2

__device__ __forceinline__ float normal_tail(float z)
{
    const float t = __builtin_amdgcn_rcpf(fmaf(TAIL_P, z, 1.f));
    float r = TAIL_C[6];
#pragma unroll
    for (int k = 5; k >= 0; --k)
        r = fmaf(r, t, TAIL_C[k]);
    r *= t;
    const float e = __builtin_amdgcn_exp2f(z * z * NEG_HALF_LOG2E);  // exp(-z^2 / 2)
    return (INV_SQRT_2PI * e) * r;
}

struct BsPair {
    float call, put;
};

__device__ __forceinline__ BsPair bs_computation(float s, const BsArgs &a)
{
    const float d1 = fmaf(__builtin_amdgcn_logf(s), a.ln2_over_vst, a.d1_offset);  // compD1
    const float d2 = d1 - a.vol_sqrt_t;                                             // compD2
    const float q1 = normal_tail(fabsf(d1));  // N(-|d1|)
    const float q2 = normal_tail(fabsf(d2));
    const float n1 = d1 >= 0.f ? 1.f - q1 : q1;  // N(d1)
    const float m1 = d1 >= 0.f ? q1 : 1.f - q1;  // N(-d1)
    const float n2 = d2 >= 0.f ? 1.f - q2 : q2;
    const float m2 = d2 >= 0.f ? q2 : 1.f - q2;
    BsPair r;
    r.call = s * n1 - a.strike_disc * n2;  // compCall
    r.put = a.strike_disc * m2 - s * m1;   // compPut
    return r;
}

__device__ __forceinline__ void bs_scalar(const BsArgs &a, int64_t j)
{
    const BsPair p = bs_computation(a.s[j], a);
    a.call_put[2 * j] = p.call;
    a.call_put[2 * j + 1] = p.put;
}

template <int VB>
__device__ __forceinline__ void bs_vector(typename Vec<VB>::type v, char *out, int64_t i, const BsArgs &a)
{
    constexpr int E = VB / 4;
    float s[E];
    if constexpr (E == 1) {
        s[0] = bits_to_float(v);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
            s[e] = bits_to_float(v[e]);
    }
    uint32_t w[2 * E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const BsPair p = bs_computation(s[e], a);
        w[2 * e] = __builtin_bit_cast(uint32_t, p.call);
        w[2 * e + 1] = __builtin_bit_cast(uint32_t, p.put);
    }
    // E pairs = 2 VB bytes: one 8- or 16-byte store, or two 16-byte stores
    if constexpr (E == 1) {
        store_stream<8>(out, i, u32x2{w[0], w[1]});
    } else if constexpr (E == 2) {
        store_stream<16>(out, i, u32x4{w[0], w[1], w[2], w[3]});
    } else {
        store_stream<16>(out, 2 * i, u32x4{w[0], w[1], w[2], w[3]});
        store_stream<16>(out, 2 * i + 1, u32x4{w[4], w[5], w[6], w[7]});
    }
}

template <int VB, int U>
__global__ void __launch_bounds__(1024) blackscholes_kernel(BsArgs a)
{
    using V = typename Vec<VB>::type;
    const int t = threadIdx.x;
    const int64_t B = blockDim.x;
    const char *sv = reinterpret_cast<const char *>(a.s) + a.head * 4;
    char *ov = reinterpret_cast<char *>(a.call_put) + a.head * 8;

    const int64_t vbeg = (int64_t)blockIdx.x * a.chunk;
    const int64_t vend = min(vbeg + a.chunk, a.nvec);
    const int64_t step = B * U;
    int64_t base = vbeg;
    for (; base + step <= vend; base += step) {
        V v[U];
#pragma unroll
        for (int k = 0; k < U; ++k)
            v[k] = load_stream<VB>(sv, base + t + k * B);
        loads_in_flight();
#pragma unroll
        for (int k = 0; k < U; ++k)
            bs_vector<VB>(v[k], ov, base + t + k * B, a);
    }
    for (int64_t i = base + t; i < vend; i += B)
        bs_vector<VB>(load_stream<VB>(sv, i), ov, i, a);

    // scalar head (work-group 0) and tail (last work-group; with one
    // work-group the same thread may own a head and a tail element)
    constexpr int E = VB / 4;
    const int64_t tail0 = a.head + a.nvec * E;
    if (blockIdx.x == 0 && t < a.head)
        bs_scalar(a, t);
    if (blockIdx.x == gridDim.x - 1 && t < a.n - tail0)
        bs_scalar(a, tail0 + t);
}

template <int VB>
static const void *bs_pick_unroll(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&blackscholes_kernel<VB, 1>);
    case 2: return reinterpret_cast<const void *>(&blackscholes_kernel<VB, 2>);
    case 4: return reinterpret_cast<const void *>(&blackscholes_kernel<VB, 4>);
    case 8: return reinterpret_cast<const void *>(&blackscholes_kernel<VB, 8>);
    default: return nullptr;
    }
}

const void *blackscholes_kernel_table(int vec_bytes, int unroll)
{
    switch (vec_bytes) {
    case 4: return bs_pick_unroll<4>(unroll);
    case 8: return bs_pick_unroll<8>(unroll);
    case 16: return bs_pick_unroll<16>(unroll);
    default: return nullptr;
    }
}

}  // namespace lift
