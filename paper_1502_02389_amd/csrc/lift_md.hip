// MD: the force on every particle from its neighbour list (Fig. 7):
//   md(ps, N, t) = map(lambda (p, ns): reduce(lambda (f, nId):
//                      updateF(f, nId, p, ps, t), 0, ns)) . zip(ps, N)
// with updateF adding the Lennard-Jones pair force of ps[nId] on p when
// their distance is below the cutoff t.
//
// The map over particles becomes groups of L lanes per particle (L = 1..16,
// 64 / L particles per wavefront); the reduce over the neighbour list is
// split over the group's lanes (split + partial reduce-seq per lane, then a
// DPP butterfly inside the group), which keeps thousands of wavefronts busy
// for the paper's 12288 particles.  Lane `sub` of a group reads index vectors
// sub, sub + L, ... of its particle's row (V indices per load, so L * V * 4
// contiguous bytes per group and step), keeps U index loads in flight, then
// gathers the U * V neighbour positions (16 bytes each; the position array
// is small and stays in cache) before any arithmetic.  Empty slots (indices
// outside [0, n)) load nothing and contribute zero.
//
// Per neighbour, in binary32: d = p - q, r2 = (dx dx + dy dy) + dz dz
// without contraction, and the cutoff test r2 < binary32(t^2).  That r2 is
// within about 5 ulps of the exact squared distance, so the test agrees
// with "distance < t" except for pairs whose squared distance lies within
// about 6 binary32 ulps of t^2; it is the same decision on every run and
// knob point.  Then 1/r2 by the hardware reciprocal, s6 = (sigma^2 / r2)^3,
// f = 24 eps / r2 * s6 * (2 s6 - 1) (zero outside the cutoff) and F += f d
// by fma.
#include "lift_device.hpp"
#include "lift_apps.hpp"
#include "lift_internal.hpp"

namespace lift {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

template <int V> struct IdxVec;
template <> struct IdxVec<1> { using type = int32_t; };
template <> struct IdxVec<2> { using type = i32x2; };
template <> struct IdxVec<4> { using type = i32x4; };

template <int V>
__device__ __forceinline__ int32_t lane_of(typename IdxVec<V>::type v, int e)
{
    if constexpr (V == 1)
        return v;
    else
        return v[e];
}

// Sum over the L lanes of an aligned group (the DPP steps of the wave
// butterfly that stay inside the group); every lane of the group gets it.
template <int L>
__device__ __forceinline__ float group_sum(float v)
{
    if constexpr (L >= 2)
        v += dpp<DPP_QUAD_XOR1>(v);
    if constexpr (L >= 4)
        v += dpp<DPP_QUAD_XOR2>(v);
    if constexpr (L >= 8)
        v += dpp<DPP_HALF_MIRROR>(v);
    if constexpr (L >= 16)
        v += dpp<DPP_ROW_MIRROR>(v);
    return v;
}

template <int L, int V, int U>
__global__ void __launch_bounds__(1024) md_kernel(MdArgs a)
{
    using IV = typename IdxVec<V>::type;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gt / L;  // particle
    const int sub = (int)(gt % L);
    if (i >= a.n)  // whole groups leave together (L divides 64)
        return;
    const f32x4 *pos = reinterpret_cast<const f32x4 *>(a.pos);
    const f32x4 p = pos[i];
    const IV *row = reinterpret_cast<const IV *>(a.nbr + i * a.k);
    const int64_t kv = a.k / V;  // index vectors per row
    const uint32_t n = (uint32_t)a.n;

    float fx = 0.f, fy = 0.f, fz = 0.f;
    for (int64_t base = 0; base < kv; base += L * U) {
        IV iv[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            iv[u] = __builtin_nontemporal_load(row + min(base + sub + (int64_t)L * u, kv - 1));
        loads_in_flight();
        f32x4 q[U][V];
        bool use[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in_row = base + sub + (int64_t)L * u < kv;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const int32_t id = lane_of<V>(iv[u], e);
                use[u][e] = in_row && (uint32_t)id < n;
                q[u][e] = p;  // empty slots load nothing
                if (use[u][e])
                    q[u][e] = pos[id];
            }
        }
        loads_in_flight();
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const float dx = p[0] - q[u][e][0], dy = p[1] - q[u][e][1], dz = p[2] - q[u][e][2];
                const float r2 = (dx * dx + dy * dy) + dz * dz;
                const float r2inv = __builtin_amdgcn_rcpf(r2);
                const float s2 = a.sigma2 * r2inv;
                const float s6 = s2 * s2 * s2;
                const float fs = a.eps24 * r2inv * s6 * (2.f * s6 - 1.f);
                const float fh = use[u][e] && r2 < a.t2 ? fs : 0.f;
                fx = fmaf(fh, dx, fx);
                fy = fmaf(fh, dy, fy);
                fz = fmaf(fh, dz, fz);
            }
    }
    fx = group_sum<L>(fx);
    fy = group_sum<L>(fy);
    fz = group_sum<L>(fz);
    if (sub == 0) {
        f32x4 f = {fx, fy, fz, 0.f};
        reinterpret_cast<f32x4 *>(a.force)[i] = f;
    }
}

template <int L, int V>
static const void *md_pick_unroll(int unroll)
{
    switch (unroll) {
    case 1: return reinterpret_cast<const void *>(&md_kernel<L, V, 1>);
    case 2: return reinterpret_cast<const void *>(&md_kernel<L, V, 2>);
    case 4: return reinterpret_cast<const void *>(&md_kernel<L, V, 4>);
    default: return nullptr;
    }
}

template <int L>
static const void *md_pick_vec(int v, int unroll)
{
    switch (v) {
    case 1: return md_pick_unroll<L, 1>(unroll);
    case 2: return md_pick_unroll<L, 2>(unroll);
    case 4: return md_pick_unroll<L, 4>(unroll);
    default: return nullptr;
    }
}

const void *md_kernel_table(int lanes, int v, int unroll)
{
    switch (lanes) {
    case 1: return md_pick_vec<1>(v, unroll);
    case 2: return md_pick_vec<2>(v, unroll);
    case 4: return md_pick_vec<4>(v, unroll);
    case 8: return md_pick_vec<8>(v, unroll);
    case 16: return md_pick_vec<16>(v, unroll);
    default: return nullptr;
    }
}

}  // namespace lift
