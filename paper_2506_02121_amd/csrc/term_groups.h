// Device helpers shared by the root finder and the lens map: reciprocals
// refined by Newton-Raphson steps, reciprocals shared by groups of terms
// through a product tree, and star tiles streamed through LDS in such groups.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mlcc {

// Reciprocal of a double: the hardware estimate refined by Newton-Raphson
// steps y <- y + y (1 - x y), each of which squares the relative error.
template <int STEPS>
__device__ __forceinline__ double rcp_refined(double x)
{
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
        double e = fma(-x, y, 1.0);
        y = fma(y, e, y);
    }
    return y;
}

// G reciprocals for the price of one: with r the refined reciprocal of the
// product of q[0..G), the reciprocals of the two halves' products are
// 1/P_lo = P_hi r and 1/P_hi = P_lo r, and so on down to single terms
// (1/a = b/(ab)).  For eight terms and one refinement step: 23 FP64
// operations and one quarter-rate v_rcp_f64, against 22 and two for two
// groups of four.  The relative error is the refined reciprocal's (~2^-47
// after one Newton step, about an ulp after two) plus a rounding per level of
// the tree.  The product of eight squared distances stays inside the double
// range for distances between 1e-19 and 1e19.  A zero distance makes every
// term of its group non-finite, as it makes its own term non-finite alone.
template <int G> struct RcpTree {
    static __device__ __forceinline__ double prod(const double *q)
    {
        return RcpTree<G / 2>::prod(q) * RcpTree<G / 2>::prod(q + G / 2);
    }
    static __device__ __forceinline__ void down(const double *q, double r, double *iq)
    {
        const double lo = RcpTree<G / 2>::prod(q), hi = RcpTree<G / 2>::prod(q + G / 2);
        RcpTree<G / 2>::down(q, hi * r, iq);
        RcpTree<G / 2>::down(q + G / 2, lo * r, iq + G / 2);
    }
};
template <> struct RcpTree<1> {
    static __device__ __forceinline__ double prod(const double *q) { return q[0]; }
    static __device__ __forceinline__ void down(const double *, double r, double *iq) { iq[0] = r; }
};

template <int G, int STEPS>
__device__ __forceinline__ void rcp_group(const double (&q)[G], double (&iq)[G])
{
    RcpTree<G>::down(q, rcp_refined<STEPS>(RcpTree<G>::prod(q)), iq);
}

// Reciprocals are shared by groups of this many consecutive terms (1, 2, 4
// or 8; see RcpTree).
#ifndef MLCC_RCP_GROUP
#define MLCC_RCP_GROUP 8
#endif

template <int G> using GroupOf = std::integral_constant<int, G>;

// Streams the records p[0..n) for a one-wave work group: tiles of 64 records
// (one per lane) fetched with coalesced vector loads, the next tile while the
// current one is consumed, parked in LDS and read back as wave-uniform
// broadcasts.  The records go to group(GroupOf<G>{}, r) with r pointing at G
// consecutive records in LDS: G = MLCC_RCP_GROUP in full tiles, and a partial
// tile ends with groups of half, a quarter ... of that, so the terms meet the
// sums in record order.  Indices past n-1 are clamped on load; `lds` holds
// two tiles.
template <class T, class Group>
__device__ __forceinline__ void stream_tiles_grouped(const T *__restrict__ p, int n, T *lds,
                                                     Group &&group)
{
    constexpr int G = MLCC_RCP_GROUP;
    static_assert(G == 1 || G == 2 || G == 4 || G == 8, "group of 1, 2, 4 or 8 terms");
    if (n <= 0) return;
    const int lane = threadIdx.x;
    const int ntiles = (n + 63) >> 6;
    T reg = p[min(lane, n - 1)];
    for (int t = 0; t < ntiles; ++t) {
        T *buf = lds + ((t & 1) << 6);
        buf[lane] = reg;
        __syncthreads();
        if (t + 1 < ntiles) reg = p[min(((t + 1) << 6) + lane, n - 1)];
        const int cnt = min(64, n - (t << 6));
        if (cnt == 64) {
#pragma unroll G >= 8 ? 1 : 8 / G
            for (int k = 0; k < 64; k += G) group(GroupOf<G>{}, buf + k);
        } else {
            int k = 0;
            for (; k + G <= cnt; k += G) group(GroupOf<G>{}, buf + k);
            if constexpr (G > 4) {
                if (k + 4 <= cnt) {
                    group(GroupOf<4>{}, buf + k);
                    k += 4;
                }
            }
            if constexpr (G > 2) {
                if (k + 2 <= cnt) {
                    group(GroupOf<2>{}, buf + k);
                    k += 2;
                }
            }
            if constexpr (G > 1) {
                if (k < cnt) group(GroupOf<1>{}, buf + k);
            }
        }
    }
    __syncthreads();
}

} // namespace mlcc
