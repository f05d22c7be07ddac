// Critical-curve root finder: parallel Aberth-Ehrlich sweeps (Sec. 3.2)
// over the phase grid, warm-started along phi and grown centre-out in
// subchains (Sec. 4.3), in plain FP64 or in a mixed-precision form.
//
// Layout and scheduling (gfx950):
//  * One lane per root, one 64-lane wavefront per work-group.  Each
//    work-group owns 64 consecutive roots of one "front" (a growing end of a
//    subchain).  Star positions and the other roots stream through LDS in
//    tiles and are read back as wave-uniform broadcasts.
//  * A block with only a few unconverged roots left (the last sweep of a row)
//    works on them one at a time with the whole wave.
//  * Jacobi double buffering: every kernel of a launch round reads iterate
//    `cur` and writes `nxt`; the host alternates the two.
//  * Each front carries a phase.  FP64 mode: every row is FP64 Aberth sweeps.
//    Mixed mode: cold starts are FP32 Aberth sweeps until the roots settle;
//    warm rows with a chain prediction start directly with FP64 Newton
//    polish passes (the paper's cutoffs on each Newton step, row identities
//    for the row), warm rows without one with a single FP32 sweep; a row the
//    polish does not settle gets one FP32 sweep of the whole row and the
//    polish again, then FP64 Aberth sweeps.
//  * A warm row's first pass may start each root from an extrapolation
//    along its chain instead of its previous-row value.
//  * A single-work-group control kernel after every round advances the
//    fronts (device-side; the host polls a status block one batch ahead).
//  * Converged roots are mapped to the caustic in the same kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "mlcc_internal.h"
#include "term_groups.h"

namespace mlcc {

// The hardware estimate v_rcp_f64 has relative error ~2^-24.4; one
// refinement step takes it below 2^-47, a few units in the last place of a
// double.  Star terms and root-root terms both take that step, so every sum
// of an FP64 Aberth sweep is formed at double precision (the paper's program
// is double precision throughout, Sec. 4.4).
constexpr int RCP_STAR = 1;
constexpr int RCP_ROOT = 1;

// Streams the records p[0..n) through body(i, rec) for a one-wave work
// group.  Tiles of 64 records (one per lane) are fetched with coalesced
// vector loads, the next tile while the current one is consumed, converted
// by cvt and parked in LDS, and read back with one wave-uniform (broadcast)
// LDS read per record; tile_end() runs after each tile.  Vector loads retire
// in order, so waiting for the older tile never waits for the prefetch
// behind it.  Indices past n-1 are clamped on load, so nothing outside the
// array is read.  `lds` holds two tiles.
template <class T, class L, class Cvt, class Body, class End>
__device__ __forceinline__ void stream_tiles_ex(const T *__restrict__ p, int n, L *lds, Cvt &&cvt,
                                                Body &&body, End &&tile_end)
{
    if (n <= 0) return;
    const int lane = threadIdx.x;
    const int ntiles = (n + 63) >> 6;
    T reg = p[min(lane, n - 1)];
    for (int t = 0; t < ntiles; ++t) {
        L *buf = lds + ((t & 1) << 6);
        buf[lane] = cvt(reg);
        __syncthreads();
        if (t + 1 < ntiles) reg = p[min(((t + 1) << 6) + lane, n - 1)];
        const int base = t << 6;
        const int cnt = min(64, n - base);
        if (cnt == 64) {
#pragma unroll 8
            for (int k = 0; k < 64; ++k) body(base + k, buf[k]);
        } else {
            for (int k = 0; k < cnt; ++k) body(base + k, buf[k]);
        }
        tile_end();
    }
    __syncthreads();
}

struct Same {
    template <class T> __device__ __forceinline__ T operator()(const T &v) const { return v; }
};
struct NoEnd {
    __device__ __forceinline__ void operator()() const {}
};

template <class T, class Body>
__device__ __forceinline__ void stream_tiles(const T *__restrict__ p, int n, T *lds, Body &&body)
{
    stream_tiles_ex(p, n, lds, Same{}, body, NoEnd{});
}

// Star records: (x, y) when all masses are equal (the common mass is applied
// once at the end), (x, y, m, 0) otherwise.
template <bool EQUAL> struct StarRec;
template <> struct StarRec<true> {
    using T = double2;
    static __device__ __forceinline__ double mass(const double2 &) { return 1.0; }
};
template <> struct StarRec<false> {
    using T = double4;
    static __device__ __forceinline__ double mass(const double4 &s) { return s.z; }
};

__device__ __forceinline__ void wave_sum(double &v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
}

// Agent-scope atomic loads: what another work group published reaches this
// one through them whichever XCD (and L2) each runs on.
__device__ __forceinline__ unsigned long long load_acquire(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_acquire(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// FP64 Aberth sweep
// ---------------------------------------------------------------------------

// Running sums for one root z, u_i = 1/(z - z_i):
//   s1 = sum u_i                (for P'/P = F'/F + 2 s1)
//   s0 = sum m_i u_i            (lens mapping; equals m0 s1 for equal masses)
//   s2 = sum m_i u_i^2          (F = gamma + s2 - (1 - kappa_s) e^{-i phi});
//                               while accumulating, s2i holds sum m_i ux uy
//                               and finish() turns it into Im s2 = -2 that
//   s3 = sum m_i u_i^3          (F' = -2 s3)
//   R  = sum_{r != k} 1/(z - z_r)
// For equal masses the m_i factors are left out and applied once at the end.
struct Sums {
    double s1r, s1i, s0r, s0i, s2r, s2i, s3r, s3i, Rr, Ri;
};

__device__ __forceinline__ void zero(Sums &S)
{
    S.s1r = S.s1i = S.s0r = S.s0i = S.s2r = S.s2i = S.s3r = S.s3i = S.Rr = S.Ri = 0.0;
}

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star_inv(Sums &S, double dx, double dy, double inv,
                                             const T &s);

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star(Sums &S, double zr, double zi, const T &s)
{
    const double dx = zr - s.x;
    const double dy = zi - s.y;
    add_star_inv<EQUAL>(S, dx, dy, rcp_refined<RCP_STAR>(fma(dx, dx, dy * dy)), s);
}

// G consecutive star terms sharing one refined reciprocal (rcp_group), in
// the order add_star would take them.
template <bool EQUAL, int G, class T>
__device__ __forceinline__ void add_star_group(Sums &S, double zr, double zi, const T *r)
{
    double dx[G], dy[G], q[G], iq[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        dx[j] = zr - r[j].x;
        dy[j] = zi - r[j].y;
        q[j] = fma(dx[j], dx[j], dy[j] * dy[j]);
    }
    rcp_group<G, RCP_STAR>(q, iq);
#pragma unroll
    for (int j = 0; j < G; ++j) add_star_inv<EQUAL>(S, dx[j], dy[j], iq[j], r[j]);
}

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star_inv(Sums &S, double dx, double dy, double inv,
                                             const T &s)
{
    // u = conj(d) / |d|^2 = ux - i uy, with a = ux^2, b = uy^2:
    //   u^2 = (a - b) - 2 i ux uy,   u^3 = ux (a - 3b) + i uy (b - 3a).
    // Since a + b = |u|^2 = inv, only b is squared: t = a - b = inv - 2b,
    // a - 3b = t - 2b and b - 3a = 4b - 3 inv = -2t - inv.  Every
    // coefficient is an inline constant of the three-operand FP64 FMA and the
    // negated inv a source modifier, so u^2 and u^3 take one product and four
    // FMAs instead of two products and four FMAs.
    const double ux = dx * inv;
    const double uy = dy * inv;
    const double b = uy * uy;
    const double t = fma(-2.0, b, inv);
    const double c3r = fma(-2.0, b, t), c3i = fma(-2.0, t, -inv);
    S.s1r += ux;
    S.s1i -= uy;
    if (EQUAL) {
        S.s2r += t;
        S.s2i = fma(ux, uy, S.s2i);
        S.s3r = fma(ux, c3r, S.s3r);
        S.s3i = fma(uy, c3i, S.s3i);
    } else {
        const double mi = StarRec<EQUAL>::mass(s);
        const double mux = mi * ux, muy = mi * uy;
        S.s0r += mux;
        S.s0i -= muy;
        S.s2r = fma(mi, t, S.s2r);
        S.s2i = fma(mux, uy, S.s2i);
        S.s3r = fma(mux, c3r, S.s3r);
        S.s3i = fma(muy, c3i, S.s3i);
    }
}

// Root-root term of the Aberth correction, 1/(z - z_r) = conj(d) / |d|^2.
__device__ __forceinline__ void add_root(Sums &S, double zr, double zi, const double2 &o)
{
    const double dx = zr - o.x, dy = zi - o.y;
    const double inv = rcp_refined<RCP_ROOT>(fma(dx, dx, dy * dy));
    S.Rr = fma(dx, inv, S.Rr);
    S.Ri = fma(-dy, inv, S.Ri);
}

// G root-root terms sharing one refined reciprocal (rcp_group), in the order
// add_root would take them.  Two iterates at one point make every term of the
// group non-finite, as one term alone would be, and the iterate is nudged.
template <int G>
__device__ __forceinline__ void add_root_group(Sums &S, double zr, double zi, const double2 *r)
{
    double dx[G], dy[G], q[G], iq[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        dx[j] = zr - r[j].x;
        dy[j] = zi - r[j].y;
        q[j] = fma(dx[j], dx[j], dy[j] * dy[j]);
    }
    rcp_group<G, RCP_STAR>(q, iq);
#pragma unroll
    for (int j = 0; j < G; ++j) {
        S.Rr = fma(dx[j], iq[j], S.Rr);
        S.Ri = fma(-dy[j], iq[j], S.Ri);
    }
}

// The root-root term with FP32 arithmetic (MLCC_FP64_R32, warm rows).  Each
// coordinate enters as an FP32 pair hi + lo (hi = the FP64 value rounded to
// FP32, lo = the rounded remainder), and the difference is formed as
// (hi_k - hi_r) + (lo_k - lo_r): the first difference is exact for nearby
// roots, so the distance carries FP32 relative accuracy (~2^-24) at any
// separation, as does the FP32 reciprocal; the term runs at the FP32 issue
// rate.
struct SplitRoot {
    __device__ __forceinline__ float4 operator()(const double2 &o) const
    {
        const float hx = (float)o.x, hy = (float)o.y;
        return make_float4(hx, hy, (float)(o.x - (double)hx), (float)(o.y - (double)hy));
    }
};

__device__ __forceinline__ void add_root_hl(float &Rr, float &Ri, const float4 &z,
                                            const float4 &o)
{
    const float dx = (z.x - o.x) + (z.z - o.z);
    const float dy = (z.y - o.y) + (z.w - o.w);
    const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
    Rr = fmaf(dx, inv, Rr);
    Ri = fmaf(-dy, inv, Ri);
}

struct Update {
    double zr, zi;   // new iterate
    double wr, wi;   // its image under the lens map
    bool flag;       // converged
    double err;      // Newton polish: estimated error of the new iterate
};

// Degenerate iterate (on a star, or two iterates equal): nudge it off.
__device__ __forceinline__ void nudge(Update &u, double zr, double zi, int k)
{
    u.zr = zr + 1e-7 * (1 + (k & 7));
    u.zi = zi + 1e-7 * (1 + (k >> 3 & 7));
    u.flag = false;
}

// One Aberth-Ehrlich update from the sums at z (Sec. 3.2), the convergence
// test of the Sec. 3.2 footnote with the App. C bound on |1/mu|, and the
// lens map at the new iterate.  The map reuses the sums: with
// z' = z - D, sum m_i/(z' - z_i) = s0 + D s2 + D^2 s3 + O(D^3 sum m_i u_i^4),
// and D is below the convergence cutoffs once a root is flagged.
// Rectangular field (Sec. 4.2, App. B): the sheet adds -P(z) to F and
// -P'(z) to F', with P(z) = sum_{k=1..n} d_2k z^2k (real d_2k, see
// sheet_poly): P = w h(w), P' = 2 z g(w), w = z^2, h = sum d_2k w^(k-1),
// g = sum k d_2k w^(k-1), both by Horner's rule.
__device__ __forceinline__ void sheet_terms(const double *__restrict__ d, int n, double zr,
                                            double zi, double &Pr, double &Pi, double &Qr,
                                            double &Qi)
{
    const double wr = zr * zr - zi * zi, wi = 2.0 * zr * zi;
    double hr = d[n - 1], hi = 0.0, gr = n * d[n - 1], gi = 0.0;
    for (int k = n - 2; k >= 0; --k) {
        const double th = hr * wr - hi * wi + d[k];
        hi = hr * wi + hi * wr;
        hr = th;
        const double tg = gr * wr - gi * wi + (k + 1) * d[k];
        gi = gr * wi + gi * wr;
        gr = tg;
    }
    Pr = hr * wr - hi * wi;
    Pi = hr * wi + hi * wr;
    Qr = 2.0 * (gr * zr - gi * zi);
    Qi = 2.0 * (gr * zi + gi * zr);
}

// Its term of the lens map: sum_k d_2k / (2k + 1) z^(2k+1) = z^3 H(z^2) with
// H = sum (d_2k / (2k + 1)) w^(k-1); the map subtracts its conjugate.
__device__ __forceinline__ void sheet_map_term(const double *__restrict__ dm, int n, double zr,
                                               double zi, double &Qr, double &Qi)
{
    const double wr = zr * zr - zi * zi, wi = 2.0 * zr * zi;
    double hr = dm[n - 1], hi = 0.0;
    for (int k = n - 2; k >= 0; --k) {
        const double th = hr * wr - hi * wi + dm[k];
        hi = hr * wi + hi * wr;
        hr = th;
    }
    const double qr = hr * wr - hi * wi, qi = hr * wi + hi * wr;   // z^2 H
    Qr = qr * zr - qi * zi;
    Qi = qr * zi + qi * zr;
}

template <bool EQUAL>
__device__ __forceinline__ Update finish(Sums S, double zr, double zi, double m0, double2 e,
                                         double gamma, double a, double a1, double tol_step2,
                                         double tol_mu, int k, const double *sheet = nullptr,
                                         int n_poly = 0)
{
    S.s2i *= -2.0;
    if (EQUAL) {   // every mass equals m0: the sums above left it out
        S.s0r = m0 * S.s1r;
        S.s0i = m0 * S.s1i;
        S.s2r *= m0;
        S.s2i *= m0;
        S.s3r *= m0;
        S.s3i *= m0;
    }
    // F = gamma + S2 - (1 - kappa_s) e^{-i phi}, F' = -2 S3
    double Fr = gamma + S.s2r - e.x, Fi = S.s2i - e.y;
    double Fpr = -2.0 * S.s3r, Fpi = -2.0 * S.s3i;
    if (n_poly > 0) {   // rectangular field: F -= P(z), F' -= P'(z)
        double Pr, Pi, Qr, Qi;
        sheet_terms(sheet, n_poly, zr, zi, Pr, Pi, Qr, Qi);
        Fr -= Pr;
        Fi -= Pi;
        Fpr -= Qr;
        Fpi -= Qi;
    }
    // Aberth step: 1 / (F'/F + 2 S1 - R) = F / (F' + F (2 S1 - R))
    const double Gr = 2.0 * S.s1r - S.Rr, Gi = 2.0 * S.s1i - S.Ri;
    const double Dr = Fpr + (Fr * Gr - Fi * Gi);
    const double Di = Fpi + (Fr * Gi + Fi * Gr);
    const double den = Dr * Dr + Di * Di;
    const double stepr = (Fr * Dr + Fi * Di) / den;
    const double stepi = (Fi * Dr - Fr * Di) / den;
    Update u;
    u.zr = zr - stepr;
    u.zi = zi - stepi;
    const double aF = sqrt(Fr * Fr + Fi * Fi);
    u.flag = (stepr * stepr + stepi * stepi < tol_step2) || (aF * (aF + 2.0 * a1) < tol_mu);
    if (!isfinite(u.zr) || !isfinite(u.zi)) nudge(u, zr, zi, k);
    // T = s0 + D s2 + D^2 s3 with D = step
    const double d2r = stepr * stepr - stepi * stepi, d2i = 2.0 * stepr * stepi;
    const double Tr = S.s0r + (stepr * S.s2r - stepi * S.s2i) + (d2r * S.s3r - d2i * S.s3i);
    const double Ti = S.s0i + (stepr * S.s2i + stepi * S.s2r) + (d2r * S.s3i + d2i * S.s3r);
    // w = (1 - kappa_s) z' + gamma conj(z') - conj(T)
    u.wr = fma(a, u.zr, gamma * u.zr) - Tr;
    u.wi = fma(a, u.zi, -gamma * u.zi) + Ti;
    if (n_poly > 0) {   // rectangular field: - conj(sum_k d_2k / (2k + 1) z'^(2k+1))
        double Qr, Qi;
        sheet_map_term(sheet + n_poly, n_poly, u.zr, u.zi, Qr, Qi);
        u.wr -= Qr;
        u.wi += Qi;
    }
    return u;
}

// Resident waves per SIMD the sweep and polish kernels are compiled for
// (register budget 512 / waves); the loops keep their instruction counts.
// MLCC_XCD_MAP 1 keeps every front's blocks on one XCD (one L2 per front's
// iterate).  Measured on n10k it is ~30% slower than the plain order, which
// spreads each front over all eight XCDs: the fronts in a full pass change
// from round to round, and whole fronts per XCD leave XCDs idle.
#ifndef MLCC_XCD_MAP
#define MLCC_XCD_MAP 0
#endif
#ifndef MLCC_SWEEP_WAVES
#define MLCC_SWEEP_WAVES 4
#endif
#ifndef MLCC_POLISH_WAVES
#define MLCC_POLISH_WAVES 4
#endif
// The persistent kernel with multipole sums spends most of its time waiting
// on dependent loads; trading registers for resident waves did not pay on
// n10k mixed (4 waves 331 ms per step, 5: 362, 6: 386, 8: 423: the spills
// cost more than the extra waves hide), so it keeps the sweep's count.
#ifndef MLCC_FMM_WAVES
#define MLCC_FMM_WAVES MLCC_SWEEP_WAVES
#endif

// Blocks with at most this many unconverged roots take the cooperative path.
constexpr int SPARSE_MAX = 16;

// An FP64 cold start still unsettled after this many sweeps (cold starts
// take 11-30) starts again from the second set of start values (the
// default of mlcc_cc_params.cold_restart_sweeps).
constexpr int STALL_START = 100;

// Newton steps a root may take within one polish pass with multipole sums.
constexpr int FMM_POLISH_STEPS = 3;

// Further rows a polish pass with multipole sums may finish after its own
// (persistent schedule; see polish_pass).
#ifndef MLCC_FMM_XROWS
#define MLCC_FMM_XROWS 7
#endif
constexpr int FMM_XROWS = MLCC_FMM_XROWS;

// With direct star sums a pass over a few dozen stars is short, and the
// queue claim, the fences and the front's advance cost more than its sums:
// fields of at most XROWS_DIRECT_MAX_N stars also let a polish pass go on
// through up to DIRECT_XROWS further rows.  Larger fields keep one row per
// pass: the front keeps only the rows every one of its blocks finished, so
// with more blocks per front more of the further rows are thrown away, and
// their passes are long enough to pay for the queue (measured on batches of
// equal fields: 2.4x faster at N = 50, 1.7x at 100, 1.1x at 200, 3x slower
// at 500).
#ifndef MLCC_XROWS_DIRECT_MAX_N
#define MLCC_XROWS_DIRECT_MAX_N 160
#endif
#ifndef MLCC_DIRECT_XROWS
#define MLCC_DIRECT_XROWS 7
#endif
constexpr int XROWS_DIRECT_MAX_N = MLCC_XROWS_DIRECT_MAX_N;
constexpr int DIRECT_XROWS = MLCC_DIRECT_XROWS;

// ---------------------------------------------------------------------------
// Fast multipole star sums (Sec. 4.1: near stars directly, far stars through
// a local Taylor series)
// ---------------------------------------------------------------------------

// The stars are binned on a G x G grid of square cells of width w covering
// [c0 - 2R, c0 + 2R]^2, R the largest star distance from c0.  For a point z
// in cell C, the stars of C's 3 x 3 neighbourhood are summed directly; every
// other star is at least 1.5 w from C's centre c while |z - c| <= w / sqrt 2,
// and its terms come from C's local expansions
//   f_C(z) = sum_far w_i / (z - z_i) = sum_k a_k (z - c)^k,  a_k = -sum w_i / (z_i - c)^(k+1),
//   g_C(z) = the same with unit weights,
// (w_i = m_i, or 1 when all masses are equal and the kernels apply the mass
// once), whose derivatives give the other sums: sum w/(z - z_i)^2 = -f',
// sum w/(z - z_i)^3 = f''/2.  The ratio |z - c| / |z_i - c| <= 0.47 bounds the
// truncation after order p by ~0.47^(p+1) of each term.  The coefficients
// are stored scaled, b_k = a_k w^k = -(1/w) sum w_i v_i^(k+1) with
// v_i = w / (z_i - c), |v_i| <= 2/3, and the series is evaluated in
// tau = (z - c) / w, |tau| <= 0.71, so no power over- or underflows whatever
// the field's scale; f' and f'' take 1/w and 1/w^2.  Points outside the
// grid (|z - c0| >= 2R) use one expansion about c0 of all stars,
// f = sum_k M_k / (z - c0)^(k+1), M_k = sum w_i (z_i - c0)^k.  The polish's
// bound sum w |u|^4 takes, for the far stars, the per-cell constant
// sum_far w_i / dist(z_i, cell)^4 (or W / (|z - c0| - R)^4 outside).
struct FmmArgs {
    int32_t on, G, p, equal;
    int32_t stride;            // coefficients per cell: p + 1 rounded up to a multiple of 8
    double x0, y0, w, inv_w;   // grid origin (lower-left corner), cell width, 1 / w
    double cx, cy, R, wsum;    // c0, R, sum of the weights
    const int32_t *cell_start; // [G*G + 1]: stars of cell q are fstars[cell_start[q] ..)
    const double4 *fstars;     // stars sorted by cell: (x, y, m, 0)
    const double2 *cf, *cg;    // [G*G][stride]: b_k of f and of g (zero for k > p)
    const double *qfar;        // [G*G]
    const double2 *mf, *mg;    // [p + 1]: M_k about c0, weighted and unit
};

// Horner's rule for sum_k a_k t^k and its first two derivatives, over a
// coefficient row padded with zeros to a multiple of 8 (leading zeros leave
// the result unchanged).  Eight coefficients are loaded at a time, so the
// loads of a chunk are in flight together: the rows live in L2 or beyond,
// and one load per step would wait out that latency p times.
__device__ __forceinline__ void horner2(const double2 *__restrict__ a, int stride, double tr,
                                        double ti, double &fr, double &fi, double &dr, double &di,
                                        double &er, double &ei)
{
    fr = fi = dr = di = er = ei = 0.0;
    for (int c = stride - 8; c >= 0; c -= 8) {
        const double4 *a4 = reinterpret_cast<const double4 *>(a + c);
        double2 q[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double4 v = a4[j];
            q[2 * j] = make_double2(v.x, v.y);
            q[2 * j + 1] = make_double2(v.z, v.w);
        }
#pragma unroll
        for (int j = 7; j >= 0; --j) {
            // e = e t + 2 d, d = d t + f, f = f t + a_k (e = f'', d = f')
            const double ner = er * tr - ei * ti + 2.0 * dr, nei = er * ti + ei * tr + 2.0 * di;
            const double ndr = dr * tr - di * ti + fr, ndi = dr * ti + di * tr + fi;
            const double nfr = fr * tr - fi * ti + q[j].x, nfi = fr * ti + fi * tr + q[j].y;
            er = ner; ei = nei; dr = ndr; di = ndi; fr = nfr; fi = nfi;
        }
    }
}

__device__ __forceinline__ void horner0(const double2 *__restrict__ a, int stride, double tr,
                                        double ti, double &fr, double &fi)
{
    fr = fi = 0.0;
    for (int c = stride - 8; c >= 0; c -= 8) {
        const double4 *a4 = reinterpret_cast<const double4 *>(a + c);
        double2 q[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double4 v = a4[j];
            q[2 * j] = make_double2(v.x, v.y);
            q[2 * j + 1] = make_double2(v.z, v.w);
        }
#pragma unroll
        for (int j = 7; j >= 0; --j) {
            const double nfr = fr * tr - fi * ti + q[j].x, nfi = fr * ti + fi * tr + q[j].y;
            fr = nfr; fi = nfi;
        }
    }
}

// Far-field sums at z: f, f', f'' of the weighted expansion, g of the unit
// one (when want_g; the polish does not use it), and the bound on
// sum_far w |u|^4.  Sets `cell` to the cell index, or -1 outside the grid
// (then every star is far).
__device__ __forceinline__ void fmm_far(const FmmArgs &M, double zr, double zi, int &cell,
                                        double2 &f, double2 &f1, double2 &f2, double2 &g,
                                        double &q, bool want_g)
{
    const double fx = floor((zr - M.x0) / M.w), fy = floor((zi - M.y0) / M.w);
    if (fx >= 0.0 && fy >= 0.0 && fx < (double)M.G && fy < (double)M.G) {
        const int ix = (int)fx, iy = (int)fy;
        cell = iy * M.G + ix;
        const double tr = (zr - (M.x0 + (ix + 0.5) * M.w)) * M.inv_w;
        const double ti = (zi - (M.y0 + (iy + 0.5) * M.w)) * M.inv_w;
        const double2 *a = M.cf + (int64_t)cell * M.stride;
        horner2(a, M.stride, tr, ti, f.x, f.y, f1.x, f1.y, f2.x, f2.y);
        const double iw2 = M.inv_w * M.inv_w;
        f1.x *= M.inv_w; f1.y *= M.inv_w;
        f2.x *= iw2; f2.y *= iw2;
        if (M.equal) {
            g = f;
        } else if (want_g) {
            horner0(M.cg + (int64_t)cell * M.stride, M.stride, tr, ti, g.x, g.y);
        } else {
            g = make_double2(0.0, 0.0);
        }
        q = M.qfar[cell];
        return;
    }
    cell = -1;
    // t = 1 / (z - c0); f = t A(t), f' = -t^2 B(t), f'' = t^3 C(t) with
    // A = sum M_k t^k, B = sum (k+1) M_k t^k, C = sum (k+1)(k+2) M_k t^k
    const double dx = zr - M.cx, dy = zi - M.cy;
    const double r2 = dx * dx + dy * dy;
    const double tr = dx / r2, ti = -dy / r2;
    double Ar = M.mf[M.p].x, Ai = M.mf[M.p].y;
    double Br = (M.p + 1) * Ar, Bi = (M.p + 1) * Ai;
    double Cr = (double)(M.p + 1) * (M.p + 2) * Ar, Ci = (double)(M.p + 1) * (M.p + 2) * Ai;
    double Gr = M.mg[M.p].x, Gi = M.mg[M.p].y;
    for (int k = M.p - 1; k >= 0; --k) {
        const double2 mk = M.mf[k];
        double nr = Ar * tr - Ai * ti + mk.x, ni = Ar * ti + Ai * tr + mk.y;
        Ar = nr; Ai = ni;
        nr = Br * tr - Bi * ti + (k + 1) * mk.x; ni = Br * ti + Bi * tr + (k + 1) * mk.y;
        Br = nr; Bi = ni;
        const double c = (double)(k + 1) * (k + 2);
        nr = Cr * tr - Ci * ti + c * mk.x; ni = Cr * ti + Ci * tr + c * mk.y;
        Cr = nr; Ci = ni;
        const double2 gk = M.mg[k];
        nr = Gr * tr - Gi * ti + gk.x; ni = Gr * ti + Gi * tr + gk.y;
        Gr = nr; Gi = ni;
    }
    const double t2r = tr * tr - ti * ti, t2i = 2.0 * tr * ti;
    const double t3r = t2r * tr - t2i * ti, t3i = t2r * ti + t2i * tr;
    f = make_double2(tr * Ar - ti * Ai, tr * Ai + ti * Ar);
    f1 = make_double2(-(t2r * Br - t2i * Bi), -(t2r * Bi + t2i * Br));
    f2 = make_double2(t3r * Cr - t3i * Ci, t3r * Ci + t3i * Cr);
    g = M.equal ? f : make_double2(tr * Gr - ti * Gi, tr * Gi + ti * Gr);
    const double dd = sqrt(r2) - M.R;
    q = M.wsum / (dd * dd * dd * dd);
}

// Local expansions of every cell from its far stars, one work group of 64
// lanes per cell.  The stars go by in blocks of 64: lane k takes star k of
// the block, forms v = w / (z_k - c) (0 for a star of the 3 x 3 near cells,
// whose cell index rides in the record's fourth component) and writes its
// powers v^1 .. v^stride to LDS; then lane j adds up power j + 1 over the
// block's stars, weighted (f) and unweighted (g).  Successive products cost
// one complex multiply per power, against ~7 for raising each lane's star
// to its own power.  Lane k also adds its star's term of the bound
// sum_far w_i / dist(z_i, cell)^4.
__global__ void __launch_bounds__(64)
fmm_p2l(int32_t G, int32_t p, int32_t stride, double x0, double y0, double w, int32_t equal,
        int32_t n, const double4 *__restrict__ fstars, double2 *__restrict__ cf,
        double2 *__restrict__ cg, double *__restrict__ qfar)
{
    __shared__ double2 pw[64 * 65];   // pw[j * 65 + k] = v_k^(j+1); the pad spreads the banks
    __shared__ double wk[64];
    const int cell = blockIdx.x;
    const int ix = cell % G, iy = cell / G;
    const double cx = x0 + (ix + 0.5) * w, cy = y0 + (iy + 0.5) * w;
    const int lane = threadIdx.x;
    double fr = 0.0, fi = 0.0, gr = 0.0, gi = 0.0, q = 0.0;
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        double vr = 0.0, vi = 0.0, wi = 0.0;
        if (i < n) {
            const double4 st = fstars[i];
            const int sc = (int)st.w;
            const int sx = sc % G, sy = sc / G;
            if (abs(sx - ix) > 1 || abs(sy - iy) > 1) {
                const double dx = st.x - cx, dy = st.y - cy;
                const double r2 = dx * dx + dy * dy;
                vr = w * dx / r2;
                vi = -w * dy / r2;
                wi = equal ? 1.0 : st.z;
                const double ex = fmax(fabs(dx) - 0.5 * w, 0.0), ey = fmax(fabs(dy) - 0.5 * w, 0.0);
                const double d2 = ex * ex + ey * ey;
                q += wi / (d2 * d2);
            }
        }
        double pr = vr, pi = vi;
        for (int j = 0; j < stride; ++j) {
            pw[j * 65 + lane] = make_double2(pr, pi);
            const double t = pr * vr - pi * vi;
            pi = pr * vi + pi * vr;
            pr = t;
        }
        wk[lane] = wi;
        __syncthreads();
        if (lane < stride) {
#pragma unroll 8
            for (int k = 0; k < 64; ++k) {
                const double2 v = pw[lane * 65 + k];
                const double wt = wk[k];
                fr = fma(-wt, v.x, fr);
                fi = fma(-wt, v.y, fi);
                gr -= v.x;
                gi -= v.y;
            }
        }
        __syncthreads();
    }
    wave_sum(q);
    if (lane < stride) {
        const double s = lane <= p ? 1.0 / w : 0.0;
        cf[(int64_t)cell * stride + lane] = make_double2(fr * s, fi * s);
        cg[(int64_t)cell * stride + lane] = make_double2(gr * s, gi * s);
    }
    if (lane == 0) qfar[cell] = q;
}

// Calls body(star) for the stars of the 3 x 3 cells around `cell`, in the
// order of the sorted list (the block's three grid rows, each a run of
// adjacent cells), and returns their number.  The records are read
// NEAR_BATCH at a time, all loads of a batch issued before the first body
// runs: lanes of a wave sit in different cells, so every record is a
// gather from L2, and one load per body would wait out that latency for
// each near star.
#ifndef MLCC_NEAR_BATCH
#define MLCC_NEAR_BATCH 4
#endif
constexpr int NEAR_BATCH = MLCC_NEAR_BATCH;

template <class Body>
__device__ __forceinline__ int fmm_near(const FmmArgs &M, int cell, Body &&body)
{
    if (cell < 0) return 0;
    const int ix = cell % M.G, iy = cell / M.G;
    const int xa = max(ix - 1, 0), xb = min(ix + 1, M.G - 1);
    int lo[3], len[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int y = iy - 1 + r;
        // the cells of one grid row are adjacent in the sorted order
        const bool in = y >= 0 && y < M.G;
        const int q0 = (in ? y : iy) * M.G + xa, q1 = (in ? y : iy) * M.G + xb;
        const int i0 = M.cell_start[q0], i1 = M.cell_start[q1 + 1];
        lo[r] = i0;
        len[r] = in ? i1 - i0 : 0;
    }
    const int l01 = len[0] + len[1], n = l01 + len[2];
    for (int j = 0; j < n; j += NEAR_BATCH) {
        double4 rec[NEAR_BATCH];
#pragma unroll
        for (int u = 0; u < NEAR_BATCH; ++u) {
            const int t = j + u;
            const int i = t < len[0] ? lo[0] + t : t < l01 ? lo[1] + (t - len[0]) : lo[2] + (t - l01);
            rec[u] = M.fstars[t < n ? i : 0];   // past the end: a valid record, not used
        }
#pragma unroll
        for (int u = 0; u < NEAR_BATCH; ++u)
            if (j + u < n) body(rec[u]);
    }
    return n;
}

// A wave's multipole tallies (see FMM_STRIPES): near-field star terms,
// far-field evaluations (lanes that updated a root) and those evaluations
// times the field's star count (the direct terms they replace).  The values
// are wave-uniform.
struct FmmTally {
    unsigned long long near = 0, far = 0, far_n = 0;
};

__device__ __forceinline__ void fmm_count(FmmTally &t, bool act, int n_near, int n_stars)
{
    int v = act ? n_near : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    v = __builtin_amdgcn_readfirstlane(v);
    const int n_act = __popcll(__ballot(act));
    t.near += (unsigned long long)v;
    t.far += (unsigned long long)n_act;
    t.far_n += (unsigned long long)n_act * (unsigned long long)n_stars;
}

// Adds a wave's tallies to its work group's copy (kind: FMM_T_*).
__device__ __forceinline__ void fmm_flush(unsigned long long *tally, int kind, const FmmTally &t)
{
    if ((threadIdx.x & 63) == 0 && t.far) {
        unsigned long long *s = tally + (blockIdx.x % FMM_STRIPES) * FMM_STRIPE_U64 + kind;
        atomicAdd(&s[0], t.near);
        atomicAdd(&s[1], t.far);
        atomicAdd(&s[2], t.far_n);
    }
}

// Arguments shared by the kernels of a round.  Stars of every realisation
// are concatenated; each front names its realisation, and the grid maps a
// block to (front, block within the front) through bmap.
template <class T> struct RoundArgs {
    const T *stars;
    const Real *reals;
    const int2 *bmap;
    const Front *fronts;
    int32_t *flagrow;
    const double2 *cur;
    double2 *nxt;
    const double2 *unit;   // (cos phi_j, -sin phi_j)
    double tol_step, tol_step2, tol_mu;
    double *out_re, *out_im, *caus_re, *caus_im;
    double2 *bnd;
    int32_t *counts;
    int32_t *passupd;  // per front: roots updated by this round's pass (the control kernel sums them)
    Control *ctl;
    unsigned long long *fmm_tally;   // multipole tallies (FMM_STRIPES copies)
    double4 *vieta;    // two per block: row sums, and their error terms
    double *errbuf;    // estimated error of each polished root
    int32_t predictor;
    int32_t persistent; // the persistent scheduler: iterates by per-front parity
    double2 *iter0, *iter1;
    const double *sheet; // rectangular fields' sheet records (Real::sheet_off)
    const FmmArgs *fmm;  // fast multipole star sums: one record per field (kernels built with them)
    // Several rows per polish pass (persistent schedule, mixed form; null
    // otherwise): per front the fewest further rows any block of the pass
    // finished (reset to its field's Real::xrows by the front's finisher), the
    // largest Real::xrows of the call, and the stride of the row-sum slots
    // (the launch's block count).
    int32_t *xrows;
    int32_t xrow_max;
    int32_t nvslots;
};

// What one block knows about its front and star field.
template <class T> struct BlockCtx {
    int f, q, r, k0, k, lane, n_r, n_stars, row, stamp, dir, pred;
    int n_poly, n_extra;   // rectangular field: sheet terms and extra roots (else 0)
    const double *sheet;   // its record: d_2k, then d_2k / (2k + 1), then extra seeds
    int vslot;   // this block's slot in the per-block row sums (front order)
    int hist, end_row;   // finished rows behind the current one (<= 3); the front's last row
    bool valid, boundary;
    bool from_out;   // first pass of a row after a pass that ran several: the previous
                     // row's roots come from the output, not the iterate buffer
    int64_t base_f, out_off, bnd_row_off;
    const T *stars;
    const double2 *zsrc;
    double2 *nxt;
    double m0, gamma, a, a1;
    double2 e;   // (1 - kappa_s) e^{-i phi} of the front's row
};

template <class T>
__device__ __forceinline__ bool enter_fq(const RoundArgs<T> &A, int phase, int f, int q,
                                         BlockCtx<T> &B)
{
    B.f = f;
    B.q = q;
    const Front *F = A.fronts + B.f;
    if (F->state != FRONT_ACTIVE || (phase >= 0 && F->phase != phase)) return false;
    const Real *R = A.reals + F->real;
    B.r = F->real;
    B.row = F->row;
    B.stamp = F->stamp;
    B.vslot = F->blk0 + B.q;
    B.dir = F->dir;
    B.pred = (F->fresh && F->dir != 0 && F->hist >= 2) ? min(A.predictor, F->hist - 1) : 0;
    B.hist = F->hist;
    B.end_row = F->end_row;
    B.from_out = F->fresh == 2 && F->dir != 0;
    B.n_r = R->n_r;
    B.n_stars = R->n_stars;
    B.n_poly = R->n_poly;
    B.n_extra = R->n_extra;
    B.sheet = R->n_poly > 0 ? A.sheet + R->sheet_off : nullptr;
    B.stars = A.stars + R->star_off;
    B.m0 = R->m0;
    B.gamma = R->gamma;
    B.a = R->a;
    B.a1 = R->a1;
    B.base_f = F->it_off;
    if (A.persistent) {   // every front keeps its own ping-pong parity
        B.zsrc = (F->par ? A.iter1 : A.iter0) + F->it_off;
        B.nxt = F->par ? A.iter0 : A.iter1;
    } else {
        B.zsrc = A.cur + A.fronts[F->src].it_off;
        B.nxt = A.nxt;
    }
    B.out_off = R->out_off;
    B.boundary = F->bnd_slot >= 0 && B.row == F->end_row;
    B.bnd_row_off = R->bnd_off + (int64_t)max(F->bnd_slot, 0) * R->n_r;
    const double2 u = A.unit[B.row];
    B.e = make_double2(B.a * u.x, B.a * u.y);
    B.lane = threadIdx.x;
    B.k0 = B.q * 64;
    B.k = B.k0 + B.lane;
    B.valid = B.k < B.n_r;
    return true;
}

// Block context of this work group in a round: (front, block) from bmap.
template <class T>
__device__ __forceinline__ bool enter(const RoundArgs<T> &A, int phase, BlockCtx<T> &B)
{
    const int2 fq = A.bmap[blockIdx.x];
    return enter_fq(A, phase, fq.x, fq.y, B);
}

// Start of a new row's first pass for root k: extrapolation along its chain
// from the previous row (z1, the converged iterate) and the rows before it,
// which the subchain has already written to the output (same labels):
// linear 2 z1 - z2, quadratic 3 (z1 - z2) + z3.
template <class T>
__device__ __forceinline__ void predict(const RoundArgs<T> &A, const BlockCtx<T> &B, int k,
                                        double &zr, double &zi)
{
    const int64_t o2 = B.out_off + (int64_t)(B.row - 2 * B.dir) * B.n_r + k;
    const double x2 = A.out_re[o2], y2 = A.out_im[o2];
    if (B.pred == 1) {
        zr = 2.0 * zr - x2;
        zi = 2.0 * zi - y2;
    } else {
        const int64_t o3 = o2 - (int64_t)B.dir * B.n_r;
        zr = fma(3.0, zr - x2, A.out_re[o3]);
        zi = fma(3.0, zi - y2, A.out_im[o3]);
    }
}

// Write-back of a converged root: its row of the output (or the duplicate
// boundary row of a subchain) and its caustic image.
template <class T>
__device__ __forceinline__ void put(const RoundArgs<T> &A, const BlockCtx<T> &B, int k,
                                    const Update &u)
{
    if (B.boundary) {
        A.bnd[B.bnd_row_off + k] = make_double2(u.zr, u.zi);
        return;
    }
    const int64_t o = B.out_off + (int64_t)B.row * B.n_r + k;
    A.out_re[o] = u.zr;
    A.out_im[o] = u.zi;
    if (A.caus_re) {
        A.caus_re[o] = u.wr;
        A.caus_im[o] = u.wi;
    }
}

// Which FP64 Aberth passes take the root-root sum in FP32 (add_root_hl):
// warm rows of a field solved in MLCC_FP64_R32.  Cold starts, where the
// repulsion between the iterates steers global convergence from the seeds,
// MLCC_FP64 and the mixed form's FP64 restarts keep it in FP64.
__device__ __forceinline__ bool fast_roots_pass(const Front &fr, const Real &r)
{
    return r.root32 && fr.dir != 0 && fr.mode == PH_F64;
}

// One FP64 Aberth pass of a block (the block context is set by enter()).
// `tiles` holds two tiles of up to 32-byte records.
template <bool EQUAL, bool FMM>
__device__ __forceinline__ void sweep_f64_pass(const RoundArgs<typename StarRec<EQUAL>::T> &A,
                                               const BlockCtx<typename StarRec<EQUAL>::T> &B,
                                               double4 *tiles)
{
    using T = typename StarRec<EQUAL>::T;
    if (A.fronts[B.f].reseed) {
        // restart the row from its start values: the seeds z_i +- 1 for a
        // cold start, the previous row of the subchain otherwise.  The second
        // set for a stalled cold start: z_i +- i, and the extra roots of a
        // rectangular sheet turned by half their spacing.
        const bool second = A.fronts[B.f].seedvar > 0;
        if (B.valid) {
            double2 z;
            if (B.dir == 0 && B.k >= 2 * B.n_stars) {   // a rectangular sheet's extra root
                const int x = B.k - 2 * B.n_stars;
                z = make_double2(B.sheet[2 * B.n_poly + 2 * x], B.sheet[2 * B.n_poly + 2 * x + 1]);
                if (second) {
                    double sn, cs;
                    sincos(M_PI / (double)B.n_extra, &sn, &cs);
                    z = make_double2(z.x * cs - z.y * sn, z.x * sn + z.y * cs);
                }
            } else if (B.dir == 0) {
                const T st = B.stars[B.k >> 1];
                const double o = (B.k & 1) ? -1.0 : 1.0;
                z = second ? make_double2(st.x, st.y + o) : make_double2(st.x + o, st.y);
            } else {
                const int64_t o = B.out_off + (int64_t)(B.row - B.dir) * B.n_r + B.k;
                z = make_double2(A.out_re[o], A.out_im[o]);
            }
            B.nxt[B.base_f + B.k] = z;
        }
        const int n_valid = __popcll(__ballot(B.valid));
        if (threadIdx.x == 0) atomicAdd(&A.counts[B.f], n_valid);
        return;
    }
    const int lane = B.lane, k0 = B.k0, k = B.k, n_r = B.n_r, n_stars = B.n_stars;
    const bool valid = B.valid;
    const int64_t base_f = B.base_f;
    const double2 *__restrict__ zsrc = B.zsrc;
    const T *__restrict__ stars = B.stars;
    double2 *__restrict__ nxt = B.nxt;
    int32_t *__restrict__ flagrow = A.flagrow;
    const double m0 = B.m0, gamma = B.gamma, a = B.a, a1 = B.a1;
    const double tol_step2 = A.tol_step2, tol_mu = A.tol_mu;
    double zr = 0.0, zi = 0.0;
    bool act = false;
    if (valid) {
        const double2 z = zsrc[k];
        zr = z.x;
        zi = z.y;
        act = flagrow[base_f + k] != B.stamp;
        if (B.pred) predict(A, B, k, zr, zi);
    }
    const unsigned long long amask = __ballot(act);
    const int n_act = __popcll(amask);
    if (valid && !act) nxt[base_f + k] = make_double2(zr, zi);   // carried forward
    if (n_act == 0) return;

    const double2 e = B.e;
    auto store = [&](int kk, const Update &u) {
        nxt[base_f + kk] = make_double2(u.zr, u.zi);
        if (!u.flag) return;
        flagrow[base_f + kk] = B.stamp;
        put(A, B, kk, u);
    };

    int n_after = 0;
    if (n_act <= SPARSE_MAX) {
        // Few roots left (a straggler sweep): the wave takes them one at a
        // time, lanes splitting the star and root sums, then a butterfly
        // reduction.  Latency per root drops ~64x against one lane doing it.
        unsigned long long mm = amask;
        while (mm) {
            const int l = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            const double xk = __shfl(zr, l, 64), yk = __shfl(zi, l, 64);
            Sums S;
            zero(S);
#pragma unroll 4
            for (int i = lane; i < n_stars; i += 64) add_star<EQUAL>(S, xk, yk, stars[i]);
            const int kk = k0 + l;
#pragma unroll 4
            for (int j = lane; j < n_r; j += 64)
                if (j != kk) add_root(S, xk, yk, zsrc[j]);
            wave_sum(S.s1r); wave_sum(S.s1i);
            if (!EQUAL) { wave_sum(S.s0r); wave_sum(S.s0i); }
            wave_sum(S.s2r); wave_sum(S.s2i);
            wave_sum(S.s3r); wave_sum(S.s3i);
            wave_sum(S.Rr); wave_sum(S.Ri);
            const Update u = finish<EQUAL>(S, xk, yk, m0, e, gamma, a, a1, tol_step2, tol_mu, kk,
                                           B.sheet, B.n_poly);
            if (lane == l) store(kk, u);
            n_after += u.flag ? 0 : 1;
        }
    } else {
        Sums S;
        zero(S);
        if constexpr (FMM) {
            int cell;
            double2 f, f1, f2, g;
            double q;
            fmm_far(A.fmm[B.r], zr, zi, cell, f, f1, f2, g, q, true);
            const int n_near = fmm_near(A.fmm[B.r], cell, [&](const double4 &s4) {
                if constexpr (EQUAL) add_star<EQUAL>(S, zr, zi, make_double2(s4.x, s4.y));
                else add_star<EQUAL>(S, zr, zi, s4);
            });
            FmmTally tl;
            fmm_count(tl, act, n_near, n_stars);
            fmm_flush(A.fmm_tally, FMM_T_F64, tl);
            // far terms in the accumulators' conventions (s2i holds -Im/2)
            S.s1r += g.x; S.s1i += g.y;
            if (!EQUAL) { S.s0r += f.x; S.s0i += f.y; }
            S.s2r -= f1.x; S.s2i += 0.5 * f1.y;
            S.s3r += 0.5 * f2.x; S.s3i += 0.5 * f2.y;
        } else {
            stream_tiles_grouped(stars, n_stars, reinterpret_cast<T *>(tiles),
                                 [&](auto g, const T *r) {
                                     add_star_group<EQUAL, decltype(g)::value>(S, zr, zi, r);
                                 });
        }
        if (!fast_roots_pass(A.fronts[B.f], A.reals[B.r])) {
            // the other roots in FP64, in groups outside the own block;
            // within it one at a time, skipping the root itself
            double2 *rtiles = reinterpret_cast<double2 *>(tiles);
            auto group = [&](auto g, const double2 *r) {
                add_root_group<decltype(g)::value>(S, zr, zi, r);
            };
            const int own_hi = min(k0 + 64, n_r);
            stream_tiles_grouped(zsrc, k0, rtiles, group);
            stream_tiles(zsrc + k0, own_hi - k0, rtiles, [&](int j, const double2 &o) {
                Sums T2 = S;
                add_root(T2, zr, zi, o);
                const bool self = j == lane;
                S.Rr = self ? S.Rr : T2.Rr;
                S.Ri = self ? S.Ri : T2.Ri;
            });
            stream_tiles_grouped(zsrc + own_hi, n_r - own_hi, rtiles, group);
            const Update u = finish<EQUAL>(S, zr, zi, m0, e, gamma, a, a1, tol_step2, tol_mu, k,
                                           B.sheet, B.n_poly);
            if (act) store(k, u);
            n_after = __popcll(__ballot(act && !u.flag));
        } else {
        // root-root sum in FP32 (add_root_hl), summed per tile and carried
        // across tiles in FP64
        float4 *rtiles = reinterpret_cast<float4 *>(tiles);
        const float4 zs = SplitRoot{}(make_double2(zr, zi));
        float pr = 0.f, pi = 0.f;
        auto other = [&](int, const float4 &o) { add_root_hl(pr, pi, zs, o); };
        auto carry = [&]() {
            S.Rr += (double)pr;
            S.Ri += (double)pi;
            pr = pi = 0.f;
        };
        const int own_hi = min(k0 + 64, n_r);
        stream_tiles_ex(zsrc, k0, rtiles, SplitRoot{}, other, carry);
        stream_tiles_ex(zsrc + k0, own_hi - k0, rtiles, SplitRoot{}, [&](int j, const float4 &o) {
            float tr = pr, ti = pi;
            add_root_hl(tr, ti, zs, o);
            const bool self = j == lane;
            pr = self ? pr : tr;
            pi = self ? pi : ti;
        }, carry);
        stream_tiles_ex(zsrc + own_hi, n_r - own_hi, rtiles, SplitRoot{}, other, carry);
        const Update u = finish<EQUAL>(S, zr, zi, m0, e, gamma, a, a1, tol_step2, tol_mu, k,
                                       B.sheet, B.n_poly);
        if (act) store(k, u);
        n_after = __popcll(__ballot(act && !u.flag));
        }
    }
    if (lane == 0) {
        if (n_after) atomicAdd(&A.counts[B.f], n_after);
        atomicAdd(&A.passupd[B.f], n_act);
    }
}

template <bool EQUAL, bool FMM>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MLCC_SWEEP_WAVES, 8)))
aberth_sweep_f64(RoundArgs<typename StarRec<EQUAL>::T> A)
{
    __shared__ double4 tiles[128];
    BlockCtx<typename StarRec<EQUAL>::T> B;
    if (!enter(A, PH_F64, B)) return;
    sweep_f64_pass<EQUAL, FMM>(A, B, tiles);
}

// ---------------------------------------------------------------------------
// FP32 Aberth sweep (mixed mode: cold starts, rows without a prediction, and
// rows the polish did not settle)
// ---------------------------------------------------------------------------

// Steps shorter than this (theta_E units) are below what the FP32 sums
// resolve reliably; the FP64 polish takes over from there.
constexpr double TOL_F32 = 1e-6;

// One Aberth step for every root of the row with the sums in FP32.  The
// distance to each star is formed in FP64 and rounded, so no precision is
// lost to the size of the coordinates; each 64-star tile is summed in FP32
// and the tile sums are carried in FP64, which keeps the large near-star
// terms from swamping the accumulation.  The other roots enter in FP32
// coordinates (they only steer the step).  The step itself and the new
// iterate are FP64.
template <bool EQUAL, bool FMM>
__device__ __forceinline__ void sweep_f32_pass(const RoundArgs<typename StarRec<EQUAL>::T> &A,
                                               const BlockCtx<typename StarRec<EQUAL>::T> &B,
                                               double4 *tiles)
{
    using T = typename StarRec<EQUAL>::T;
    const int lane = B.lane, k0 = B.k0, k = B.k, n_r = B.n_r, n_stars = B.n_stars;
    const bool valid = B.valid;
    const int64_t base_f = B.base_f;
    const double2 *__restrict__ zsrc = B.zsrc;
    const T *__restrict__ stars = B.stars;
    const double m0 = B.m0, gamma = B.gamma;
    double zr = 0.0, zi = 0.0;
    if (valid) {
        const double2 z = zsrc[k];
        zr = z.x;
        zi = z.y;
        if (B.pred) predict(A, B, k, zr, zi);
    }
    // star sums: FP32 within a tile, FP64 across tiles (with multipole
    // sums: the near stars' terms and the cell's series, in FP64)
    double S1r = 0, S1i = 0, S2r = 0, S2i = 0, S3r = 0, S3i = 0;
    float p1r = 0, p1i = 0, p2r = 0, p2i = 0, p3r = 0, p3i = 0;
    if constexpr (FMM) {
        Sums S;
        zero(S);
        int cell;
        double2 f, f1, f2, g;
        double q;
        fmm_far(A.fmm[B.r], zr, zi, cell, f, f1, f2, g, q, true);
        const int n_near = fmm_near(A.fmm[B.r], cell, [&](const double4 &s4) {
            if constexpr (EQUAL) add_star<EQUAL>(S, zr, zi, make_double2(s4.x, s4.y));
            else add_star<EQUAL>(S, zr, zi, s4);
        });
        FmmTally tl;
        fmm_count(tl, valid, n_near, n_stars);
        fmm_flush(A.fmm_tally, FMM_T_F32, tl);
        S1r = S.s1r + g.x; S1i = S.s1i + g.y;
        S2r = S.s2r - f1.x; S2i = S.s2i + 0.5 * f1.y;
        S3r = S.s3r + 0.5 * f2.x; S3i = S.s3i + 0.5 * f2.y;
    } else {
        stream_tiles_ex(
            stars, n_stars, reinterpret_cast<T *>(tiles), Same{},
            [&](int, const T &s) {
                const float dx = (float)(zr - s.x), dy = (float)(zi - s.y);
                const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
                // a = ux^2, b = uy^2: p2i accumulates sum m ux uy (Im u^2 =
                // -2 ux uy), and since a + b = inv, a - 3b = inv - 4b and
                // b - 3a = inv - 4a
                const float ux = dx * inv, uy = dy * inv;
                const float a = ux * ux, b = uy * uy;
                p1r += ux;
                p1i -= uy;
                if (EQUAL) {
                    p2r += a - b;
                    p2i = fmaf(ux, uy, p2i);
                    p3r = fmaf(ux, fmaf(-4.0f, b, inv), p3r);
                    p3i = fmaf(uy, fmaf(-4.0f, a, inv), p3i);
                } else {
                    const float mi = (float)StarRec<EQUAL>::mass(s);
                    const float mux = mi * ux, muy = mi * uy;
                    p2r = fmaf(mi, a - b, p2r);
                    p2i = fmaf(mux, uy, p2i);
                    p3r = fmaf(mux, fmaf(-4.0f, b, inv), p3r);
                    p3i = fmaf(muy, fmaf(-4.0f, a, inv), p3i);
                }
            },
            [&]() {
                S1r += p1r; S1i += p1i; S2r += p2r; S2i += p2i; S3r += p3r; S3i += p3i;
                p1r = p1i = p2r = p2i = p3r = p3i = 0.f;
            });
    }
    // root-root sum in FP32 coordinates
    const float zr32 = (float)zr, zi32 = (float)zi;
    double Rr = 0, Ri = 0;
    float qr = 0, qi = 0;
    float2 *rt = reinterpret_cast<float2 *>(tiles);
    auto to32 = [](const double2 &o) { return make_float2((float)o.x, (float)o.y); };
    auto flush = [&]() { Rr += qr; Ri += qi; qr = qi = 0.f; };
    auto other = [&](int, const float2 &o) {
        const float dx = zr32 - o.x, dy = zi32 - o.y;
        const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
        qr = fmaf(dx, inv, qr);
        qi = fmaf(-dy, inv, qi);
    };
    const int own_hi = min(k0 + 64, n_r);
    stream_tiles_ex(zsrc, k0, rt, to32, other, flush);
    stream_tiles_ex(zsrc + k0, own_hi - k0, rt, to32,
                    [&](int j, const float2 &o) {
                        const float dx = zr32 - o.x, dy = zi32 - o.y;
                        const float inv = __builtin_amdgcn_rcpf(fmaf(dx, dx, dy * dy));
                        const bool self = j == lane;
                        qr = self ? qr : fmaf(dx, inv, qr);
                        qi = self ? qi : fmaf(-dy, inv, qi);
                    },
                    flush);
    stream_tiles_ex(zsrc + own_hi, n_r - own_hi, rt, to32, other, flush);

    S2i *= -2.0;
    if (EQUAL) {
        S2r *= m0; S2i *= m0; S3r *= m0; S3i *= m0;
    }
    const double2 e = B.e;
    const double Fr = gamma + S2r - e.x, Fi = S2i - e.y;
    const double Fpr = -2.0 * S3r, Fpi = -2.0 * S3i;
    const double Gr = 2.0 * S1r - Rr, Gi = 2.0 * S1i - Ri;
    const double Dr = Fpr + (Fr * Gr - Fi * Gi);
    const double Di = Fpi + (Fr * Gi + Fi * Gr);
    const double den = Dr * Dr + Di * Di;
    Update u;
    u.zr = zr - (Fr * Dr + Fi * Di) / den;
    u.zi = zi - (Fi * Dr - Fr * Di) / den;
    if (!isfinite(u.zr) || !isfinite(u.zi)) nudge(u, zr, zi, k);
    if (valid) B.nxt[base_f + k] = make_double2(u.zr, u.zi);
    const int n_valid = __popcll(__ballot(valid));
    // roots that moved by more than the FP32 sweep can resolve are still
    // on their way (the control kernel uses this for cold starts)
    const double mr = u.zr - zr, mi = u.zi - zi;
    const int n_moving = __popcll(__ballot(valid && !(mr * mr + mi * mi <= TOL_F32 * TOL_F32)));
    if (lane == 0) {
        if (n_moving) atomicAdd(&A.counts[B.f], n_moving);
        atomicAdd(&A.passupd[B.f], n_valid);
    }
}

template <bool EQUAL, bool FMM>
__global__ void __launch_bounds__(64)
aberth_sweep_f32(RoundArgs<typename StarRec<EQUAL>::T> A)
{
    __shared__ double4 tiles[128];
    BlockCtx<typename StarRec<EQUAL>::T> B;
    if (!enter(A, PH_F32, B)) return;
    sweep_f32_pass<EQUAL, FMM>(A, B, tiles);
}

// ---------------------------------------------------------------------------
// FP64 Newton polish (mixed mode)
// ---------------------------------------------------------------------------

// Sums for the Newton polish: s0 = sum m u, s2 = sum m u^2, s3 = sum m u^3
// (F = gamma + s2 - (1 - kappa_s) e^{-i phi}, F' = -2 s3) and the real
// q = sum m |u|^4, which bounds |F''| = 6 |sum m u^4| <= 6 q.
struct PSums {
    double s0r, s0i, s2r, s2i, s3r, s3i, q;
};

__device__ __forceinline__ void zero(PSums &S)
{
    S.s0r = S.s0i = S.s2r = S.s2i = S.s3r = S.s3i = S.q = 0.0;
}

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star_polish_inv(PSums &S, double dx, double dy, double inv,
                                                    const T &s);

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star_polish(PSums &S, double zr, double zi, const T &s)
{
    const double dx = zr - s.x;
    const double dy = zi - s.y;
    add_star_polish_inv<EQUAL>(S, dx, dy, rcp_refined<RCP_STAR>(fma(dx, dx, dy * dy)), s);
}

// G consecutive polish star terms sharing one refined reciprocal.
template <bool EQUAL, int G, class T>
__device__ __forceinline__ void add_star_polish_group(PSums &S, double zr, double zi, const T *r)
{
    double dx[G], dy[G], q[G], iq[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        dx[j] = zr - r[j].x;
        dy[j] = zi - r[j].y;
        q[j] = fma(dx[j], dx[j], dy[j] * dy[j]);
    }
    rcp_group<G, RCP_STAR>(q, iq);
#pragma unroll
    for (int j = 0; j < G; ++j) add_star_polish_inv<EQUAL>(S, dx[j], dy[j], iq[j], r[j]);
}

template <bool EQUAL, class T>
__device__ __forceinline__ void add_star_polish_inv(PSums &S, double dx, double dy, double inv,
                                                    const T &s)
{
    // u = ux - i uy, a = ux^2, b = uy^2:  u^2 = (a - b) - 2i ux uy,
    // u^3 = ux (a - 3b) + i uy (b - 3a), formed from b alone as in
    // add_star_inv (t = a - b = inv - 2b, a - 3b = t - 2b, b - 3a = -2t - inv);
    // |u|^4 = inv^2
    // (s2i accumulates sum m ux uy; polish_finish turns it into Im s2 = -2 that)
    const double uy = dy * inv;
    const double b = uy * uy;
    const double t = fma(-2.0, b, inv);
    const double c3r = fma(-2.0, b, t), c3i = fma(-2.0, t, -inv);
    if (EQUAL) {
        const double ux = dx * inv;
        S.s0r += ux; S.s0i -= uy;
        S.s2r += t;
        S.s2i = fma(ux, uy, S.s2i);
        S.s3r = fma(ux, c3r, S.s3r);
        S.s3i = fma(uy, c3i, S.s3i);
        S.q = fma(inv, inv, S.q);
    } else {
        // the mass enters through m inv, shared by m u = conj(d) m inv and
        // the bound's m inv^2; u's real part is not needed on its own
        const double mi = StarRec<EQUAL>::mass(s);
        const double minv = mi * inv;
        const double mux = dx * minv, muy = mi * uy;
        S.s0r += mux; S.s0i -= muy;
        S.s2r = fma(mi, t, S.s2r);
        S.s2i = fma(mux, uy, S.s2i);
        S.s3r = fma(mux, c3r, S.s3r);
        S.s3i = fma(muy, c3i, S.s3i);
        S.q = fma(minv, inv, S.q);
    }
}

// Newton step z' = z - D, D = F/F', accepted on the paper's cutoffs for the
// step just taken (|D| < tol_step, or the App. C bound on |1/mu| at z), or
// when the error it leaves, at most ~|F''| |D|^2 / (2 |F'|) by quadratic
// convergence, is below POLISH_ERR_FRACTION * tol_step -- always while
// |D| |F''/F'| < 0.1 on the bound |F''| <= 6 q, so that z' lies well inside
// the region where Newton's method converges to one root.  The error bound
// is recorded for the row identities.  The caustic of z' reuses
// the sums: sum m/(z' - z_i) = s0 + D s2 + D^2 s3 + O(D^3 sum m |u|^4).
constexpr double POLISH_ERR_FRACTION = 1e-3;

template <bool EQUAL>
__device__ __forceinline__ Update polish_finish(PSums S, double zr, double zi, double m0,
                                                double2 e, double gamma, double a, double a1,
                                                double tol_step2, double tol_mu, int k)
{
    S.s2i *= -2.0;
    if (EQUAL) {
        S.s0r *= m0; S.s0i *= m0; S.s2r *= m0; S.s2i *= m0;
        S.s3r *= m0; S.s3i *= m0; S.q *= m0;
    }
    const double Fr = gamma + S.s2r - e.x, Fi = S.s2i - e.y;
    const double Fpr = -2.0 * S.s3r, Fpi = -2.0 * S.s3i;
    const double den = Fpr * Fpr + Fpi * Fpi;
    const double Dr = (Fr * Fpr + Fi * Fpi) / den;
    const double Di = (Fi * Fpr - Fr * Fpi) / den;
    Update u;
    u.zr = zr - Dr;
    u.zi = zi - Di;
    const double aD2 = Dr * Dr + Di * Di, aD = sqrt(aD2);
    const double ratio = 6.0 * S.q / sqrt(den);   // bound on |F''/F'|
    const double aF = sqrt(Fr * Fr + Fi * Fi);
    u.err = 0.5 * ratio * aD2;
    u.flag = (aD2 < tol_step2 || aF * (aF + 2.0 * a1) < tol_mu ||
              u.err * u.err < POLISH_ERR_FRACTION * POLISH_ERR_FRACTION * tol_step2) &&
             aD * ratio < 0.1;
    if (!isfinite(u.zr) || !isfinite(u.zi)) nudge(u, zr, zi, k);
    const double d2r = Dr * Dr - Di * Di, d2i = 2.0 * Dr * Di;
    const double Tr = S.s0r + (Dr * S.s2r - Di * S.s2i) + (d2r * S.s3r - d2i * S.s3i);
    const double Ti = S.s0i + (Dr * S.s2i + Di * S.s2r) + (d2r * S.s3i + d2i * S.s3r);
    u.wr = fma(a, u.zr, gamma * u.zr) - Tr;
    u.wi = fma(a, u.zi, -gamma * u.zi) + Ti;
    return u;
}

template <bool EQUAL, bool FMM>
__device__ __forceinline__ void polish_pass(const RoundArgs<typename StarRec<EQUAL>::T> &A,
                                            const BlockCtx<typename StarRec<EQUAL>::T> &B,
                                            double4 *tiles)
{
    using T = typename StarRec<EQUAL>::T;
    const int lane = B.lane, k0 = B.k0, k = B.k, n_stars = B.n_stars;
    const bool valid = B.valid;
    const int64_t base_f = B.base_f;
    const double2 *__restrict__ zsrc = B.zsrc;
    const T *__restrict__ stars = B.stars;
    double2 *__restrict__ nxt = B.nxt;
    int32_t *__restrict__ flagrow = A.flagrow;
    const double m0 = B.m0, gamma = B.gamma, a = B.a, a1 = B.a1;
    const double tol_step2 = A.tol_step2, tol_mu = A.tol_mu;
    double zr = 0.0, zi = 0.0;
    bool act = false;
    double er_ = 0.0;   // estimated error of the value this root ends the pass with
    FmmTally ptl;       // multipole tallies of the whole pass, added once at its end
    if (valid) {
        if (B.from_out) {
            const int64_t o = B.out_off + (int64_t)(B.row - B.dir) * B.n_r + k;
            zr = A.out_re[o];
            zi = A.out_im[o];
        } else {
            const double2 z = zsrc[k];
            zr = z.x;
            zi = z.y;
        }
        act = flagrow[base_f + k] != B.stamp;
        if (B.pred) predict(A, B, k, zr, zi);
        if (!act) er_ = A.errbuf[base_f + k];   // accepted in an earlier pass of this row
    }
    const unsigned long long amask = __ballot(act);
    const int n_act = __popcll(amask);
    const double2 e = B.e;
    double fr_ = zr, fi_ = zi;   // value this root ends the pass with
    int n_after = 0;
    int n_steps = -1;   // Newton steps this lane took (-1: one per active root)
    // (with multipole sums a root's star terms are a few near stars and one
    // series, as cheap per lane as a wave's share of a direct sum, so the
    // wave never takes its few roots one at a time)
    if (n_act > 0 && n_act <= SPARSE_MAX && !FMM) {
        unsigned long long mm = amask;
        while (mm) {
            const int l = __ffsll((long long)mm) - 1;
            mm &= mm - 1;
            const double xk = __shfl(zr, l, 64), yk = __shfl(zi, l, 64);
            PSums S;
            zero(S);
#pragma unroll 4
            for (int i = lane; i < n_stars; i += 64) add_star_polish<EQUAL>(S, xk, yk, stars[i]);
            wave_sum(S.s0r); wave_sum(S.s0i); wave_sum(S.s2r); wave_sum(S.s2i);
            wave_sum(S.s3r); wave_sum(S.s3i); wave_sum(S.q);
            const int kk = k0 + l;
            const Update u = polish_finish<EQUAL>(S, xk, yk, m0, e, gamma, a, a1, tol_step2, tol_mu, kk);
            if (lane == l) {
                nxt[base_f + kk] = make_double2(u.zr, u.zi);
                fr_ = u.zr;
                fi_ = u.zi;
                if (u.flag) {
                    er_ = u.err;
                    A.errbuf[base_f + kk] = u.err;
                    flagrow[base_f + kk] = B.stamp;
                    put(A, B, kk, u);
                }
            }
            n_after += u.flag ? 0 : 1;
        }
    } else if (n_act > 0) {
        Update u{};
        if constexpr (FMM) {
            // A Newton step needs only its own root's sums, and with
            // multipole sums those cost a few near stars and one series: a
            // root the acceptance test turns down takes its next step in the
            // same pass (up to FMM_POLISH_STEPS), instead of waiting a pass.
            double xr = zr, xi = zi;
            bool open = act;
            n_steps = 0;
            for (int it = 0; it < FMM_POLISH_STEPS; ++it) {
                PSums S;
                zero(S);
                int cell;
                double2 f, f1, f2, g;
                double q;
                fmm_far(A.fmm[B.r], xr, xi, cell, f, f1, f2, g, q, false);
                const int n_near = fmm_near(A.fmm[B.r], cell, [&](const double4 &s4) {
                    if constexpr (EQUAL)
                        add_star_polish<EQUAL>(S, xr, xi, make_double2(s4.x, s4.y));
                    else add_star_polish<EQUAL>(S, xr, xi, s4);
                });
                fmm_count(ptl, open, n_near, n_stars);
                S.s0r += f.x; S.s0i += f.y;
                S.s2r -= f1.x; S.s2i += 0.5 * f1.y;
                S.s3r += 0.5 * f2.x; S.s3i += 0.5 * f2.y;
                S.q += q;
                const Update v = polish_finish<EQUAL>(S, xr, xi, m0, e, gamma, a, a1, tol_step2,
                                                      tol_mu, k);
                if (open) {
                    u = v;
                    n_steps += 1;
                    if (v.flag) {
                        open = false;
                    } else {
                        xr = v.zr;
                        xi = v.zi;
                    }
                }
                if (!__ballot(open)) break;
            }
        } else {
            PSums S;
            zero(S);
            stream_tiles_grouped(stars, n_stars, reinterpret_cast<T *>(tiles),
                                 [&](auto g, const T *r) {
                                     add_star_polish_group<EQUAL, decltype(g)::value>(S, zr, zi,
                                                                                      r);
                                 });
            u = polish_finish<EQUAL>(S, zr, zi, m0, e, gamma, a, a1, tol_step2, tol_mu, k);
        }
        if (act) {
            nxt[base_f + k] = make_double2(u.zr, u.zi);
            fr_ = u.zr;
            fi_ = u.zi;
            if (u.flag) {
                er_ = u.err;
                A.errbuf[base_f + k] = u.err;
                flagrow[base_f + k] = B.stamp;
                put(A, B, k, u);
            }
        }
        n_after = __popcll(__ballot(act && !u.flag));
    }
    if (valid && !act) nxt[base_f + k] = make_double2(zr, zi);
    // this block's share of the row sums sum r and sum r^2 (row identities),
    // and of what bounds their error: the roots' own estimated errors, and
    // sum |r|, sum |r|^2 for the rounding of the sums
    double s1r = valid ? fr_ : 0.0, s1i = valid ? fi_ : 0.0;
    double s2r = valid ? fr_ * fr_ - fi_ * fi_ : 0.0, s2i = valid ? 2.0 * fr_ * fi_ : 0.0;
    const double ab2 = valid ? fr_ * fr_ + fi_ * fi_ : 0.0, ab = sqrt(ab2);
    double t_e = er_, t_e2 = er_ * (2.0 * ab + er_), t_a = ab, t_a2 = ab2;
    wave_sum(s1r); wave_sum(s1i); wave_sum(s2r); wave_sum(s2i);
    wave_sum(t_e); wave_sum(t_e2); wave_sum(t_a); wave_sum(t_a2);
    if (lane == 0) {
        A.vieta[2 * B.vslot] = make_double4(s1r, s1i, s2r, s2i);
        A.vieta[2 * B.vslot + 1] = make_double4(t_e, t_e2, t_a, t_a2);
        if (n_after) atomicAdd(&A.counts[B.f], n_after);
    }
    int n_xsteps = 0;   // Newton steps this lane took in further rows
    const int xmax = A.xrows ? A.reals[B.r].xrows : 0;
    if (xmax > 0) {
        // Several rows per pass: once every root of the block is accepted in
        // this row, the block goes on through the next rows of its front by
        // itself, each root from the chain prediction of its own earlier rows,
        // as the front's first pass of that row would (a Newton step couples
        // no roots).  A row counts only when every root of the block is
        // accepted in it: then its roots and caustics are written and its row
        // sums kept in slot x; the first row that leaves a root open ends the
        // pass, and nothing of it is kept.  The front's last row is left to a
        // pass of its own.
        int done = 0;
        if (B.dir != 0 && A.predictor > 0 && n_after == 0) {
            double pr = fr_, pi = fi_;   // this root in the row before
            const unsigned long long vmask = __ballot(valid);
            for (int x = 1; x <= xmax; ++x) {
                BlockCtx<T> C = B;
                C.row = B.row + x * B.dir;
                if ((C.row - B.end_row) * B.dir >= 0) break;
                // another block of the front already stopped short of this row:
                // the front will not keep it
                if (load_relaxed(&A.xrows[B.f]) < x) break;
                C.boundary = false;
                C.pred = min(A.predictor, min(B.hist + x, 3) - 1);
                const double2 un = A.unit[C.row];
                const double2 ex = make_double2(a * un.x, a * un.y);
                double xr = pr, xi = pi;
                if (valid && C.pred) predict(A, C, k, xr, xi);
                bool open = valid;
                Update u{};
                if constexpr (FMM) {
                    for (int it = 0; it < FMM_POLISH_STEPS; ++it) {
                        PSums S;
                        zero(S);
                        int cell;
                        double2 f, f1, f2, g;
                        double q;
                        fmm_far(A.fmm[B.r], xr, xi, cell, f, f1, f2, g, q, false);
                        const int n_near = fmm_near(A.fmm[B.r], cell, [&](const double4 &s4) {
                            if constexpr (EQUAL)
                                add_star_polish<EQUAL>(S, xr, xi, make_double2(s4.x, s4.y));
                            else add_star_polish<EQUAL>(S, xr, xi, s4);
                        });
                        fmm_count(ptl, open, n_near, n_stars);
                        S.s0r += f.x; S.s0i += f.y;
                        S.s2r -= f1.x; S.s2i += 0.5 * f1.y;
                        S.s3r += 0.5 * f2.x; S.s3i += 0.5 * f2.y;
                        S.q += q;
                        const Update v = polish_finish<EQUAL>(S, xr, xi, m0, ex, gamma, a, a1,
                                                              tol_step2, tol_mu, k);
                        if (open) {
                            u = v;
                            n_xsteps += 1;
                            if (v.flag) {
                                open = false;
                            } else {
                                xr = v.zr;
                                xi = v.zi;
                            }
                        }
                        if (!__ballot(open)) break;
                    }
                } else {
                    // one Newton step per root from direct sums, exactly as
                    // the first pass of the row takes it: the whole wave per
                    // root when the block holds few roots, else one lane each
                    if (__popcll(vmask) <= SPARSE_MAX) {
                        unsigned long long mm = vmask;
                        while (mm) {
                            const int l = __ffsll((long long)mm) - 1;
                            mm &= mm - 1;
                            const double xk = __shfl(xr, l, 64), yk = __shfl(xi, l, 64);
                            PSums S;
                            zero(S);
#pragma unroll 4
                            for (int i = lane; i < n_stars; i += 64)
                                add_star_polish<EQUAL>(S, xk, yk, stars[i]);
                            wave_sum(S.s0r); wave_sum(S.s0i); wave_sum(S.s2r); wave_sum(S.s2i);
                            wave_sum(S.s3r); wave_sum(S.s3i); wave_sum(S.q);
                            const Update v = polish_finish<EQUAL>(S, xk, yk, m0, ex, gamma, a,
                                                                  a1, tol_step2, tol_mu, k0 + l);
                            if (lane == l) u = v;
                        }
                    } else {
                        PSums S;
                        zero(S);
                        stream_tiles_grouped(stars, n_stars, reinterpret_cast<T *>(tiles),
                                             [&](auto g, const T *r) {
                                                 add_star_polish_group<EQUAL, decltype(g)::value>(
                                                     S, xr, xi, r);
                                             });
                        u = polish_finish<EQUAL>(S, xr, xi, m0, ex, gamma, a, a1, tol_step2, tol_mu,
                                                 k);
                    }
                    open = valid && !u.flag;
                }
                // (with direct sums the finisher counts the rows the front keeps)
                if (__ballot(open)) {
                    if (lane == 0) atomicMin(&A.xrows[B.f], done);   // tell the other blocks now
                    break;
                }
                if (valid) put(A, C, k, u);
                double t1r = valid ? u.zr : 0.0, t1i = valid ? u.zi : 0.0;
                double t2r = valid ? u.zr * u.zr - u.zi * u.zi : 0.0;
                double t2i = valid ? 2.0 * u.zr * u.zi : 0.0;
                const double b2 = valid ? u.zr * u.zr + u.zi * u.zi : 0.0, b1 = sqrt(b2);
                const double ue = valid ? u.err : 0.0;
                double q_e = ue, q_e2 = ue * (2.0 * b1 + ue), q_a = b1, q_a2 = b2;
                wave_sum(t1r); wave_sum(t1i); wave_sum(t2r); wave_sum(t2i);
                wave_sum(q_e); wave_sum(q_e2); wave_sum(q_a); wave_sum(q_a2);
                if (lane == 0) {
                    const int64_t sl = 2 * ((int64_t)x * A.nvslots + B.vslot);
                    A.vieta[sl] = make_double4(t1r, t1i, t2r, t2i);
                    A.vieta[sl + 1] = make_double4(q_e, q_e2, q_a, q_a2);
                }
                pr = u.zr;
                pi = u.zi;
                done = x;
            }
        }
        if (lane == 0) atomicMin(&A.xrows[B.f], done);
    }
    // updates of the pass: one per active root, or its Newton steps (those of
    // further rows included)
    int n_upd = (n_steps >= 0 ? n_steps : 0) + n_xsteps;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) n_upd += __shfl_xor(n_upd, off, 64);
    if (n_steps < 0) n_upd += n_act;
    if (lane == 0 && n_upd) atomicAdd(&A.passupd[B.f], n_upd);
    if constexpr (FMM) fmm_flush(A.fmm_tally, FMM_T_POLISH, ptl);
}

template <bool EQUAL, bool FMM>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MLCC_POLISH_WAVES, 8)))
newton_polish_f64(RoundArgs<typename StarRec<EQUAL>::T> A)
{
    __shared__ double4 tiles[128];
    BlockCtx<typename StarRec<EQUAL>::T> B;
    if (!enter(A, PH_POLISH, B)) return;
    polish_pass<EQUAL, FMM>(A, B, tiles);
}

// ---------------------------------------------------------------------------
// Seeds and front control
// ---------------------------------------------------------------------------

// Cold-start seeds at the centre row of each subchain: root 2i <- z_i + 1,
// root 2i+1 <- z_i - 1 (Sec. 3.2).  One thread per root of every front that
// starts cold (the downward front of each subchain).
template <class T>
__global__ void seed_centres(const T *__restrict__ stars, const Real *__restrict__ reals,
                             const Front *__restrict__ fronts, const int2 *__restrict__ bmap,
                             const double *__restrict__ sheet, double2 *__restrict__ iter)
{
    const int2 fq = bmap[blockIdx.x];
    const Front *F = fronts + fq.x;
    if (F->dir != 0) return;
    const Real *R = reals + F->real;
    const int k = fq.y * 64 + threadIdx.x;
    if (k >= R->n_r) return;
    if (k >= 2 * R->n_stars) {   // a rectangular sheet's extra root (Sec. 3.2: on a circle)
        const double *sx = sheet + R->sheet_off + 2 * R->n_poly + 2 * (k - 2 * R->n_stars);
        iter[F->it_off + k] = make_double2(sx[0], sx[1]);
        return;
    }
    const T z = stars[R->star_off + (k >> 1)];
    iter[F->it_off + k] = make_double2(z.x + ((k & 1) ? -1.0 : 1.0), z.y);
}

// Row sums of every front in the polish phase: one wave per front adds its
// blocks' partial sums in a fixed order (lanes stride over the blocks, then
// a butterfly), so the control kernel reads eight numbers per front.
__global__ void __launch_bounds__(64)
row_sums(const Front *__restrict__ fronts, const Real *__restrict__ reals,
         const double4 *__restrict__ vieta, double4 *__restrict__ vsum)
{
    const int f = blockIdx.x;
    const Front *F = fronts + f;
    if (F->state != FRONT_ACTIVE || F->phase != PH_POLISH) return;
    const int bpf = (reals[F->real].n_r + 63) / 64;
    double v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0;
    for (int b = threadIdx.x; b < bpf; b += 64) {
        const double4 t = vieta[2 * (F->blk0 + b)], q = vieta[2 * (F->blk0 + b) + 1];
        v0 += t.x; v1 += t.y; v2 += t.z; v3 += t.w;
        v4 += q.x; v5 += q.y; v6 += q.z; v7 += q.w;
    }
    wave_sum(v0); wave_sum(v1); wave_sum(v2); wave_sum(v3);
    wave_sum(v4); wave_sum(v5); wave_sum(v6); wave_sum(v7);
    if (threadIdx.x == 0) {
        vsum[2 * f] = make_double4(v0, v1, v2, v3);
        vsum[2 * f + 1] = make_double4(v4, v5, v6, v7);
    }
}

constexpr int CONTROL_THREADS = 256;
constexpr int MAX_FRONTS = 1 << 16;
constexpr int MAX_POLISH = 3;
constexpr int F32_STALL = 4;

// Puts a front at the start of its (new) row.  Mixed mode: a row with a
// chain prediction goes straight to the FP64 polish; one without (the two
// rows next to a subchain centre, or predictor 0) starts with an FP32 sweep.
__device__ __forceinline__ void start_row(Front &fr, int predictor)
{
    fr.sweeps = 0;
    fr.passes = 0;
    fr.tried = 0;
    fr.f32 = 0;
    fr.best = 0x7fffffff;
    fr.stall = 0;
    fr.passes_row = 0;
    fr.reseed = 0;
    fr.stamp = 4 * fr.row;
    fr.fresh = 1;
    if (fr.mode == PH_F64)
        fr.phase = PH_F64;
    else
        fr.phase = (predictor > 0 && fr.hist >= 2) ? PH_POLISH : PH_F32;
}

__device__ __forceinline__ void row_done(Front &fr, int32_t *st, int f, int predictor)
{
    if (fr.row == fr.end_row) {
        fr.state = FRONT_DONE;
        if (st) st[f] = FRONT_DONE;
    } else {
        fr.row += fr.dir;
        fr.hist = min(fr.hist + 1, 3);
        start_row(fr, predictor);
    }
}

// Every root of the current row converged.  A cold start hands the upward
// half of its subchain to its partner front and turns downward itself; a
// warm row moves one row on or finishes at its end row.
__device__ __forceinline__ int row_converged(Front &fr, int f, Front *fronts, int32_t *st,
                                             int f0, int predictor)
{
    if (fr.dir == 0) {
        fr.cold = fr.passes_row;
        const int p = fr.partner;
        const int centre = fr.row;
        Front pr = fronts[p];
        pr.state = FRONT_ACTIVE;
        pr.row = centre + 1;
        pr.dir = 1;
        pr.src = f;    // first pass reads the converged centre row
        pr.hist = 1;   // the centre row
        start_row(pr, predictor);
        fronts[p] = pr;
        if (st) st[p - f0] = FRONT_ACTIVE;
        fr.dir = -1;
        fr.row = centre - 1;
        fr.hist = 1;
        start_row(fr, predictor);
        return p;
    }
    fr.max_warm = max(fr.max_warm, fr.passes_row);
    row_done(fr, st, f - f0, predictor);
    return -1;
}

// The two row identities of a polished row (see aberth_control) from its
// row sums rs: sum r and sum r^2, then the error terms.
__device__ __forceinline__ bool row_identities_hold(const Real &R, double2 u, const double4 *rs)
{
    const int bpf = (R.n_r + 63) / 64;
    const double4 t = rs[0], q = rs[1];
    const double a1r = t.x, a1i = t.y, a2r = t.z, a2i = t.w;
    const double se = q.x, se2 = q.y, sa = q.z, sa2 = q.w;
    const double cr = R.gamma - R.a * u.x, ci = -R.a * u.y;   // c(phi)
    const double cc = cr * cr + ci * ci;
    const double mcr = R.M * cr / cc, mci = -R.M * ci / cc;   // M / c
    const double e1r = a1r - 2.0 * R.sz_r, e1i = a1i - 2.0 * R.sz_i;
    const double e2r = a2r - (2.0 * R.sz2_r - 2.0 * mcr);
    const double e2i = a2i - (2.0 * R.sz2_i - 2.0 * mci);
    const double u_ro = 1.1102230246251565e-16;
    const double tol1 = 2.0 * se + 2.0 * (12 + bpf) * u_ro * sa + R.tol1;
    const double tol2 = 2.0 * se2 + 2.0 * (13 + bpf) * u_ro * sa2 + R.tol2 +
                        16.0 * u_ro * sqrt(mcr * mcr + mci * mci);
    return sqrt(e1r * e1r + e1i * e1i) <= tol1 && sqrt(e2r * e2r + e2i * e2i) <= tol2;
}

// One front after its pass (c = its roots still unconverged, or, after an
// FP32 sweep, still moving; rs = its row sums when the pass was a polish).
// Returns the partner front a finished cold start activated, else -1.
// `st` (the control kernel's LDS copy of the states) may be null.
__device__ __attribute__((noinline)) int advance_front(Front &fr, int f, int32_t c, const double4 *rs, Front *fronts,
                             int32_t *st, int f0, Control *ctl, const Real *reals,
                             const double2 *unit, int max_cold, int max_warm, int predictor)
{
    int partner = -1;
    fr.npass += 1;
    fr.src = f;
    fr.fresh = 0;
    fr.passes_row += 1;
    if (fr.phase == PH_F32) {
        fr.f32 += 1;
        bool polish = true;
        if (fr.dir == 0) {
            if (c < fr.best) {
                fr.best = c;
                fr.stall = 0;
            } else {
                fr.stall += 1;
            }
            polish = c == 0 || fr.stall >= F32_STALL || fr.f32 >= max_cold;
        }
        if (polish) {
            if (fr.tried & TRIED_POLISH) fr.stamp += 1;   // polish every root again
            fr.tried |= TRIED_F32;
            fr.phase = PH_POLISH;
            fr.passes = 0;
        }
    } else if (fr.phase == PH_POLISH) {
        fr.tried |= TRIED_POLISH;
        bool retry = false;
        if (c == 0) {
            if (row_identities_hold(reals[fr.real], unit[fr.row], rs))
                partner = row_converged(fr, f, fronts, st, f0, predictor);
            else
                retry = true;
        } else if (++fr.passes >= MAX_POLISH) {
            retry = true;
        }
        if (retry) {
            if (!(fr.tried & TRIED_F32)) {
                fr.phase = PH_F32;
            } else {
                // plain FP64 Aberth sweeps over every root from the row's
                // start values: Newton steps may have sent two columns to
                // one root, which Aberth steps from there would not undo
                fr.stamp += 1;
                fr.reseed = 1;
                fr.phase = PH_F64;
                fr.sweeps = 0;
                atomicAdd((unsigned long long *)&ctl->rows_fallback, 1ull);
            }
        }
    } else if (fr.reseed) {
        fr.reseed = 0;   // the restart pass only reloaded the start values
    } else if (c == 0) {
        partner = row_converged(fr, f, fronts, st, f0, predictor);
    } else {
        fr.sweeps += 1;
        if (fr.dir == 0 && fr.phase == PH_F64 && fr.seedvar == 0 &&
            fr.sweeps >= reals[fr.real].restart && fr.sweeps < max_cold) {
            // a stalled cold start: once, all over again from other seeds
            fr.seedvar = 1;
            fr.reseed = 1;
            fr.stamp += 1;
            fr.sweeps = 0;
            atomicAdd((unsigned long long *)&ctl->cold_restarts, 1ull);
        } else if (fr.sweeps >= (fr.dir == 0 ? max_cold : max_warm)) {
            fr.state = FRONT_FAILED;
            if (st) st[f - f0] = FRONT_FAILED;
            atomicAdd(&ctl->failed_rows, 1);
            atomicAdd((unsigned long long *)&ctl->unconverged, (unsigned long long)c);
            if (fr.dir == 0) {
                fronts[fr.partner].state = FRONT_FAILED;
                if (st) st[fr.partner - f0] = FRONT_FAILED;
            }
        }
    }
    return partner;
}

// Advances every front after a round (counts[f] = roots of front f still
// unconverged after its pass, or, after an FP32 sweep, still moving).
//   FP64 phase: a converged row moves on (row_converged); a front that
//     reaches its sweep cap stops and is counted as failed (with a partner
//     it can no longer start).
//   FP32 phase (mixed): warm rows take one sweep; a cold start sweeps until
//     no root moves by more than TOL_F32, or that count has not fallen for
//     F32_STALL sweeps, or max_cold; then the polish.
//   Polish phase (mixed): a row whose roots were all accepted and whose sums
//     satisfy the row identities has converged.  Otherwise more polish
//     passes (up to MAX_POLISH); then, once per row, an FP32 sweep of the
//     whole row and the polish again; then the row restarts from its start
//     values (seeds, or the previous row) with plain FP64 Aberth sweeps.
//
// Row identities: the rationalised polynomial has leading coefficient
// c = gamma - (1 - kappa_s) e^{-i phi} and next coefficient -2 c sum z_i, so
// sum r = 2 sum z_i and sum r^2 = 2 sum z_i^2 - 2 M / c (M = sum m_i).  A
// root found twice and one missed shifts them by the distance of the two.
// The test allows the roots' own estimated errors (twice over) plus a
// bound on the rounding of the sums: partial sums of 64 values by a
// butterfly, then (row_sums) lanes striding over the blocks and another
// butterfly, gives at most (12 + blocks) unit roundoffs of sum |r| (one
// more for sum |r|^2, whose terms round too).
//
// `st` keeps the states in LDS: the two fronts of a subchain sit in adjacent
// lanes of one wave, which read their states before either is written, so
// a partner activated in this pass is not also advanced in it.  With more
// fronts than fit, the kernel runs as several work groups over disjoint
// ranges that keep each subchain's two fronts together.
__global__ void __launch_bounds__(CONTROL_THREADS)
aberth_control(Front *__restrict__ fronts, int32_t *__restrict__ counts, int32_t n_fronts,
               Control *__restrict__ ctl, int32_t max_cold, int32_t max_warm,
               int32_t *__restrict__ workflag, const double4 *__restrict__ vsum,
               const Real *__restrict__ reals, const double2 *__restrict__ unit,
               int32_t fronts_per_group, int32_t predictor, int32_t *__restrict__ passupd)
{
    __shared__ int32_t st[4096];
    __shared__ int32_t s_active, s_live;
    __shared__ unsigned long long s_upd[4], s_star[4];   // by phase; [3]: fast-root FP64 passes
    const int tid = threadIdx.x;
    const int f0 = blockIdx.x * fronts_per_group;
    const int f1 = min(n_fronts, f0 + fronts_per_group);
    if (tid == 0) {
        s_active = 0;
        s_live = 0;
    }
    if (tid < 4) s_upd[tid] = s_star[tid] = 0ull;
    unsigned long long my_upd[4] = {0ull, 0ull, 0ull, 0ull}, my_star[4] = {0ull, 0ull, 0ull, 0ull};
    for (int f = f0 + tid; f < f1; f += CONTROL_THREADS) st[f - f0] = fronts[f].state;
    __syncthreads();
    for (int f = f0 + tid; f < f1; f += CONTROL_THREADS) {
        if (st[f - f0] != FRONT_ACTIVE) continue;
        Front fr = fronts[f];
        atomicOr(&s_live, 1 << fr.phase);
        {   // this round's updates of the front, by pass kind (FLOP counts weigh them by N)
            const unsigned long long u = (unsigned)passupd[f];
            passupd[f] = 0;
            const unsigned long long us = u * (unsigned)reals[fr.real].n_stars;
            my_upd[fr.phase] += u;
            my_star[fr.phase] += us;
            if (fr.phase == PH_F64 && fast_roots_pass(fr, reals[fr.real])) {
                my_upd[3] += u;
                my_star[3] += us;
            }
        }
        const int32_t c = counts[f];
        counts[f] = 0;
        advance_front(fr, f, c, vsum + 2 * f, fronts, st, f0, ctl, reals, unit, max_cold,
                      max_warm, predictor);
        fronts[f] = fr;
    }
    for (int q = 0; q < 4; ++q) {
        if (my_upd[q]) {
            atomicAdd(&s_upd[q], my_upd[q]);
            atomicAdd(&s_star[q], my_star[q]);
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (s_upd[PH_F64]) {
            atomicAdd(&ctl->updates, s_upd[PH_F64]);
            atomicAdd(&ctl->star_updates, s_star[PH_F64]);
        }
        if (s_upd[PH_F32]) {
            atomicAdd(&ctl->updates_f32, s_upd[PH_F32]);
            atomicAdd(&ctl->star_updates_f32, s_star[PH_F32]);
        }
        if (s_upd[PH_POLISH]) {
            atomicAdd(&ctl->polish_updates, s_upd[PH_POLISH]);
            atomicAdd(&ctl->star_updates_polish, s_star[PH_POLISH]);
        }
        if (s_upd[3]) {
            atomicAdd(&ctl->updates_fast, s_upd[3]);
            atomicAdd(&ctl->star_updates_fast, s_star[3]);
        }
    }
    int mine = 0;
    for (int f = f0 + tid; f < f1; f += CONTROL_THREADS)
        mine += (st[f - f0] == FRONT_ACTIVE || st[f - f0] == FRONT_IDLE);
    if (mine) atomicAdd(&s_active, mine);
    __syncthreads();
    if (tid == 0) {
        // several groups: each adds its share; the first round of counting is
        // reset by the host-side clear kernel below
        atomicAdd(&ctl->active_fronts, s_active);
        if (s_live) atomicOr(workflag, s_live);
    }
}

// Clears the per-round totals the control groups add into, and counts the
// round as live if any group saw an active front (runs after them).
__global__ void control_begin(Control *__restrict__ ctl, int32_t *__restrict__ workflag)
{
    if (threadIdx.x == 0) {
        ctl->active_fronts = 0;
        *workflag = 0;
    }
}

__global__ void control_end(Control *__restrict__ ctl, const int32_t *__restrict__ workflag)
{
    if (threadIdx.x == 0 && *workflag) ctl->live_sweeps += 1;
}

// ---------------------------------------------------------------------------
// Persistent scheduler
// ---------------------------------------------------------------------------
//
// One launch of as many single-wave work groups as fit on the chip.  Work
// items are (front, block) passes in a device-side ring: a worker claims
// the next slot, waits until it is filled, runs the pass the front's phase
// asks for, and the worker that completes the last block of a front's pass
// advances that front (advance_front) and queues its next pass, so fronts
// move on independently instead of in global rounds.  Each front keeps its
// own ping-pong parity; a cold start hands its converged centre row to its
// partner by copying it into the partner's buffer.  No worker ever waits
// for another one's pass: it waits only for its claimed slot, which the
// worker that queued the work fills, and leaves when every front is done,
// or, failing that, after a wall-clock interval without any pass finishing
// anywhere (the call then reports an error).

// Queue header; every counter sits on a cache line of its own, so workers
// polling one of them do not slow the atomics on another.
struct PQueue {
    unsigned long long head;      // next slot to claim
    unsigned long long pad0[31];
    unsigned long long tail;      // next slot to fill
    unsigned long long pad1[31];
    unsigned long long progress;  // passes completed
    unsigned long long pad2[31];
    int32_t done;                 // fronts finished (DONE or FAILED)
    int32_t pad3[63];
    int32_t abort;                // a worker saw no progress for too long
    int32_t pad4[63];
};
// Slot sequence numbers are spread one per 64-byte line.
constexpr int SEQ_STRIDE = 8;

// Queues the bpf block passes of front f (whole wave).
__device__ __forceinline__ void push_front(PQueue *q, int2 *tasks, unsigned long long *seq,
                                           unsigned long long mask, int f, int bpf)
{
    unsigned long long base = 0;
    if (threadIdx.x == 0) base = atomicAdd(&q->tail, (unsigned long long)bpf);
    base = __shfl(base, 0, 64);
    for (int i = threadIdx.x; i < bpf; i += 64) tasks[(base + i) & mask] = make_int2(f, i);
    // publishes the tasks and everything the wave wrote before them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int i = threadIdx.x; i < bpf; i += 64)
        __hip_atomic_store(&seq[((base + i) & mask) * SEQ_STRIDE], base + i + 1,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool EQUAL, bool FMM>
__global__ void __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(FMM ? MLCC_FMM_WAVES : MLCC_SWEEP_WAVES, 8)))
aberth_persistent(RoundArgs<typename StarRec<EQUAL>::T> A, Front *__restrict__ fronts_w,
                  PQueue *__restrict__ q, int2 *__restrict__ tasks,
                  unsigned long long *__restrict__ seq, unsigned long long mask,
                  int32_t *__restrict__ fdone, int32_t n_fronts, int32_t max_cold,
                  int32_t max_warm, unsigned long long stall_ticks)
{
    using T = typename StarRec<EQUAL>::T;
    __shared__ double4 tiles[128];
    const int lane = threadIdx.x;
    for (;;) {
        int tf = -1, tq = 0;
        if (lane == 0) {
            const unsigned long long t = atomicAdd(&q->head, 1ull);
            const unsigned long long *my = &seq[(t & mask) * SEQ_STRIDE];
            unsigned long long seen = load_relaxed(&q->progress);
            unsigned long long t0 = wall_clock64();
            for (unsigned it = 1;; ++it) {
                if (load_relaxed(my) == t + 1) {
                    (void)load_acquire(my);
                    const int2 w = tasks[t & mask];
                    tf = w.x;
                    tq = w.y;
                    break;
                }
                if ((it & 31) == 0) {   // the shared counters, now and then
                    if (load_relaxed(&q->abort)) break;
                    if (load_relaxed(&q->done) >= n_fronts) break;
                    const unsigned long long pnow = load_relaxed(&q->progress);
                    const unsigned long long now = wall_clock64();
                    if (pnow != seen) {
                        seen = pnow;
                        t0 = now;
                    } else if (now - t0 > stall_ticks) {
                        atomicExch(&q->abort, 1);
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        tf = __shfl(tf, 0, 64);
        tq = __shfl(tq, 0, 64);
        if (tf < 0) return;

        BlockCtx<T> B;
        if (enter_fq(A, -1, tf, tq, B)) {
            const int ph = A.fronts[tf].phase;
            if (ph == PH_F64)
                sweep_f64_pass<EQUAL, FMM>(A, B, tiles);
            else if (ph == PH_F32)
                sweep_f32_pass<EQUAL, FMM>(A, B, tiles);
            else
                polish_pass<EQUAL, FMM>(A, B, tiles);
        }
        // the last block of the front's pass advances the front; every
        // block publishes its writes before counting itself done
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const Front *F = A.fronts + tf;
        const Real *R = A.reals + F->real;
        const int bpf = (R->n_r + 63) >> 6;
        int last = 0;
        if (lane == 0) last = atomicAdd(&fdone[tf], 1) + 1 == bpf;
        last = __shfl(last, 0, 64);
        if (!last) continue;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        Front fr = fronts_w[tf];
        double4 rs[2] = {make_double4(0, 0, 0, 0), make_double4(0, 0, 0, 0)};
        if (fr.phase == PH_POLISH) {
            double v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0;
            for (int b = lane; b < bpf; b += 64) {
                const double4 t = A.vieta[2 * (fr.blk0 + b)], u = A.vieta[2 * (fr.blk0 + b) + 1];
                v0 += t.x; v1 += t.y; v2 += t.z; v3 += t.w;
                v4 += u.x; v5 += u.y; v6 += u.z; v7 += u.w;
            }
            wave_sum(v0); wave_sum(v1); wave_sum(v2); wave_sum(v3);
            wave_sum(v4); wave_sum(v5); wave_sum(v6); wave_sum(v7);
            rs[0] = make_double4(v0, v1, v2, v3);
            rs[1] = make_double4(v4, v5, v6, v7);
        }
        int partner = -1, state = FRONT_ACTIVE, finished = 0, xr = 0, dir0 = 0;
        int64_t p_off = 0;
        int p_par = 0;
        if (lane == 0) {
            fdone[tf] = 0;
            const unsigned long long u = (unsigned)A.passupd[tf];
            A.passupd[tf] = 0;
            const unsigned long long us = u * (unsigned)R->n_stars;
            if (fr.phase == PH_F64) {
                atomicAdd(&A.ctl->updates, u);
                atomicAdd(&A.ctl->star_updates, us);
                if (fast_roots_pass(fr, *R)) {
                    atomicAdd(&A.ctl->updates_fast, u);
                    atomicAdd(&A.ctl->star_updates_fast, us);
                }
            } else if (fr.phase == PH_F32) {
                atomicAdd(&A.ctl->updates_f32, u);
                atomicAdd(&A.ctl->star_updates_f32, us);
            } else {
                atomicAdd(&A.ctl->polish_updates, u);
                atomicAdd(&A.ctl->star_updates_polish, us);
            }
            const int32_t c = A.counts[tf];
            A.counts[tf] = 0;
            dir0 = fr.dir;
            const int row0 = fr.row, ph0 = fr.phase;
            partner = advance_front(fr, tf, c, rs, fronts_w, nullptr, 0, A.ctl, A.reals, A.unit,
                                    max_cold, max_warm, A.predictor);
            fr.par ^= 1;   // the pass wrote the other buffer
            if (A.xrows && ph0 == PH_POLISH) {
                // further rows the pass finished in every block (see polish_pass)
                xr = A.xrows[tf];
                A.xrows[tf] = R->xrows;
                if (!(dir0 != 0 && fr.state == FRONT_ACTIVE && fr.phase == PH_POLISH &&
                      fr.row == row0 + dir0))
                    xr = 0;
            }
        }
        // the further rows, in order, while their row identities hold
        xr = __shfl(xr, 0, 64);
        int moved = 0;
        for (int x = 1; x <= xr; ++x) {
            double v0 = 0, v1 = 0, v2 = 0, v3 = 0, v4 = 0, v5 = 0, v6 = 0, v7 = 0;
            for (int b = lane; b < bpf; b += 64) {
                const int64_t sl = 2 * ((int64_t)x * A.nvslots + fr.blk0 + b);
                const double4 t = A.vieta[sl], u = A.vieta[sl + 1];
                v0 += t.x; v1 += t.y; v2 += t.z; v3 += t.w;
                v4 += u.x; v5 += u.y; v6 += u.z; v7 += u.w;
            }
            wave_sum(v0); wave_sum(v1); wave_sum(v2); wave_sum(v3);
            wave_sum(v4); wave_sum(v5); wave_sum(v6); wave_sum(v7);
            int ok = 0;
            if (lane == 0) {
                const double4 rx[2] = {make_double4(v0, v1, v2, v3), make_double4(v4, v5, v6, v7)};
                if (row_identities_hold(*R, A.unit[fr.row], rx)) {
                    row_converged(fr, tf, fronts_w, nullptr, 0, A.predictor);
                    ok = 1;
                }
            }
            ok = __shfl(ok, 0, 64);
            if (!ok) break;
            moved = x;
        }
        if (lane == 0) {
            if constexpr (!FMM) {
                // the further rows the front keeps, one Newton step per root
                // each, as the first pass of each row would have counted them
                if (moved) {
                    const unsigned long long ux = (unsigned long long)moved * (unsigned)R->n_r;
                    atomicAdd(&A.ctl->polish_updates, ux);
                    atomicAdd(&A.ctl->star_updates_polish, ux * (unsigned)R->n_stars);
                }
            }
            if (moved) fr.fresh = 2;   // its first pass takes the previous row from the output
            fronts_w[tf] = fr;
            state = fr.state;
            if (state != FRONT_ACTIVE) finished = (state == FRONT_FAILED && dir0 == 0) ? 2 : 1;
            if (partner >= 0) {
                p_off = fronts_w[partner].it_off;
                p_par = fronts_w[partner].par;
            }
        }
        partner = __shfl(partner, 0, 64);
        state = __shfl(state, 0, 64);
        finished = __shfl(finished, 0, 64);
        if (partner >= 0) {
            // the partner starts from the converged centre row
            p_off = __shfl(p_off, 0, 64);
            p_par = __shfl(p_par, 0, 64);
            const int cur_par = __shfl(fr.par, 0, 64);
            const int64_t my_off = __shfl(fr.it_off, 0, 64);
            const double2 *src = (cur_par ? A.iter1 : A.iter0) + my_off;
            double2 *dst = (p_par ? A.iter1 : A.iter0) + p_off;
            for (int i = lane; i < R->n_r; i += 64) dst[i] = src[i];
            push_front(q, tasks, seq, mask, partner, bpf);
        }
        if (state == FRONT_ACTIVE) push_front(q, tasks, seq, mask, tf, bpf);
        if (lane == 0) {
            if (finished) atomicAdd(&q->done, finished);
            atomicAdd(&q->progress, 1ull);
        }
    }
}

// ---------------------------------------------------------------------------
// Subchains and the autotuner
// ---------------------------------------------------------------------------

// Subchain counts S must divide m/2 (integer centre rows).  The autotuner
// prices a run with S subchains from measured costs of the kernels on
// gfx950 and picks the cheapest S.
//
// Cost of one wave's pass over a field of N stars and n_r = 2N roots, in
// SIMD cycles (issue costs measured per wave64 instruction with eight
// independent chains per lane: FP64 add/mul ~4.8, FMA ~5.3, v_rcp_f64
// ~16.6; FP32 add/mul ~2.7, FMA ~4.1, v_rcp_f32 ~8.6), fitted when the
// kernels spent ~21 instructions per star term and ~9 per root term in a
// sweep and ~22 per star term in the polish (now ~19, ~9 and ~20 with the
// eight-term reciprocal groups; S depends on the ratios of these costs,
// which moved by a few per cent):
//   FP64 Aberth sweep   114 N + 47 n_r
//   FP32 Aberth sweep    56 N + 22 n_r
//   FP64 Newton polish  120 N
// (Warm rows of MLCC_FP64_R32 take their root terms in FP32, ~40 instead of
// ~47 cycles per root; the model keeps 47, and S sweeps of measured run
// times put its choice within 1% of the best S on the workloads tried.)
// A run does, per field, u (m + S) row passes of every block (u ~ 1.03
// with the chain predictor, ~2 without; in the mixed form a row without a
// prediction takes an FP32 sweep and a polish) plus S cold starts of ~27
// sweeps.  Its time is that work over the 1024 SIMDs (fewer when fewer than
// two waves per SIMD are in flight), plus, for every round, the tail of a
// round: ~0.8 of the longest wave pass, plus ~40 us of launches and control.
// The number of rounds is ~2.1 per row of a front's m / 2S rows, plus the
// cold start.
// With multipole star sums (one field) a wave's star part is a few near
// stars and one series of order ~48: ~3,400 instructions, but bound by the
// latency of its chain of dependent loads (cell, coefficients chunk by
// chunk, near-cell ranges): measured on n10k at 4 waves per SIMD, a polish
// pass occupies ~94k SIMD cycles whatever N, and the star part of a sweep
// is priced the same; the root terms keep their cost.  In the persistent
// mixed form a multipole polish pass goes on through up to 7 further rows
// (polish_pass): a front then needs ~6x fewer passes in a row per row, which
// an S sweep of n10k (S = 5 ... 40: 299, 288, 289, 303, 311, 340 ms at S = 5,
// 8, 10, 20, 25, 40) and of the batched workload (S = 2 best) bear out.
struct TuneModel {
    double cold_sweeps = 27.0, rounds_per_row = 2.1, tail = 0.8, round_us = 40.0;
    double clock_hz = 2.4e9, simds = 1024.0;
    double fmm_star_cycles = 94000.0;
    double fmm_rows_per_pass = 6.0;
};

static double pass_cycles(int kind, double n, bool fmm)
{
    const TuneModel tm;
    const double n_r = 2.0 * n;
    if (kind == PH_F64) return (fmm ? tm.fmm_star_cycles : 114.0 * n) + 47.0 * n_r;
    if (kind == PH_F32) return (fmm ? tm.fmm_star_cycles : 56.0 * n) + 22.0 * n_r;
    return fmm ? tm.fmm_star_cycles : 120.0 * n;
}

static double predicted_seconds(const std::vector<RealHost> &reals, int64_t m, int64_t s, bool mixed,
                         int predictor, bool fmm, bool xrows)
{
    const TuneModel tm;
    double work = 0.0, blocks_all = 0.0, longest = 0.0;
    for (const RealHost &r : reals) {
        const double n = (double)r.n, blocks = std::ceil(2.0 * n / 64.0);
        double row, cold;
        if (!mixed) {
            row = (predictor > 0 ? 1.03 : 2.0) * pass_cycles(PH_F64, n, fmm);
            cold = tm.cold_sweeps * pass_cycles(PH_F64, n, fmm);
        } else {
            row = 1.02 * pass_cycles(PH_POLISH, n, fmm) +
                  (predictor > 0 ? 0.0 : pass_cycles(PH_F32, n, fmm));
            cold = tm.cold_sweeps * pass_cycles(PH_F32, n, fmm) + pass_cycles(PH_POLISH, n, fmm);
        }
        work += blocks * (row * (double)(m + s) + cold * (double)s);
        blocks_all += blocks;
        longest = std::max(longest, mixed ? pass_cycles(PH_POLISH, n, fmm)
                                          : pass_cycles(PH_F64, n, fmm));
    }
    // about half of the 2S fronts are in a full pass at any time
    const double waves = (double)s * blocks_all;
    const double simds = std::min(tm.simds, std::max(1.0, waves / 2.0));
    const double rows_per_pass = (xrows && mixed && fmm && predictor > 0) ? tm.fmm_rows_per_pass : 1.0;
    const double rounds =
        tm.rounds_per_row * (double)(m / 2) / (double)s / rows_per_pass + tm.cold_sweeps;
    return work / (simds * tm.clock_hz) +
           rounds * (tm.tail * longest / tm.clock_hz + tm.round_us * 1e-6);
}

// Picks S for every field of a call (all fields share one round clock, so a
// common S keeps their fronts in step): the divisor of m/2 with the lowest
// predicted time among those that leave every subchain at least 16 rows and
// keep the front table within MAX_FRONTS.
static int autotune_subchains(const std::vector<RealHost> &reals, int64_t m, bool mixed,
                              int predictor, bool fmm, bool persistent)
{
    const int64_t half = m / 2;
    const int64_t s_max = std::max<int64_t>(
        1, std::min<int64_t>(MAX_FRONTS / (2 * (int64_t)reals.size()), m / 16));
    double best = 1e300;
    int best_s = 1;
    for (int64_t s = 1; s <= std::min<int64_t>(half, std::min<int64_t>(s_max, 4096)); ++s) {
        if (half % s) continue;
        const double t = predicted_seconds(reals, m, s, mixed, predictor, fmm, persistent);
        if (t < best * 0.999) {
            best = t;
            best_s = (int)s;
        }
    }
    return best_s;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------

// Builds the fast-multipole grids of every field of the call: each field's
// stars binned and sorted by cell (the kernels then take the stars in that
// order), its expansions about the field centre on the host, its cells'
// local expansions on the device; one FmmArgs record per field, with
// pointers into the concatenated arrays.
static mlcc_status build_fmm(Ctx *c, int order, bool equal, std::vector<FmmArgs> &recs)
{
    const std::vector<double4> &st = c->hstars;
    const int pp = order > 0 ? order : 48;
    const int stride = (pp + 8) & ~7;
    const int n_real = (int)c->reals.size();
    struct Grid { int G; double x0, y0, w, cx, cy, R, wsum; int64_t cs_off, cell_off; };
    std::vector<Grid> grids(n_real);
    int64_t n_cs = 0, n_cells = 0;
    const int64_t n_all = (int64_t)st.size();
    std::vector<double4> sorted(n_all);
    std::vector<int32_t> starts;
    std::vector<double2> mm((size_t)n_real * 2 * (pp + 1), make_double2(0.0, 0.0));
    for (int r = 0; r < n_real; ++r) {
        const int64_t o = c->reals[r].star_off, n = c->reals[r].n;
        double xmin = st[o].x, xmax = st[o].x, ymin = st[o].y, ymax = st[o].y;
        for (int64_t i = o; i < o + n; ++i) {
            xmin = std::min(xmin, st[i].x); xmax = std::max(xmax, st[i].x);
            ymin = std::min(ymin, st[i].y); ymax = std::max(ymax, st[i].y);
        }
        Grid &g = grids[r];
        g.cx = 0.5 * (xmin + xmax);
        g.cy = 0.5 * (ymin + ymax);
        g.R = 0.0;
        g.wsum = 0.0;
        for (int64_t i = o; i < o + n; ++i) {
            g.R = std::max(g.R, std::hypot(st[i].x - g.cx, st[i].y - g.cy));
            g.wsum += equal ? 1.0 : st[i].z;
        }
        if (!(g.R > 0.0)) g.R = 1.0;
        g.R *= 1.0 + 1e-12;   // every star strictly inside the radius
        g.G = (int)std::min<double>(256.0, std::max(4.0, std::round(std::sqrt(1.7 * (double)n))));
        g.w = 4.0 * g.R / g.G;
        g.x0 = g.cx - 2.0 * g.R;
        g.y0 = g.cy - 2.0 * g.R;
        g.cs_off = n_cs;
        g.cell_off = n_cells;
        const int G = g.G;
        n_cs += (int64_t)G * G + 1;
        n_cells += (int64_t)G * G;
        // counting sort by cell; indices local to the field
        std::vector<int32_t> cell_of(n), start((size_t)G * G + 1, 0);
        for (int64_t i = 0; i < n; ++i) {
            const double4 &a = st[o + i];
            const int ix = std::min(G - 1, std::max(0, (int)std::floor((a.x - g.x0) / g.w)));
            const int iy = std::min(G - 1, std::max(0, (int)std::floor((a.y - g.y0) / g.w)));
            cell_of[i] = iy * G + ix;
            start[cell_of[i] + 1] += 1;
        }
        for (int q = 0; q < G * G; ++q) start[q + 1] += start[q];
        // sorted by cell; the fourth component carries the cell index
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            double4 a = st[o + i];
            a.w = (double)cell_of[i];
            sorted[o + fill[cell_of[i]]++] = a;
        }
        starts.insert(starts.end(), start.begin(), start.end());
        // expansions about the centre: M_k = sum w_i (z_i - c0)^k, and unit weights
        double2 *mf = mm.data() + (size_t)r * 2 * (pp + 1), *mg = mf + (pp + 1);
        for (int64_t i = o; i < o + n; ++i) {
            const double dx = st[i].x - g.cx, dy = st[i].y - g.cy, wi = equal ? 1.0 : st[i].z;
            double pr = 1.0, pi = 0.0;
            for (int k = 0; k <= pp; ++k) {
                mf[k].x += wi * pr; mf[k].y += wi * pi;
                mg[k].x += pr; mg[k].y += pi;
                const double t = pr * dx - pi * dy;
                pi = pr * dy + pi * dx;
                pr = t;
            }
        }
    }
    MLCC_TRY(c->fmm_cs.reserve(starts.size() * sizeof(int32_t)));
    MLCC_TRY(c->fmm_st.reserve(std::max<int64_t>(n_all, 1) * sizeof(double4)));
    MLCC_TRY(c->fmm_st2.reserve(std::max<int64_t>(n_all, 1) * sizeof(double2)));
    MLCC_TRY(c->fmm_cf.reserve((size_t)n_cells * stride * sizeof(double2)));
    MLCC_TRY(c->fmm_cg.reserve((size_t)n_cells * stride * sizeof(double2)));
    MLCC_TRY(c->fmm_q.reserve((size_t)n_cells * sizeof(double)));
    MLCC_TRY(c->fmm_m.reserve(mm.size() * sizeof(double2)));
    MLCC_TRY(c->fmm_args.reserve((size_t)n_real * sizeof(FmmArgs)));
    std::vector<double2> sorted2(n_all);
    for (int64_t i = 0; i < n_all; ++i) sorted2[i] = make_double2(sorted[i].x, sorted[i].y);
    MLCC_HIP(hipMemcpyAsync(c->fmm_cs.p, starts.data(), starts.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->fmm_st.p, sorted.data(), n_all * sizeof(double4),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->fmm_st2.p, sorted2.data(), n_all * sizeof(double2),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->fmm_m.p, mm.data(), mm.size() * sizeof(double2),
                            hipMemcpyHostToDevice, c->stream));
    recs.assign(n_real, FmmArgs{});
    for (int r = 0; r < n_real; ++r) {
        const Grid &g = grids[r];
        const int64_t o = c->reals[r].star_off;
        FmmArgs &M = recs[r];
        M.on = 1;
        M.G = g.G;
        M.p = pp;
        M.equal = equal;
        M.stride = stride;
        M.x0 = g.x0; M.y0 = g.y0; M.w = g.w; M.inv_w = 1.0 / g.w;
        M.cx = g.cx; M.cy = g.cy; M.R = g.R; M.wsum = g.wsum;
        M.cell_start = c->fmm_cs.as<int32_t>() + g.cs_off;
        M.fstars = c->fmm_st.as<double4>() + o;
        M.cf = c->fmm_cf.as<double2>() + g.cell_off * stride;
        M.cg = c->fmm_cg.as<double2>() + g.cell_off * stride;
        M.qfar = c->fmm_q.as<double>() + g.cell_off;
        M.mf = c->fmm_m.as<double2>() + (size_t)r * 2 * (pp + 1);
        M.mg = M.mf + (pp + 1);
        const unsigned ncell = (unsigned)((int64_t)g.G * g.G);
        hipLaunchKernelGGL(fmm_p2l, dim3(ncell), dim3(64), 0, c->stream, g.G, pp, stride, g.x0,
                           g.y0, g.w, (int32_t)equal, (int32_t)c->reals[r].n, M.fstars,
                           const_cast<double2 *>(M.cf), const_cast<double2 *>(M.cg),
                           const_cast<double *>(M.qfar));
    }
    MLCC_HIP(hipGetLastError());
    MLCC_HIP(hipMemcpyAsync(c->fmm_args.p, recs.data(), recs.size() * sizeof(FmmArgs),
                            hipMemcpyHostToDevice, c->stream));
    // host vectors must outlive the copies
    MLCC_HIP(hipStreamSynchronize(c->stream));
    return MLCC_OK;
}

mlcc_status find_critical_curves_impl(Ctx *c, const mlcc_cc_params *p, double *roots_re,
                                      double *roots_im, double *caus_re, double *caus_im,
                                      int32_t *chain_next, mlcc_cc_stats *stats)
{
    const bool mixed = p->precision == MLCC_MIXED;
    const int64_t m = p->m_steps;
    const int n_real = (int)c->reals.size();
    // one field with equal masses: (x, y) records, the mass applied once
    const bool equal = !c->batched && c->equal_mass;
    int S = p->n_subchains;
    if (S <= 0)
        S = autotune_subchains(c->reals, m, mixed, p->predictor,
                               p->star_sums == MLCC_STARS_FMM,
                               p->schedule == MLCC_SCHEDULE_PERSISTENT);
    if ((m / 2) % S) return fail(MLCC_ERR_INVALID, "n_subchains=%d must divide m/2", S);
    const int64_t L = m / S;
    const int max_cold = p->max_iter_cold > 0 ? p->max_iter_cold : 500;
    const int max_warm = p->max_iter_warm > 0 ? p->max_iter_warm : 100;
    constexpr int MAX_BATCH = 256;
    constexpr int KINDS = 3;   // timed kernels per round: FP64 sweep, FP32 sweep, polish

    // fronts, blocks and offsets of every field
    std::vector<Real> rd(n_real);
    std::vector<double> sheet_host;   // rectangular fields' sheet records
    std::vector<Front> fr;
    std::vector<int2> bmap;
    int64_t it_total = 0, bnd_total = 0, max_nr = 0;
    const int32_t warm_phase = mixed ? PH_F32 : PH_F64;
    for (int r = 0; r < n_real; ++r) {
        const RealHost &h = c->reals[r];
        const SheetPoly sp = sheet_poly(h);
        const int64_t n_r = 2 * h.n + sp.n_extra;
        if (n_r > ((int64_t)1 << 30)) return fail(MLCC_ERR_INVALID, "too many roots");
        max_nr = std::max(max_nr, n_r);
        Real &R = rd[r];
        R.star_off = h.star_off;
        R.out_off = (m + 1) * 2 * h.star_off;
        R.bnd_off = bnd_total;
        bnd_total += (int64_t)(S - 1) * n_r;
        R.n_stars = (int32_t)h.n;
        R.n_r = (int32_t)n_r;
        R.m0 = h.m0;
        R.gamma = h.gamma - sp.d0;   // a rectangular sheet's constant term joins the shear
        R.n_poly = sp.n;
        R.n_extra = sp.n_extra;
        R.sheet_off = (int64_t)sheet_host.size();
        if (sp.n > 0) {
            // d_2k, then the lens-map terms, then the extra roots' start values:
            // evenly spread on the circle through the corners (Sec. 3.2), at
            // angles 2 pi (k + 1/2) / (t - 1)
            sheet_host.insert(sheet_host.end(), sp.d, sp.d + sp.n);
            sheet_host.insert(sheet_host.end(), sp.dmap, sp.dmap + sp.n);
            for (int k = 0; k < sp.n_extra; ++k) {
                const double ang = 2.0 * M_PI * ((double)k + 0.5) / (double)sp.n_extra;
                sheet_host.push_back(sp.seed_r * std::cos(ang));
                sheet_host.push_back(sp.seed_r * std::sin(ang));
            }
        }
        R.a = 1.0 - h.kappa_s;
        R.a1 = std::fabs(R.a);
        R.sz_r = h.sum_z.x;
        R.sz_i = h.sum_z.y;
        R.sz2_r = h.sum_z2.x;
        R.sz2_i = h.sum_z2.y;
        R.M = h.mass_total;
        // rounding of the reference values 2 sum z_i and 2 sum z_i^2 (compensated
        // sums on the host, then the squares and the doubling)
        const double u_ro = 1.1102230246251565e-16;
        R.tol1 = 8.0 * u_ro * h.sum_abs_z;
        R.tol2 = 16.0 * u_ro * h.sum_abs_z2;
        R.root32 = p->precision == MLCC_FP64_R32 ? 1 : 0;
        R.restart = p->cold_restart_sweeps > 0 ? p->cold_restart_sweeps : STALL_START;
        // further rows per polish pass (persistent mixed form with the chain
        // predictor): every field with multipole sums, small fields with direct
        // ones
        R.xrows = 0;
        if (mixed && p->schedule == MLCC_SCHEDULE_PERSISTENT && p->predictor > 0) {
            if (p->star_sums == MLCC_STARS_FMM) R.xrows = FMM_XROWS;
            else if (h.n <= XROWS_DIRECT_MAX_N) R.xrows = DIRECT_XROWS;
        }
        const int bpf = (int)ceil_div(n_r, 64);
        for (int s = 0; s < S; ++s) {
            const int32_t lo = (int32_t)(s * L), hi = (int32_t)(lo + L), cen = (int32_t)(lo + L / 2);
            const int fd = (int)fr.size();
            Front d{};
            d.row = cen; d.dir = 0; d.end_row = lo; d.state = FRONT_ACTIVE;
            d.src = fd; d.partner = fd + 1; d.bnd_slot = s >= 1 ? s - 1 : -1;
            d.lo = lo; d.hi = hi;
            d.phase = warm_phase; d.mode = warm_phase; d.stamp = 4 * cen;
            d.best = 0x7fffffff;
            d.real = r;
            Front u{};
            u.row = cen + 1; u.dir = 1; u.end_row = hi; u.state = FRONT_IDLE;
            u.src = fd + 1; u.partner = -1; u.bnd_slot = -1; u.lo = lo; u.hi = hi;
            u.phase = warm_phase; u.mode = warm_phase; u.stamp = 4 * (cen + 1);
            u.real = r;
            for (Front *x : {&d, &u}) {
                x->it_off = it_total;
                it_total += n_r;
                x->blk0 = (int32_t)bmap.size();
                const int fi = (int)fr.size();
                for (int q = 0; q < bpf; ++q) bmap.push_back(make_int2(fi, q));
                fr.push_back(*x);
            }
        }
    }
    const int F = (int)fr.size();
    const int64_t nblocks = (int64_t)bmap.size();   // blocks of all fronts, in front order
    if (F > MAX_FRONTS || nblocks > 0x3fffffff)
        return fail(MLCC_ERR_INVALID, "too many fronts (%d) for one call", F);
#if MLCC_XCD_MAP
    // Launch-grid order: work group g runs on XCD g mod 8, so the blocks of
    // one front are all placed at indices of one residue, and each XCD's L2
    // holds the iterates of its own fronts only (fronts go to the least
    // loaded XCD, largest first).  Unused grid slots point at a sentinel
    // front that is never active.
    {
        constexpr int XCDS = 8;
        std::vector<int> byblocks(F);
        for (int f = 0; f < F; ++f) byblocks[f] = f;
        auto nb = [&](int f) { return ceil_div(rd[fr[f].real].n_r, 64); };
        std::stable_sort(byblocks.begin(), byblocks.end(),
                         [&](int a, int b) { return nb(a) > nb(b); });
        std::vector<std::vector<int2>> lists(XCDS);
        std::vector<int64_t> load(XCDS, 0);
        for (int f : byblocks) {
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int64_t q = 0; q < nb(f); ++q) lists[x].push_back(make_int2(f, (int)q));
            load[x] += nb(f);
        }
        const int64_t per = *std::max_element(load.begin(), load.end());
        bmap.assign((size_t)(per * XCDS), make_int2(F, 0));
        for (int x = 0; x < XCDS; ++x)
            for (size_t i = 0; i < lists[x].size(); ++i) bmap[i * XCDS + x] = lists[x][i];
    }
#endif
    const int64_t ngrid = (int64_t)bmap.size();
    {
        Front sentinel{};
        sentinel.state = FRONT_DONE;
        sentinel.dir = 1;
        fr.push_back(sentinel);
    }
    // the control kernel's groups hold whole subchains (two fronts) in LDS
    const int fronts_per_group = 4096;
    const int control_groups = (int)ceil_div(F, fronts_per_group);

    MLCC_TRY(c->iter[0].reserve((size_t)it_total * sizeof(double2)));
    MLCC_TRY(c->iter[1].reserve((size_t)it_total * sizeof(double2)));
    MLCC_TRY(c->flagrow.reserve((size_t)it_total * sizeof(int32_t)));
    MLCC_TRY(c->fronts.reserve((size_t)(F + 1) * sizeof(Front)));
    MLCC_TRY(c->counts.reserve((size_t)F * sizeof(int32_t)));
    MLCC_TRY(c->passupd.reserve((size_t)F * sizeof(int32_t)));
    MLCC_TRY(c->control.reserve(sizeof(Control)));
    MLCC_TRY(c->fmm_tally.reserve((size_t)FMM_STRIPES * FMM_STRIPE_U64 * sizeof(uint64_t)));
    MLCC_TRY(c->etab.reserve((size_t)(m + 1) * sizeof(double2)));
    MLCC_TRY(c->bnd.reserve((size_t)std::max<int64_t>(bnd_total, 1) * sizeof(double2)));
    // several rows per polish pass: row sums for the most further rows any
    // field takes
    int xrow_max = 0;
    for (const Real &R : rd) xrow_max = std::max(xrow_max, (int)R.xrows);
    const bool xrows_on = xrow_max > 0;
    MLCC_TRY(c->vieta.reserve((size_t)2 * (xrow_max + 1) * nblocks * sizeof(double4)));
    MLCC_TRY(c->vsum.reserve((size_t)2 * F * sizeof(double4)));
    if (mixed) MLCC_TRY(c->errbuf.reserve((size_t)it_total * sizeof(double)));
    MLCC_TRY(c->reals_d.reserve((size_t)n_real * sizeof(Real)));
    MLCC_TRY(c->sheet.reserve(std::max<size_t>(1, sheet_host.size()) * sizeof(double)));
    // With multipole sums the kernels take each field's stars in cell order,
    // so that the seeds z_i +- 1 of a work group's roots, and the roots grown
    // from them, share a few cells (and those cells' series) instead of 64.
    std::vector<FmmArgs> fmm_recs;
    const bool fmm_on = p->star_sums == MLCC_STARS_FMM;
    const double2 *stars2 = c->stars.as<double2>();
    const double4 *stars4 = c->stars4.as<double4>();
    if (fmm_on) {
        MLCC_TRY(build_fmm(c, p->fmm_order, equal, fmm_recs));
        stars2 = c->fmm_st2.as<double2>();
        stars4 = c->fmm_st.as<double4>();
    }
    const FmmArgs *fmm_dev = fmm_on ? c->fmm_args.as<FmmArgs>() : nullptr;
    MLCC_TRY(c->bmap.reserve((size_t)ngrid * sizeof(int2)));
    MLCC_TRY(c->workflags.reserve(2 * MAX_BATCH * sizeof(int32_t)));
    MLCC_TRY(ensure_pinned(c, 2 * (sizeof(Control) + MAX_BATCH * sizeof(int32_t))));

    // unit phase table (cos phi_j, -sin phi_j), phi_j = 2 pi j / m (host libm);
    // each field scales it by its own 1 - kappa_s
    std::vector<double2> unit(m + 1);
    for (int64_t j = 0; j <= m; ++j) {
        const double phi = (2.0 * M_PI * (double)j) / (double)m;
        unit[j] = make_double2(std::cos(phi), -std::sin(phi));
    }
    Control ctl0{};
    ctl0.active_fronts = F;
    MLCC_HIP(hipMemcpyAsync(c->etab.p, unit.data(), (m + 1) * sizeof(double2),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->fronts.p, fr.data(), (F + 1) * sizeof(Front), hipMemcpyHostToDevice,
                            c->stream));
    if (!sheet_host.empty())
        MLCC_HIP(hipMemcpyAsync(c->sheet.p, sheet_host.data(), sheet_host.size() * sizeof(double),
                                hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->reals_d.p, rd.data(), n_real * sizeof(Real), hipMemcpyHostToDevice,
                            c->stream));
    MLCC_HIP(hipMemcpyAsync(c->bmap.p, bmap.data(), ngrid * sizeof(int2), hipMemcpyHostToDevice,
                            c->stream));
    MLCC_HIP(hipMemcpyAsync(c->control.p, &ctl0, sizeof ctl0, hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemsetAsync(c->flagrow.p, 0xff, (size_t)it_total * sizeof(int32_t), c->stream));
    MLCC_HIP(hipMemsetAsync(c->counts.p, 0, F * sizeof(int32_t), c->stream));
    MLCC_HIP(hipMemsetAsync(c->fmm_tally.p, 0,
                            (size_t)FMM_STRIPES * FMM_STRIPE_U64 * sizeof(uint64_t), c->stream));
    MLCC_HIP(hipMemsetAsync(c->passupd.p, 0, F * sizeof(int32_t), c->stream));
    if (equal)
        hipLaunchKernelGGL(seed_centres<double2>, dim3((unsigned)ngrid), dim3(64), 0, c->stream,
                           stars2, c->reals_d.as<Real>(), c->fronts.as<Front>(),
                           c->bmap.as<int2>(), c->sheet.as<double>(), c->iter[0].as<double2>());
    else
        hipLaunchKernelGGL(seed_centres<double4>, dim3((unsigned)ngrid), dim3(64), 0, c->stream,
                           stars4, c->reals_d.as<Real>(), c->fronts.as<Front>(),
                           c->bmap.as<int2>(), c->sheet.as<double>(), c->iter[0].as<double2>());
    MLCC_HIP(hipGetLastError());
    // Host copies must finish before the vectors above go out of scope.
    MLCC_HIP(hipStreamSynchronize(c->stream));
    // The rounds run on the caller's stream, or, when that is the legacy null
    // stream (which cannot be captured into a graph), on a stream of the
    // context's own; the call is synchronous either way.
    hipStream_t rs = c->stream;
    if (!rs) {
        if (!c->own_stream) MLCC_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
        rs = c->own_stream;
    }

    RoundArgs<double2> A2{};
    RoundArgs<double4> A4{};
    auto fill = [&](auto &A, auto stars, const double2 *cur, double2 *nxt) {
        A.stars = stars;
        A.reals = c->reals_d.as<Real>();
        A.bmap = c->bmap.as<int2>();
        A.fronts = c->fronts.as<Front>();
        A.flagrow = c->flagrow.as<int32_t>();
        A.cur = cur;
        A.nxt = nxt;
        A.unit = c->etab.as<double2>();
        A.tol_step = p->tol_step;
        A.tol_step2 = p->tol_step * p->tol_step;
        A.tol_mu = p->tol_inv_mu;
        A.out_re = roots_re;
        A.out_im = roots_im;
        A.caus_re = caus_re;
        A.caus_im = caus_im;
        A.bnd = c->bnd.as<double2>();
        A.counts = c->counts.as<int32_t>();
        A.passupd = c->passupd.as<int32_t>();
        A.ctl = c->control.as<Control>();
        A.fmm_tally = c->fmm_tally.as<unsigned long long>();
        A.vieta = c->vieta.as<double4>();
        A.predictor = p->predictor;
        A.errbuf = mixed ? c->errbuf.as<double>() : nullptr;
        A.sheet = c->sheet.as<double>();
        A.fmm = fmm_dev;
    };
    const dim3 grid((unsigned)ngrid);
    auto launch_kind = [&](int kind, const double2 *cur, double2 *nxt) {
        // each kernel comes with and without multipole sums, so that the
        // direct kernels carry none of the multipole code's registers
        auto go = [&](auto &A, auto eq, auto fm) {
            constexpr bool E = decltype(eq)::value, M = decltype(fm)::value;
            if (kind == 0) hipLaunchKernelGGL((aberth_sweep_f64<E, M>), grid, dim3(64), 0, rs, A);
            if (kind == 1) hipLaunchKernelGGL((aberth_sweep_f32<E, M>), grid, dim3(64), 0, rs, A);
            if (kind == 2) hipLaunchKernelGGL((newton_polish_f64<E, M>), grid, dim3(64), 0, rs, A);
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        if (equal) {
            fill(A2, stars2, cur, nxt);
            if (fmm_on) go(A2, T_{}, T_{}); else go(A2, T_{}, F_{});
        } else {
            fill(A4, stars4, cur, nxt);
            if (fmm_on) go(A4, F_{}, T_{}); else go(A4, F_{}, F_{});
        }
    };

    Control *dctl = c->control.as<Control>();
    char *pin = static_cast<char *>(c->pinned);
    auto pin_ctl = [&](int slot) {
        return reinterpret_cast<Control *>(pin + slot * (sizeof(Control) + MAX_BATCH * 4));
    };
    auto pin_flags = [&](int slot) {
        return reinterpret_cast<int32_t *>(pin + slot * (sizeof(Control) + MAX_BATCH * 4) +
                                           sizeof(Control));
    };

    // event pairs: [slot][round][kind][begin, end]
    std::vector<hipEvent_t> evs;
    auto ev = [&](int slot, int i, int kind, int end) -> hipEvent_t & {
        return evs[(((size_t)slot * MAX_BATCH + i) * KINDS + kind) * 2 + end];
    };
    if (p->timing) {
        evs.resize((size_t)2 * MAX_BATCH * KINDS * 2);
        for (auto &e : evs) MLCC_HIP(hipEventCreate(&e));
    }
    hipEvent_t done_ev[2];
    MLCC_HIP(hipEventCreateWithFlags(&done_ev[0], hipEventDisableTiming));
    MLCC_HIP(hipEventCreateWithFlags(&done_ev[1], hipEventDisableTiming));
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_len = 0;
    auto cleanup = [&]() {
        for (auto &e : evs) (void)hipEventDestroy(e);
        evs.clear();
        for (auto &g : gexec)
            if (g) (void)hipGraphExecDestroy(g);
        (void)hipEventDestroy(done_ev[0]);
        (void)hipEventDestroy(done_ev[1]);
    };

    const bool persistent = p->schedule == MLCC_SCHEDULE_PERSISTENT;
    const bool use_graphs = !p->timing && !persistent;
    int parity = 0;
    int batch_len[2] = {0, 0};
    int G = 4;
    double kind_ms[KINDS] = {0.0, 0.0, 0.0};
    int64_t kind_launches[KINDS] = {0, 0, 0};
    double persistent_ms = 0.0;
    int64_t persistent_launches = 0;
    int32_t polls = 0;
    // Every front finishes within max_cold + (L/2 + 1) * (max_warm + polish
    // rounds) rounds; the extra margin covers the batches enqueued ahead of
    // the last poll.
    const int64_t launch_cap =
        (int64_t)max_cold + (L / 2 + 2) * (int64_t)(max_warm + MAX_POLISH + 2) + 4 * MAX_BATCH;
    int64_t launched = 0;
    // One round: every pass kind once over every block (blocks whose front is
    // in another phase return at once), then the control kernel.
    auto enqueue_rounds = [&](int slot, int g, bool timed) -> mlcc_status {
        for (int i = 0; i < g; ++i) {
            const double2 *cur = c->iter[parity].as<double2>();
            double2 *nxt = c->iter[parity ^ 1].as<double2>();
            for (int kind = 0; kind < (mixed ? KINDS : 1); ++kind) {
                if (timed) MLCC_HIP(hipEventRecord(ev(slot, i, kind, 0), rs));
                launch_kind(kind, cur, nxt);
                if (timed) MLCC_HIP(hipEventRecord(ev(slot, i, kind, 1), rs));
                if (kind == 2)
                    hipLaunchKernelGGL(row_sums, dim3((unsigned)F), dim3(64), 0, rs,
                                       c->fronts.as<Front>(), c->reals_d.as<Real>(),
                                       c->vieta.as<double4>(), c->vsum.as<double4>());
            }
            int32_t *wf = c->workflags.as<int32_t>() + slot * MAX_BATCH + i;
            hipLaunchKernelGGL(control_begin, dim3(1), dim3(64), 0, rs, dctl, wf);
            hipLaunchKernelGGL(aberth_control, dim3(control_groups), dim3(CONTROL_THREADS), 0,
                               rs, c->fronts.as<Front>(), c->counts.as<int32_t>(), F, dctl,
                               max_cold, max_warm, wf, c->vsum.as<double4>(),
                               c->reals_d.as<Real>(), c->etab.as<double2>(), fronts_per_group,
                               p->predictor, c->passupd.as<int32_t>());
            hipLaunchKernelGGL(control_end, dim3(1), dim3(64), 0, rs, dctl, wf);
            parity ^= 1;
        }
        MLCC_HIP(hipGetLastError());
        MLCC_HIP(hipMemcpyAsync(pin_ctl(slot), dctl, sizeof(Control), hipMemcpyDeviceToHost,
                                rs));
        MLCC_HIP(hipMemcpyAsync(pin_flags(slot), c->workflags.as<int32_t>() + slot * MAX_BATCH,
                                g * sizeof(int32_t), hipMemcpyDeviceToHost, rs));
        return MLCC_OK;
    };
    auto enqueue_batch = [&](int slot, int g) -> mlcc_status {
        if (gexec[slot]) {
            MLCC_HIP(hipGraphLaunch(gexec[slot], rs));
            g = graph_len;
        } else {
            MLCC_TRY(enqueue_rounds(slot, g, p->timing != 0));
        }
        MLCC_HIP(hipEventRecord(done_ev[slot], rs));
        batch_len[slot] = g;
        launched += g;
        return MLCC_OK;
    };
    // Without per-kernel timing the rounds of a batch are captured once per
    // slot into a hipGraph (an even number of rounds, so the ping-pong buffers
    // line up) and replayed until the fronts are done.
    auto build_graphs = [&](int g) -> mlcc_status {
        g = std::max(2, g & ~1);
        for (int slot = 0; slot < 2; ++slot) {
            hipGraph_t graph = nullptr;
            const int saved = parity;
            parity = 0;
            MLCC_HIP(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
            mlcc_status s = enqueue_rounds(slot, g, false);
            hipError_t e = hipStreamEndCapture(rs, &graph);
            parity = saved;
            if (s != MLCC_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            MLCC_HIP(e);
            e = hipGraphInstantiate(&gexec[slot], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            MLCC_HIP(e);
        }
        graph_len = g;
        return MLCC_OK;
    };
    auto harvest = [&](int slot) {
        // live bits per round: 1 << phase of every front that was active
        const int kind_phase[KINDS] = {PH_F64, PH_F32, PH_POLISH};
        for (int i = 0; i < batch_len[slot]; ++i) {
            const int32_t live = pin_flags(slot)[i];
            for (int kind = 0; kind < KINDS; ++kind) {
                if (!(live & (1 << kind_phase[kind]))) continue;
                kind_launches[kind] += 1;
                if (p->timing && !gexec[slot]) {
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, ev(slot, i, kind, 0), ev(slot, i, kind, 1));
                    kind_ms[kind] += ms;
                }
            }
        }
    };

    // The persistent scheduler: one launch, fronts advance independently.
    auto run_persistent = [&]() -> mlcc_status {
        int64_t cap = 1024;
        while (cap < 2 * nblocks) cap <<= 1;
        const size_t o_tasks = (sizeof(PQueue) + 255) & ~(size_t)255;
        const size_t o_seq = o_tasks + (size_t)cap * sizeof(int2);
        const size_t o_fdone = o_seq + (size_t)cap * SEQ_STRIDE * sizeof(unsigned long long);
        const size_t o_xrows = o_fdone + (((size_t)F * sizeof(int32_t) + 255) & ~(size_t)255);
        MLCC_TRY(c->pq.reserve(o_xrows + (size_t)F * sizeof(int32_t)));
        char *base = static_cast<char *>(c->pq.p);
        PQueue *dq = reinterpret_cast<PQueue *>(base);
        int2 *dtasks = reinterpret_cast<int2 *>(base + o_tasks);
        unsigned long long *dseq = reinterpret_cast<unsigned long long *>(base + o_seq);
        int32_t *dfdone = reinterpret_cast<int32_t *>(base + o_fdone);
        int32_t *dxrows = reinterpret_cast<int32_t *>(base + o_xrows);
        std::vector<int32_t> xr0((size_t)F, 0);
        for (int f = 0; f < F; ++f) xr0[f] = rd[fr[f].real].xrows;
        std::vector<int2> t0;
        for (int f = 0; f < F; ++f) {
            if (fr[f].state != FRONT_ACTIVE) continue;
            for (int64_t qb = 0; qb < ceil_div(rd[fr[f].real].n_r, 64); ++qb)
                t0.push_back(make_int2(f, (int)qb));
        }
        std::vector<unsigned long long> s0(t0.size() * SEQ_STRIDE, 0ull);
        for (size_t i = 0; i < t0.size(); ++i) s0[i * SEQ_STRIDE] = i + 1;
        PQueue hq{};
        hq.tail = (unsigned long long)t0.size();
        MLCC_HIP(hipMemsetAsync(base, 0, o_fdone + (size_t)F * sizeof(int32_t), rs));
        MLCC_HIP(hipMemcpyAsync(dq, &hq, sizeof hq, hipMemcpyHostToDevice, rs));
        MLCC_HIP(hipMemcpyAsync(dtasks, t0.data(), t0.size() * sizeof(int2), hipMemcpyHostToDevice,
                                rs));
        MLCC_HIP(hipMemcpyAsync(dseq, s0.data(), s0.size() * sizeof(unsigned long long),
                                hipMemcpyHostToDevice, rs));
        if (xrows_on)
            MLCC_HIP(hipMemcpyAsync(dxrows, xr0.data(), xr0.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, rs));
        auto set_xrows = [&](auto &A) {
            A.xrows = xrows_on ? dxrows : nullptr;
            A.xrow_max = xrow_max;
            A.nvslots = (int32_t)nblocks;
        };
        int cus = 0, per_cu = 0, clock_khz = 0;
        MLCC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
        MLCC_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, c->device));
        const void *kfn =
            equal ? (fmm_on ? reinterpret_cast<const void *>(&aberth_persistent<true, true>)
                            : reinterpret_cast<const void *>(&aberth_persistent<true, false>))
                  : (fmm_on ? reinterpret_cast<const void *>(&aberth_persistent<false, true>)
                            : reinterpret_cast<const void *>(&aberth_persistent<false, false>));
        MLCC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 64, 0));
        if (cus < 1 || per_cu < 1 || clock_khz < 1)
            return fail(MLCC_ERR_HIP, "cannot size the persistent launch");
        const unsigned workers = (unsigned)(cus * per_cu);
        // a worker gives up after watchdog_ms (default 5 s) in which no pass
        // finished anywhere
        const unsigned long long stall =
            (unsigned long long)clock_khz * (unsigned long long)(p->watchdog_ms > 0 ? p->watchdog_ms : 5000);
        const double2 *cur0 = c->iter[0].as<double2>();
        // The one launch is captured into a hipGraph (a single kernel node; the
        // queue and counters above are set by copies outside it) and run from
        // the graph.
        auto launch = [&]() {
            if (equal) {
                fill(A2, stars2, cur0, c->iter[1].as<double2>());
                set_xrows(A2);
                A2.persistent = 1;
                A2.iter0 = c->iter[0].as<double2>();
                A2.iter1 = c->iter[1].as<double2>();
                if (fmm_on)
                    hipLaunchKernelGGL((aberth_persistent<true, true>), dim3(workers), dim3(64), 0,
                                       rs, A2, c->fronts.as<Front>(), dq, dtasks, dseq,
                                       (unsigned long long)(cap - 1), dfdone, F, max_cold, max_warm,
                                       stall);
                else
                    hipLaunchKernelGGL((aberth_persistent<true, false>), dim3(workers), dim3(64), 0,
                                       rs, A2, c->fronts.as<Front>(), dq, dtasks, dseq,
                                       (unsigned long long)(cap - 1), dfdone, F, max_cold, max_warm,
                                       stall);
            } else {
                fill(A4, stars4, cur0, c->iter[1].as<double2>());
                set_xrows(A4);
                A4.persistent = 1;
                A4.iter0 = c->iter[0].as<double2>();
                A4.iter1 = c->iter[1].as<double2>();
                if (fmm_on)
                    hipLaunchKernelGGL((aberth_persistent<false, true>), dim3(workers), dim3(64), 0,
                                       rs, A4, c->fronts.as<Front>(), dq, dtasks, dseq,
                                       (unsigned long long)(cap - 1), dfdone, F, max_cold, max_warm,
                                       stall);
                else
                    hipLaunchKernelGGL((aberth_persistent<false, false>), dim3(workers), dim3(64), 0,
                                       rs, A4, c->fronts.as<Front>(), dq, dtasks, dseq,
                                       (unsigned long long)(cap - 1), dfdone, F, max_cold, max_warm,
                                       stall);
            }
        };
        hipGraph_t graph = nullptr;
        hipGraphExec_t gx = nullptr;
        MLCC_HIP(hipStreamBeginCapture(rs, hipStreamCaptureModeThreadLocal));
        launch();
        const hipError_t le = hipGetLastError();
        hipError_t e = hipStreamEndCapture(rs, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            MLCC_HIP(le);
            MLCC_HIP(e);
        }
        e = hipGraphInstantiate(&gx, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        MLCC_HIP(e);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (p->timing) {
            MLCC_HIP(hipEventCreate(&e0));
            MLCC_HIP(hipEventCreate(&e1));
            MLCC_HIP(hipEventRecord(e0, rs));
        }
        e = hipGraphLaunch(gx, rs);
        if (e == hipSuccess && p->timing) e = hipEventRecord(e1, rs);
        if (e == hipSuccess) e = hipStreamSynchronize(rs);
        (void)hipGraphExecDestroy(gx);
        MLCC_HIP(e);
        if (p->timing) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            persistent_ms = ms;
        }
        persistent_launches = 1;
        MLCC_HIP(hipMemcpy(&hq, dq, sizeof hq, hipMemcpyDeviceToHost));
        if (hq.abort)
            return fail(MLCC_ERR_HIP, "persistent scheduler: no pass finished for %d ms "
                                      "(%d of %d fronts done)",
                        p->watchdog_ms > 0 ? p->watchdog_ms : 5000, hq.done, F);
        return MLCC_OK;
    };

    mlcc_status st = MLCC_OK;
    int slot = 0;
    auto t_last = std::chrono::steady_clock::now();
    if (persistent) st = run_persistent();
    else st = enqueue_batch(slot, G);
    while (!persistent && st == MLCC_OK) {
        // keep one batch queued behind the one being polled
        const int next = slot ^ 1;
        if (use_graphs && !gexec[0] && polls == 1 && parity == 0) {
            // G now holds the batch length that takes ~4 ms
            st = build_graphs(std::min(G, 64));
            if (st != MLCC_OK) break;
        }
        st = enqueue_batch(next, G);
        if (st != MLCC_OK) break;
        if (hipEventSynchronize(done_ev[slot]) != hipSuccess) {
            st = fail(MLCC_ERR_HIP, "sweep batch failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        ++polls;
        const Control h = *pin_ctl(slot);
        harvest(slot);
        if (h.active_fronts == 0) {
            // drain the batch queued ahead (it found nothing to do)
            if (hipEventSynchronize(done_ev[next]) != hipSuccess) {
                st = fail(MLCC_ERR_HIP, "sweep batch failed");
                break;
            }
            harvest(next);
            break;
        }
        if (launched > launch_cap) {
            st = fail(MLCC_ERR_HIP, "root finder exceeded %lld rounds", (long long)launch_cap);
            break;
        }
        // poll roughly every 4 ms of GPU work
        auto now = std::chrono::steady_clock::now();
        const double dt = std::chrono::duration<double, std::milli>(now - t_last).count();
        t_last = now;
        const double per = dt / std::max(1, batch_len[slot]);
        G = (int)std::min<double>(MAX_BATCH, std::max<double>(2.0, 4.0 / std::max(per, 1e-3)));
        G &= ~1;   // even batches keep the ping-pong parity at 0 between batches
        slot = next;
    }
    (void)hipStreamSynchronize(rs);
    cleanup();
    if (st != MLCC_OK) return st;

    Control h{};
    MLCC_HIP(hipMemcpyAsync(&h, dctl, sizeof h, hipMemcpyDeviceToHost, c->stream));
    std::vector<uint64_t> tally((size_t)FMM_STRIPES * FMM_STRIPE_U64);
    MLCC_HIP(hipMemcpyAsync(tally.data(), c->fmm_tally.p, tally.size() * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, c->stream));
    std::vector<Front> fin(F);
    MLCC_HIP(hipMemcpyAsync(fin.data(), c->fronts.p, F * sizeof(Front), hipMemcpyDeviceToHost,
                            c->stream));
    MLCC_HIP(hipStreamSynchronize(c->stream));
    // the multipole tallies, summed over their copies
    uint64_t ft[9] = {};
    for (int q = 0; q < FMM_STRIPES; ++q)
        for (int v = 0; v < 9; ++v) ft[v] += tally[(size_t)q * FMM_STRIPE_U64 + v];
    const uint64_t fmm_near = ft[FMM_T_F64], fmm_far[2] = {ft[FMM_T_F64 + 1], ft[FMM_T_F64 + 2]};
    const uint64_t fmm_near_polish = ft[FMM_T_POLISH],
                   fmm_far_polish[2] = {ft[FMM_T_POLISH + 1], ft[FMM_T_POLISH + 2]};
    const uint64_t fmm_near_f32 = ft[FMM_T_F32],
                   fmm_far_f32[2] = {ft[FMM_T_F32 + 1], ft[FMM_T_F32 + 2]};

    mlcc_status result = MLCC_OK;
    double maxdist = 0.0;
    if (h.failed_rows > 0) {
        result = fail(MLCC_ERR_NOT_CONVERGED, "%d rows hit the sweep cap (%lld roots unconverged)",
                      h.failed_rows, (long long)h.unconverged);
    } else {
        // join subchains: pair each duplicate boundary row with the stored
        // copy, compose the pairings into global labels, relabel the blocks;
        // then pair row m with row 0 for chain_next
        std::vector<PairJob> jobs;
        int64_t perm_total = 0;
        for (int r = 0; r < n_real; ++r) perm_total += (int64_t)S * rd[r].n_r;
        MLCC_TRY(c->perm.reserve((size_t)std::max<int64_t>(perm_total, 1) * sizeof(int32_t)));
        int32_t *perm = c->perm.as<int32_t>();
        std::vector<int64_t> perm_off(n_real);
        int64_t po = 0;
        for (int r = 0; r < n_real; ++r) {
            perm_off[r] = po;
            const int64_t n_r = rd[r].n_r;
            double *ore = roots_re + rd[r].out_off, *oim = roots_im + rd[r].out_off;
            for (int s = 1; s < S; ++s) {
                PairJob j{};
                j.a2 = c->bnd.as<double2>() + rd[r].bnd_off + (int64_t)(s - 1) * n_r;
                j.b_re = ore + s * L * n_r;
                j.b_im = oim + s * L * n_r;
                j.perm = perm + po + s * n_r;
                j.n = n_r;
                jobs.push_back(j);
            }
            po += (int64_t)S * n_r;
        }
        double md = 0.0;
        MLCC_TRY(pair_all(c, jobs, 1e-6, &md));
        maxdist = std::max(maxdist, md);
        if (S > 1) {
            std::vector<int32_t> hp((size_t)perm_total), lab((size_t)perm_total);
            MLCC_HIP(hipMemcpyAsync(hp.data(), perm, (size_t)perm_total * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, c->stream));
            MLCC_HIP(hipStreamSynchronize(c->stream));
            for (int r = 0; r < n_real; ++r) {
                const int64_t n_r = rd[r].n_r, b = perm_off[r];
                for (int64_t k = 0; k < n_r; ++k) lab[b + k] = (int32_t)k;
                for (int s = 1; s < S; ++s)
                    for (int64_t k = 0; k < n_r; ++k)
                        lab[b + s * n_r + k] = lab[b + (s - 1) * n_r + hp[b + s * n_r + k]];
            }
            MLCC_HIP(hipMemcpyAsync(perm, lab.data(), (size_t)perm_total * sizeof(int32_t),
                                    hipMemcpyHostToDevice, c->stream));
            std::vector<RelabelJob> rj;
            for (int r = 0; r < n_real; ++r) {
                const int64_t n_r = rd[r].n_r;
                for (int s = 1; s < S; ++s) {
                    const int32_t *lb = perm + perm_off[r] + s * n_r;
                    rj.push_back(RelabelJob{roots_re + rd[r].out_off, roots_im + rd[r].out_off,
                                            n_r, s * L + 1, (s + 1) * L + 1, lb});
                    if (caus_re)
                        rj.push_back(RelabelJob{caus_re + rd[r].out_off, caus_im + rd[r].out_off,
                                                n_r, s * L + 1, (s + 1) * L + 1, lb});
                }
            }
            MLCC_TRY(relabel_all(c, rj));
            MLCC_HIP(hipStreamSynchronize(c->stream));
        }
        if (chain_next) {
            jobs.clear();
            for (int r = 0; r < n_real; ++r) {
                const int64_t n_r = rd[r].n_r;
                double *ore = roots_re + rd[r].out_off, *oim = roots_im + rd[r].out_off;
                PairJob j{};
                j.a_re = ore + m * n_r;
                j.a_im = oim + m * n_r;
                j.b_re = ore;
                j.b_im = oim;
                j.perm = chain_next + 2 * c->reals[r].star_off;
                j.n = n_r;
                jobs.push_back(j);
            }
            MLCC_TRY(pair_all(c, jobs, 1e-6, &md));
            maxdist = std::max(maxdist, md);
        }
        MLCC_HIP(hipStreamSynchronize(c->stream));
    }

    if (stats) {
        *stats = mlcc_cc_stats{};
        if (persistent) {   // no global rounds: the longest chain of passes of one front
            int64_t mp = 0;
            for (const Front &x : fin) mp = std::max<int64_t>(mp, x.npass);
            stats->sweeps = mp;
        } else {
            stats->sweeps = h.live_sweeps;
        }
        stats->root_updates = (int64_t)h.updates;
        stats->root_updates_f32 = (int64_t)h.updates_f32;
        stats->polish_updates = (int64_t)h.polish_updates;
        stats->unconverged = h.unconverged;
        stats->rows_capped = h.failed_rows;
        stats->cold_restarts = h.cold_restarts;
        stats->rows_fallback = h.rows_fallback;
        stats->n_subchains = S;
        int32_t mw = 0, mc = 0;
        for (const Front &x : fin) {
            mw = std::max(mw, x.max_warm);
            mc = std::max(mc, x.cold);
        }
        stats->max_row_sweeps = mw;
        stats->cold_sweeps = mc;
        stats->polls = polls;
        stats->match_maxdist = maxdist;
        stats->sweep_ms = kind_ms[0];
        stats->sweep_f32_ms = kind_ms[1];
        stats->polish_ms = kind_ms[2];
        stats->sweep_launches = kind_launches[0];
        stats->sweep_f32_launches = kind_launches[1];
        stats->polish_launches = kind_launches[2];
        stats->persistent_ms = persistent_ms;
        stats->persistent_launches = persistent_launches;
        // algorithmic FLOP of one update of a root of a field of N stars
        // (FMA = 2, add/mul/reciprocal = 1): 29 per star term (difference,
        // |d|^2, reciprocal, u, u^2, u^3 and their sums) and 10 per root
        // term, 29 N + 10 (2N - 1) for an Aberth update, 29 N for a polish
        // update (star terms only); the device counts updates and
        // updates x N, which gives the sums over mixed field sizes
        // star terms in FP64; root terms in FP64 except in fast-root passes
        // With fast-multipole star sums (one field), an update that took
        // them has its near stars' terms at 29 FLOP each and one evaluation
        // of the cell's series of order p in place of the other N - near
        // terms: Horner's rule for f, f' and f'' together takes 26 FLOP per
        // order (the unit-weight series of unequal masses 8 more in the
        // sweeps), plus ~20 for the cell and the sums.  The outside-grid
        // expansion, rarely taken, is counted the same.
        // The FP32 sweeps take such sums in FP64: their star terms move from
        // the FP32 count to the FP64 one.
        double star64 = (double)h.star_updates, starpol = (double)h.star_updates_polish;
        double far64 = 0.0, farpol = 0.0, star32_off = 0.0;
        if (fmm_on) {
            const double pf = (double)fmm_recs[0].p;
            const double unit_g = equal ? 0.0 : 8.0 * pf;
            far64 = (double)fmm_far[0] * (26.0 * pf + 20.0 + unit_g) +
                    (double)fmm_far_f32[0] * (26.0 * pf + 20.0 + unit_g) +
                    29.0 * (double)fmm_near_f32;
            farpol = (double)fmm_far_polish[0] * (26.0 * pf + 20.0);
            star64 += (double)fmm_near - (double)fmm_far[1];
            starpol += (double)fmm_near_polish - (double)fmm_far_polish[1];
            star32_off = 29.0 * (double)fmm_far_f32[1];
            stats->fmm_near_terms = (int64_t)(fmm_near + fmm_near_polish + fmm_near_f32);
            stats->fmm_far_evals =
                (int64_t)(fmm_far[0] + fmm_far_polish[0] + fmm_far_f32[0]);
        }
        stats->algorithmic_flop = 29.0 * star64 + far64 +
                                  20.0 * (double)(h.star_updates - h.star_updates_fast) -
                                  10.0 * (double)(h.updates - h.updates_fast);
        stats->algorithmic_flop_sweep_roots =
            20.0 * (double)h.star_updates_fast - 10.0 * (double)h.updates_fast;
        if (n_real == 1) {   // a rectangular field's extra roots: 10 FLOP per root term each
            const double ex = 10.0 * (double)sheet_poly(c->reals[0]).n_extra;
            stats->algorithmic_flop += ex * (double)(h.updates - h.updates_fast);
            stats->algorithmic_flop_sweep_roots += ex * (double)h.updates_fast;
        }
        stats->algorithmic_flop_f32 =
            49.0 * (double)h.star_updates_f32 - 10.0 * (double)h.updates_f32 - star32_off;
        stats->algorithmic_flop_polish = 29.0 * starpol + farpol;
    }
    return result;
}

} // namespace mlcc
