// Critical-curve root finder: parallel Aberth-Ehrlich sweeps (Sec. 3.2)
// over the phase grid, warm-started along phi and grown centre-out in
// subchains (Sec. 4.3).
//
// Layout and scheduling (gfx950):
//  * One lane per root, one 64-lane wavefront per work-group.  Each
//    work-group owns 64 consecutive roots of one "front" (a growing end of a
//    subchain).  Star positions and the other roots stream through LDS in
//    tiles and are read back as wave-uniform broadcasts.
//  * A block with only a few unflagged roots left (the last sweep of a row)
//    works on them one at a time with the whole wave, so such sweeps cost
//    ~1/64 of a full one instead of the same latency.
//  * Roots flagged converged are mapped to the caustic in the same kernel.
//  * Jacobi double buffering: a sweep reads iterate `cur` and writes `nxt`;
//    the host alternates the two on every launch.  A root flagged converged
//    is copied forward unchanged.
//  * A single-work-group control kernel after every sweep advances the
//    fronts whose rows have converged (device-side, so the host only polls
//    a small status block every few launches, one batch ahead).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "mlcc_internal.h"

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

// The hardware estimate v_rcp_f64 has relative error ~2^-24.4.  Star terms
// take 2 refinement steps (fully accurate): F itself must be exact to the
// last bits.  The root-root sum R only enters the step as F * (2 S1 - R);
// that factor vanishes at a zero of F, so an error in R cannot move a
// converged root, it only perturbs the path at second order in the error
// of the iterate.  R therefore uses the unrefined estimate.
constexpr int RCP_STAR = 2;
constexpr int RCP_ROOT = 0;

// Streams the records p[0..n) through body(i, p[i]) for a one-wave work
// group.  Tiles of 64 records (one per lane) are fetched with coalesced
// vector loads, the next tile while the current one is consumed, parked in
// LDS, and read back with one wave-uniform (broadcast) LDS read per record.
// Vector loads retire in order, so waiting for the older tile never waits
// for the prefetch behind it.  Indices past n-1 are clamped on load, so
// nothing outside the array is read.  `lds` holds two tiles.
template <class T, class Body>
__device__ __forceinline__ void stream_tiles(const T *__restrict__ p, int n, T *lds, Body &&body)
{
    if (n <= 0) return;
    const int lane = threadIdx.x;
    const int ntiles = (n + 63) >> 6;
    T reg = p[min(lane, n - 1)];
    for (int t = 0; t < ntiles; ++t) {
        T *buf = lds + ((t & 1) << 6);
        buf[lane] = reg;
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
    }
    __syncthreads();
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

// Running sums for one root z, u_i = 1/(z - z_i):
//   s1 = sum u_i                (for P'/P = F'/F + 2 s1)
//   s0 = sum m_i u_i            (lens mapping; equals m0 s1 for equal masses)
//   s2 = sum m_i u_i^2          (F = gamma + s2 - (1 - kappa_s) e^{-i phi})
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
__device__ __forceinline__ void add_star(Sums &S, double zr, double zi, const T &s)
{
    const double dx = zr - s.x;
    const double dy = zi - s.y;
    const double inv = rcp_refined<RCP_STAR>(fma(dx, dx, dy * dy));
    // u = ux - i uy = conj(d) / |d|^2
    const double ux = dx * inv;
    const double uy = dy * inv;
    S.s1r += ux;
    S.s1i -= uy;
    // u^2 = vx + i vy
    const double vx = fma(ux, ux, -uy * uy);
    const double vy = -2.0 * ux * uy;
    // u^3 = u^2 u
    const double tx = fma(vx, ux, vy * uy);
    const double ty = fma(vy, ux, -vx * uy);
    if (EQUAL) {
        S.s2r += vx;
        S.s2i += vy;
        S.s3r += tx;
        S.s3i += ty;
    } else {
        const double mi = StarRec<EQUAL>::mass(s);
        S.s0r = fma(mi, ux, S.s0r);
        S.s0i = fma(-mi, uy, S.s0i);
        S.s2r = fma(mi, vx, S.s2r);
        S.s2i = fma(mi, vy, S.s2i);
        S.s3r = fma(mi, tx, S.s3r);
        S.s3i = fma(mi, ty, S.s3i);
    }
}

__device__ __forceinline__ void add_root(Sums &S, double zr, double zi, const double2 &o)
{
    const double dx = zr - o.x, dy = zi - o.y;
    const double inv = rcp_refined<RCP_ROOT>(fma(dx, dx, dy * dy));
    S.Rr = fma(dx, inv, S.Rr);
    S.Ri = fma(-dy, inv, S.Ri);
}

__device__ __forceinline__ void wave_sum(double &v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
}

struct Update {
    double zr, zi;   // new iterate
    double wr, wi;   // its image under the lens map
    bool flag;       // converged
};

// One Aberth-Ehrlich update from the sums at z (Sec. 3.2), the convergence
// test of the Sec. 3.2 footnote with the App. C bound on |1/mu|, and the
// lens map at the new iterate.  The map reuses the sums: with
// z' = z - D, sum m_i/(z' - z_i) = s0 + D s2 + D^2 s3 + O(D^3 sum m_i u_i^4),
// and D is below the convergence cutoffs once a root is flagged.
template <bool EQUAL>
__device__ __forceinline__ Update finish(Sums S, double zr, double zi, double m0, double2 e,
                                         double gamma, double a, double a1, double tol_step2,
                                         double tol_mu, int k)
{
    if (EQUAL) {   // every mass equals m0: the sums above left it out
        S.s0r = m0 * S.s1r;
        S.s0i = m0 * S.s1i;
        S.s2r *= m0;
        S.s2i *= m0;
        S.s3r *= m0;
        S.s3i *= m0;
    }
    // F = gamma + S2 - (1 - kappa_s) e^{-i phi}, F' = -2 S3
    const double Fr = gamma + S.s2r - e.x, Fi = S.s2i - e.y;
    const double Fpr = -2.0 * S.s3r, Fpi = -2.0 * S.s3i;
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
    if (!isfinite(u.zr) || !isfinite(u.zi)) {
        // the iterate hit a star or two roots met: nudge it off, keep iterating
        u.zr = zr + 1e-7 * (1 + (k & 7));
        u.zi = zi + 1e-7 * (1 + (k >> 3 & 7));
        u.flag = false;
    }
    // T = s0 + D s2 + D^2 s3 with D = step
    const double d2r = stepr * stepr - stepi * stepi, d2i = 2.0 * stepr * stepi;
    const double Tr = S.s0r + (stepr * S.s2r - stepi * S.s2i) + (d2r * S.s3r - d2i * S.s3i);
    const double Ti = S.s0i + (stepr * S.s2i + stepi * S.s2r) + (d2r * S.s3i + d2i * S.s3r);
    // w = (1 - kappa_s) z' + gamma conj(z') - conj(T)
    u.wr = fma(a, u.zr, gamma * u.zr) - Tr;
    u.wi = fma(a, u.zi, -gamma * u.zi) + Ti;
    return u;
}

// Blocks with at most this many unflagged roots take the cooperative path.
constexpr int SPARSE_MAX = 16;

template <bool EQUAL>
__global__ void __launch_bounds__(64)
aberth_sweep_f64(const typename StarRec<EQUAL>::T *__restrict__ stars, double m0, int32_t n_stars,
                 const double2 *__restrict__ cur, double2 *__restrict__ nxt,
                 int32_t *__restrict__ flagrow, const Front *__restrict__ fronts,
                 const double2 *__restrict__ etab, double gamma, double a, double a1,
                 double tol_step2, double tol_mu, int32_t n_r, int32_t blocks_per_front,
                 double *__restrict__ out_re, double *__restrict__ out_im,
                 double *__restrict__ caus_re, double *__restrict__ caus_im,
                 double2 *__restrict__ bnd, int32_t *__restrict__ counts,
                 unsigned long long *__restrict__ updates)
{
    using T = typename StarRec<EQUAL>::T;
    __shared__ double4 tiles[128];   // two tiles of up to 32-byte records
    const int f = blockIdx.x / blocks_per_front;
    const int q = blockIdx.x - f * blocks_per_front;
    const int state = fronts[f].state;
    if (state != FRONT_ACTIVE) return;
    const int row = fronts[f].row;
    const int src = fronts[f].src;
    const int lane = threadIdx.x;
    const int64_t base_f = (int64_t)f * n_r;
    const double2 *__restrict__ zsrc = cur + (int64_t)src * n_r;
    const int k0 = q * 64;
    const int k = k0 + lane;
    const bool valid = k < n_r;
    double zr = 0.0, zi = 0.0;
    bool act = false;
    if (valid) {
        const double2 z = zsrc[k];
        zr = z.x;
        zi = z.y;
        act = flagrow[base_f + k] != row;
    }
    const unsigned long long amask = __ballot(act);
    const int n_act = __popcll(amask);
    if (valid && !act) nxt[base_f + k] = make_double2(zr, zi);   // carried forward
    if (n_act == 0) return;

    const double2 e = etab[row];
    const bool boundary = fronts[f].bnd_slot >= 0 && row == fronts[f].end_row;
    double2 *__restrict__ bnd_row = bnd + (int64_t)max(fronts[f].bnd_slot, 0) * n_r;
    auto store = [&](int kk, const Update &u) {
        nxt[base_f + kk] = make_double2(u.zr, u.zi);
        if (!u.flag) return;
        flagrow[base_f + kk] = row;
        if (boundary) {
            bnd_row[kk] = make_double2(u.zr, u.zi);
        } else {
            const int64_t o = (int64_t)row * n_r + kk;
            out_re[o] = u.zr;
            out_im[o] = u.zi;
            if (caus_re) {
                caus_re[o] = u.wr;
                caus_im[o] = u.wi;
            }
        }
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
            const Update u = finish<EQUAL>(S, xk, yk, m0, e, gamma, a, a1, tol_step2, tol_mu, kk);
            if (lane == l) store(kk, u);
            n_after += u.flag ? 0 : 1;
        }
    } else {
        Sums S;
        zero(S);
        stream_tiles(stars, n_stars, reinterpret_cast<T *>(tiles),
                     [&](int, const T &s) { add_star<EQUAL>(S, zr, zi, s); });
        double2 *rtiles = reinterpret_cast<double2 *>(tiles);
        auto other = [&](int, const double2 &o) { add_root(S, zr, zi, o); };
        const int own_hi = min(k0 + 64, n_r);
        stream_tiles(zsrc, k0, rtiles, other);
        stream_tiles(zsrc + k0, own_hi - k0, rtiles, [&](int j, const double2 &o) {
            Sums T2 = S;
            add_root(T2, zr, zi, o);
            const bool self = j == lane;
            S.Rr = self ? S.Rr : T2.Rr;
            S.Ri = self ? S.Ri : T2.Ri;
        });
        stream_tiles(zsrc + own_hi, n_r - own_hi, rtiles, other);
        const Update u = finish<EQUAL>(S, zr, zi, m0, e, gamma, a, a1, tol_step2, tol_mu, k);
        if (act) store(k, u);
        n_after = __popcll(__ballot(act && !u.flag));
    }
    if (lane == 0) {
        if (n_after) atomicAdd(&counts[f], n_after);
        atomicAdd(updates, (unsigned long long)n_act);
    }
}

// Cold-start seeds at the centre row of each subchain: root 2i <- z_i + 1,
// root 2i+1 <- z_i - 1 (Sec. 3.2).
__global__ void seed_centres(const double2 *__restrict__ stars, int32_t n_r, int32_t n_sub,
                             double2 *__restrict__ iter)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_sub * n_r) return;
    const int s = (int)(t / n_r);
    const int k = (int)(t - (int64_t)s * n_r);
    const double2 z = stars[k >> 1];
    iter[(int64_t)(2 * s) * n_r + k] = make_double2(z.x + ((k & 1) ? -1.0 : 1.0), z.y);
}

constexpr int CONTROL_THREADS = 256;
constexpr int MAX_FRONTS = 4096;

// Advances every front whose row converged in the sweep just run: a cold
// start at a subchain centre hands the upward half to its partner front and
// turns downward itself; a warm row moves one row on, or finishes at its end
// row.  A front that reaches its sweep cap stops and is counted as failed,
// together with a partner it can no longer start.
__global__ void __launch_bounds__(CONTROL_THREADS)
aberth_control(Front *__restrict__ fronts, int32_t *__restrict__ counts, int32_t n_fronts,
               Control *__restrict__ ctl, int32_t max_cold, int32_t max_warm,
               int32_t *__restrict__ workflag)
{
    __shared__ int32_t st[MAX_FRONTS];
    __shared__ int32_t s_active, s_live;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_active = 0;
        s_live = 0;
    }
    for (int f = tid; f < n_fronts; f += CONTROL_THREADS) st[f] = fronts[f].state;
    __syncthreads();
    for (int f = tid; f < n_fronts; f += CONTROL_THREADS) {
        if (st[f] != FRONT_ACTIVE) continue;
        atomicOr(&s_live, 1);
        Front fr = fronts[f];
        const int32_t c = counts[f];
        counts[f] = 0;
        fr.src = f;
        if (c == 0) {
            if (fr.dir == 0) {
                fr.cold = fr.sweeps + 1;
                const int p = fr.partner;
                const int centre = fr.row;
                Front pr = fronts[p];
                pr.state = FRONT_ACTIVE;
                pr.row = centre + 1;
                pr.dir = 1;
                pr.src = f;   // first sweep reads the converged centre row
                pr.sweeps = 0;
                fronts[p] = pr;
                st[p] = FRONT_ACTIVE;
                fr.dir = -1;
                fr.row = centre - 1;
                fr.sweeps = 0;
            } else {
                fr.max_warm = max(fr.max_warm, fr.sweeps + 1);
                if (fr.row == fr.end_row) {
                    fr.state = FRONT_DONE;
                    st[f] = FRONT_DONE;
                } else {
                    fr.row += fr.dir;
                    fr.sweeps = 0;
                }
            }
        } else {
            fr.sweeps += 1;
            if (fr.sweeps >= (fr.dir == 0 ? max_cold : max_warm)) {
                fr.state = FRONT_FAILED;
                st[f] = FRONT_FAILED;
                atomicAdd(&ctl->failed_rows, 1);
                atomicAdd((unsigned long long *)&ctl->unconverged, (unsigned long long)c);
                if (fr.dir == 0) {
                    fronts[fr.partner].state = FRONT_FAILED;
                    st[fr.partner] = FRONT_FAILED;
                }
            }
        }
        fronts[f] = fr;
    }
    __syncthreads();
    int mine = 0;
    for (int f = tid; f < n_fronts; f += CONTROL_THREADS)
        mine += (st[f] == FRONT_ACTIVE || st[f] == FRONT_IDLE);
    if (mine) atomicAdd(&s_active, mine);
    __syncthreads();
    if (tid == 0) {
        ctl->active_fronts = s_active;
        if (s_live) ctl->live_sweeps += 1;
        *workflag = s_live;
    }
}

// Library choice of S: enough fronts to give every SIMD several waves, few
// enough that the S cold starts stay a small share of the work, and S must
// divide m/2 so that every subchain has an integer centre row.
static int choose_subchains(int64_t n_r, int64_t m, int rpl)
{
    const int64_t waves_per_front = ceil_div(n_r, 64 * rpl);
    const int64_t target_waves = 1024 * 10;
    int64_t want = ceil_div(target_waves, 2 * waves_per_front);
    want = std::min<int64_t>(want, std::max<int64_t>(1, m / 150));
    want = std::min<int64_t>(want, MAX_FRONTS / 2);
    want = std::max<int64_t>(want, 1);
    const int64_t half = m / 2;
    for (int64_t s = want; s >= 1; --s)
        if (half % s == 0) return (int)s;
    return 1;
}

template <bool EQUAL>
static void launch_sweep(Ctx *c, int n_fronts, int bpf, const double2 *cur, double2 *nxt,
                         const double2 *etab, double a, double a1, double tol_step2,
                         double tol_mu, int32_t n_r, double *out_re, double *out_im,
                         double *caus_re, double *caus_im)
{
    using T = typename StarRec<EQUAL>::T;
    const T *stars = EQUAL ? reinterpret_cast<const T *>(c->stars.p)
                           : reinterpret_cast<const T *>(c->stars4.p);
    hipLaunchKernelGGL((aberth_sweep_f64<EQUAL>), dim3(n_fronts * bpf), dim3(64), 0, c->stream,
                       stars, c->mass0, (int32_t)c->n, cur, nxt, c->flagrow.as<int32_t>(),
                       c->fronts.as<Front>(), etab, c->gamma, a, a1, tol_step2, tol_mu, n_r, bpf,
                       out_re, out_im, caus_re, caus_im, c->bnd.as<double2>(),
                       c->counts.as<int32_t>(), &c->control.as<Control>()->updates);
}

mlcc_status find_critical_curves_fp64(Ctx *c, const mlcc_cc_params *p, double *roots_re,
                                      double *roots_im, double *caus_re, double *caus_im,
                                      int32_t *chain_next, mlcc_cc_stats *stats)
{
    constexpr int RPL = 1;
    const int64_t n = c->n, n_r = 2 * n, m = p->m_steps;
    if (n_r > ((int64_t)1 << 30)) return fail(MLCC_ERR_INVALID, "too many roots");
    const int S = p->n_subchains > 0 ? p->n_subchains : choose_subchains(n_r, m, RPL);
    if (S > MAX_FRONTS / 2) return fail(MLCC_ERR_INVALID, "n_subchains > %d", MAX_FRONTS / 2);
    const int64_t L = m / S;
    const int F = 2 * S;
    const int bpf = (int)ceil_div(n_r, 64 * RPL);
    if ((int64_t)F * bpf > 0x7fffffff) return fail(MLCC_ERR_INVALID, "launch too large");
    const int max_cold = p->max_iter_cold > 0 ? p->max_iter_cold : 500;
    const int max_warm = p->max_iter_warm > 0 ? p->max_iter_warm : 100;
    constexpr int MAX_BATCH = 256;

    MLCC_TRY(c->iter[0].reserve((size_t)F * n_r * sizeof(double2)));
    MLCC_TRY(c->iter[1].reserve((size_t)F * n_r * sizeof(double2)));
    MLCC_TRY(c->flagrow.reserve((size_t)F * n_r * sizeof(int32_t)));
    MLCC_TRY(c->fronts.reserve((size_t)F * sizeof(Front)));
    MLCC_TRY(c->counts.reserve((size_t)F * sizeof(int32_t)));
    MLCC_TRY(c->control.reserve(sizeof(Control)));
    MLCC_TRY(c->etab.reserve((size_t)(m + 1) * sizeof(double2)));
    MLCC_TRY(c->bnd.reserve((size_t)std::max(S - 1, 1) * n_r * sizeof(double2)));
    MLCC_TRY(c->workflags.reserve(2 * MAX_BATCH * sizeof(int32_t)));
    MLCC_TRY(ensure_pinned(c, 2 * (sizeof(Control) + MAX_BATCH * sizeof(int32_t))));

    // phase table: (1 - kappa_s) e^{-i phi_j}, phi_j = 2 pi j / m (host libm)
    std::vector<double2> et(m + 1);
    const double a = 1.0 - c->kappa_s;
    for (int64_t j = 0; j <= m; ++j) {
        const double phi = (2.0 * M_PI * (double)j) / (double)m;
        et[j] = make_double2(a * std::cos(phi), a * -std::sin(phi));
    }
    std::vector<Front> fr(F);
    for (int s = 0; s < S; ++s) {
        const int32_t lo = (int32_t)(s * L), hi = (int32_t)(lo + L), cen = (int32_t)(lo + L / 2);
        Front &d = fr[2 * s];
        d = Front{};
        d.row = cen; d.dir = 0; d.end_row = lo; d.state = FRONT_ACTIVE; d.sweeps = 0;
        d.src = 2 * s; d.partner = 2 * s + 1; d.bnd_slot = s >= 1 ? s - 1 : -1;
        d.lo = lo; d.hi = hi;
        Front &u = fr[2 * s + 1];
        u = Front{};
        u.row = cen + 1; u.dir = 1; u.end_row = hi; u.state = FRONT_IDLE; u.sweeps = 0;
        u.src = 2 * s + 1; u.partner = -1; u.bnd_slot = -1; u.lo = lo; u.hi = hi;
    }
    Control ctl0{};
    ctl0.active_fronts = F;
    MLCC_HIP(hipMemcpyAsync(c->etab.p, et.data(), (m + 1) * sizeof(double2),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(c->fronts.p, fr.data(), F * sizeof(Front), hipMemcpyHostToDevice,
                            c->stream));
    MLCC_HIP(hipMemcpyAsync(c->control.p, &ctl0, sizeof ctl0, hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemsetAsync(c->flagrow.p, 0xff, (size_t)F * n_r * sizeof(int32_t), c->stream));
    MLCC_HIP(hipMemsetAsync(c->counts.p, 0, F * sizeof(int32_t), c->stream));
    {
        const int64_t tot = (int64_t)S * n_r;
        hipLaunchKernelGGL(seed_centres, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                           c->stream, c->stars.as<double2>(), (int32_t)n_r, S,
                           c->iter[0].as<double2>());
        MLCC_HIP(hipGetLastError());
    }
    // Host copies must finish before the vectors above go out of scope.
    MLCC_HIP(hipStreamSynchronize(c->stream));

    const double tol_step2 = p->tol_step * p->tol_step;
    const double a1 = std::fabs(a);
    const double2 *etab = c->etab.as<double2>();
    Control *dctl = c->control.as<Control>();
    char *pin = static_cast<char *>(c->pinned);
    auto pin_ctl = [&](int slot) {
        return reinterpret_cast<Control *>(pin + slot * (sizeof(Control) + MAX_BATCH * 4));
    };
    auto pin_flags = [&](int slot) {
        return reinterpret_cast<int32_t *>(pin + slot * (sizeof(Control) + MAX_BATCH * 4) +
                                           sizeof(Control));
    };

    std::vector<hipEvent_t> evs;
    if (p->timing) {
        evs.resize(4 * MAX_BATCH);
        for (auto &e : evs) MLCC_HIP(hipEventCreate(&e));
    }
    auto cleanup = [&]() {
        for (auto &e : evs) (void)hipEventDestroy(e);
        evs.clear();
    };
    hipEvent_t done_ev[2];
    MLCC_HIP(hipEventCreateWithFlags(&done_ev[0], hipEventDisableTiming));
    MLCC_HIP(hipEventCreateWithFlags(&done_ev[1], hipEventDisableTiming));

    int parity = 0;
    int batch_len[2] = {0, 0};
    int G = 4;
    double sweep_ms = 0.0;
    int32_t polls = 0;
    // Every front finishes within max_cold + (L/2 + 1) * max_warm sweeps; the
    // extra margin covers the batches enqueued ahead of the last poll.
    const int64_t launch_cap = (int64_t)max_cold + (L / 2 + 2) * (int64_t)max_warm + 4 * MAX_BATCH;
    int64_t launched = 0;
    auto enqueue_batch = [&](int slot, int g) -> mlcc_status {
        for (int i = 0; i < g; ++i) {
            const double2 *cur = c->iter[parity].as<double2>();
            double2 *nxt = c->iter[parity ^ 1].as<double2>();
            if (p->timing) MLCC_HIP(hipEventRecord(evs[(slot * MAX_BATCH + i) * 2], c->stream));
            if (c->equal_mass)
                launch_sweep<true>(c, F, bpf, cur, nxt, etab, a, a1, tol_step2, p->tol_inv_mu,
                                   (int32_t)n_r, roots_re, roots_im, caus_re, caus_im);
            else
                launch_sweep<false>(c, F, bpf, cur, nxt, etab, a, a1, tol_step2, p->tol_inv_mu,
                                    (int32_t)n_r, roots_re, roots_im, caus_re, caus_im);
            if (p->timing) MLCC_HIP(hipEventRecord(evs[(slot * MAX_BATCH + i) * 2 + 1], c->stream));
            hipLaunchKernelGGL(aberth_control, dim3(1), dim3(CONTROL_THREADS), 0, c->stream,
                               c->fronts.as<Front>(), c->counts.as<int32_t>(), F, dctl, max_cold,
                               max_warm, c->workflags.as<int32_t>() + slot * MAX_BATCH + i);
            parity ^= 1;
        }
        MLCC_HIP(hipGetLastError());
        MLCC_HIP(hipMemcpyAsync(pin_ctl(slot), dctl, sizeof(Control), hipMemcpyDeviceToHost,
                                c->stream));
        MLCC_HIP(hipMemcpyAsync(pin_flags(slot), c->workflags.as<int32_t>() + slot * MAX_BATCH,
                                g * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        MLCC_HIP(hipEventRecord(done_ev[slot], c->stream));
        batch_len[slot] = g;
        launched += g;
        return MLCC_OK;
    };

    mlcc_status st = MLCC_OK;
    int slot = 0;
    auto t_last = std::chrono::steady_clock::now();
    st = enqueue_batch(slot, G);
    while (st == MLCC_OK) {
        // keep one batch queued behind the one being polled
        const int next = slot ^ 1;
        st = enqueue_batch(next, G);
        if (st != MLCC_OK) break;
        if (hipEventSynchronize(done_ev[slot]) != hipSuccess) {
            st = fail(MLCC_ERR_HIP, "sweep batch failed: %s", hipGetErrorString(hipGetLastError()));
            break;
        }
        ++polls;
        const Control h = *pin_ctl(slot);
        if (p->timing) {
            for (int i = 0; i < batch_len[slot]; ++i) {
                if (!pin_flags(slot)[i]) continue;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, evs[(slot * MAX_BATCH + i) * 2],
                                          evs[(slot * MAX_BATCH + i) * 2 + 1]);
                sweep_ms += ms;
            }
        }
        if (h.active_fronts == 0) {
            // drain the batch queued ahead (it found nothing to do)
            MLCC_HIP(hipEventSynchronize(done_ev[next]));
            if (p->timing) {
                for (int i = 0; i < batch_len[next]; ++i) {
                    if (!pin_flags(next)[i]) continue;
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, evs[(next * MAX_BATCH + i) * 2],
                                              evs[(next * MAX_BATCH + i) * 2 + 1]);
                    sweep_ms += ms;
                }
            }
            break;
        }
        if (launched > launch_cap) {
            st = fail(MLCC_ERR_HIP, "root finder exceeded %lld launches", (long long)launch_cap);
            break;
        }
        // poll roughly every 4 ms of GPU work
        auto now = std::chrono::steady_clock::now();
        const double dt = std::chrono::duration<double, std::milli>(now - t_last).count();
        t_last = now;
        const double per = dt / std::max(1, batch_len[slot]);
        G = (int)std::min<double>(MAX_BATCH, std::max<double>(2.0, 4.0 / std::max(per, 1e-3)));
        slot = next;
    }
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(done_ev[0]);
    (void)hipEventDestroy(done_ev[1]);
    cleanup();
    if (st != MLCC_OK) return st;

    Control h{};
    MLCC_HIP(hipMemcpy(&h, dctl, sizeof h, hipMemcpyDeviceToHost));
    std::vector<Front> fin(F);
    MLCC_HIP(hipMemcpy(fin.data(), c->fronts.p, F * sizeof(Front), hipMemcpyDeviceToHost));

    mlcc_status result = MLCC_OK;
    double maxdist = 0.0;
    if (h.failed_rows > 0) {
        result = fail(MLCC_ERR_NOT_CONVERGED, "%d rows hit the sweep cap (%lld roots unconverged)",
                      h.failed_rows, (long long)h.unconverged);
    } else {
        // join subchains: pair each duplicate boundary row with the stored
        // copy, compose the pairings into global labels, relabel the blocks
        if (S > 1) {
            MLCC_TRY(c->perm.reserve((size_t)(S + 1) * n_r * sizeof(int32_t)));
            int32_t *perm = c->perm.as<int32_t>();
            for (int s = 1; s < S; ++s) {
                double md = 0.0;
                const int64_t lo = s * L;
                MLCC_TRY(pair_rows(c, n_r, c->bnd.as<double2>() + (int64_t)(s - 1) * n_r,
                                   roots_re + lo * n_r, roots_im + lo * n_r,
                                   perm + (int64_t)s * n_r, 1e-6, &md));
                maxdist = std::max(maxdist, md);
            }
            std::vector<int32_t> hp((size_t)S * n_r), lab((size_t)S * n_r);
            MLCC_HIP(hipMemcpy(hp.data(), perm, (size_t)S * n_r * sizeof(int32_t),
                               hipMemcpyDeviceToHost));
            for (int64_t k = 0; k < n_r; ++k) lab[k] = (int32_t)k;
            for (int s = 1; s < S; ++s)
                for (int64_t k = 0; k < n_r; ++k)
                    lab[s * n_r + k] = lab[(s - 1) * n_r + hp[s * n_r + k]];
            MLCC_HIP(hipMemcpy(perm, lab.data(), (size_t)S * n_r * sizeof(int32_t),
                               hipMemcpyHostToDevice));
            for (int s = 1; s < S; ++s) {
                MLCC_TRY(relabel_rows(c, roots_re, roots_im, n_r, s * L + 1, (s + 1) * L + 1,
                                      perm + (int64_t)s * n_r));
                if (caus_re)
                    MLCC_TRY(relabel_rows(c, caus_re, caus_im, n_r, s * L + 1, (s + 1) * L + 1,
                                          perm + (int64_t)s * n_r));
            }
        }
        if (chain_next) {
            double md = 0.0;
            MLCC_TRY(pair_rows_soa(c, n_r, roots_re + m * n_r, roots_im + m * n_r, roots_re,
                                   roots_im, chain_next, 1e-6, &md));
            maxdist = std::max(maxdist, md);
        }
        MLCC_HIP(hipStreamSynchronize(c->stream));
    }

    if (stats) {
        *stats = mlcc_cc_stats{};
        stats->sweeps = h.live_sweeps;
        stats->root_updates = (int64_t)h.updates;
        stats->unconverged = h.unconverged;
        stats->rows_capped = h.failed_rows;
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
        stats->sweep_ms = sweep_ms;
        stats->algorithmic_flop =
            (double)h.updates * (29.0 * (double)n + 10.0 * (double)(n_r - 1));
    }
    return result;
}

} // namespace mlcc
