// Critical-curve root finder: parallel Aberth-Ehrlich sweeps (Sec. 3.2)
// over the phase grid, warm-started along phi and grown centre-out in
// subchains (Sec. 4.3).
//
// Layout and scheduling (gfx950):
//  * One lane per root, one 64-lane wavefront per work-group.  Each
//    work-group owns 64*RPL consecutive roots of one "front" (a growing end
//    of a subchain).  Star positions and the other roots are wave-uniform
//    reads, so they arrive through scalar loads and feed the FP64 VALU as
//    SGPR operands: no LDS, no barriers.
//  * Jacobi double buffering: a sweep reads iterate `cur` and writes `nxt`;
//    the host alternates the two on every launch.  A root flagged converged
//    is copied forward unchanged.
//  * A single-work-group control kernel after every sweep advances the
//    fronts whose rows have converged (device-side, so the host only polls
//    a small status block every few launches, one batch ahead).
#include <algorithm>
#include <chrono>
#include <cmath>
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

// Star-sum steps per root: 2 refinement steps give a fully accurate
// reciprocal, as F itself must be exact to the last bits.  The root-root sum
// only enters the step through F * R, which vanishes at convergence, so one
// step (relative error ~1e-14) suffices there.
constexpr int RCP_STAR = 2;
constexpr int RCP_ROOT = 1;

template <int RPL, bool EQUAL>
__global__ void __launch_bounds__(64)
aberth_sweep_f64(const double2 *__restrict__ stars, const double *__restrict__ mass,
                 double m0, int32_t n_stars, const double2 *__restrict__ cur, double2 *__restrict__ nxt,
                 int32_t *__restrict__ flagrow, const Front *__restrict__ fronts,
                 const double2 *__restrict__ etab, double gamma, double a1, double tol_step2,
                 double tol_mu, int32_t n_r, int32_t blocks_per_front,
                 double *__restrict__ out_re, double *__restrict__ out_im,
                 double2 *__restrict__ bnd, int32_t *__restrict__ counts,
                 unsigned long long *__restrict__ updates)
{
    const int f = blockIdx.x / blocks_per_front;
    const int q = blockIdx.x - f * blocks_per_front;
    const int state = fronts[f].state;
    if (state != FRONT_ACTIVE) return;
    const int row = fronts[f].row;
    const int src = fronts[f].src;
    const int lane = threadIdx.x;
    const int64_t base_f = (int64_t)f * n_r;
    const double2 *__restrict__ zsrc = cur + (int64_t)src * n_r;
    const int k0 = q * 64 * RPL;

    double zr[RPL], zi[RPL];
    bool act[RPL], valid[RPL];
    bool any = false;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int k = k0 + r * 64 + lane;
        valid[r] = k < n_r;
        if (valid[r]) {
            const double2 z = zsrc[k];
            zr[r] = z.x;
            zi[r] = z.y;
            act[r] = flagrow[base_f + k] != row;
        } else {
            zr[r] = 0.0;
            zi[r] = 0.0;
            act[r] = false;
        }
        any = any || act[r];
    }
    if (__ballot(any) == 0) {
        // every root of this block already converged on this row: carry it
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (valid[r]) nxt[base_f + k0 + r * 64 + lane] = make_double2(zr[r], zi[r]);
        return;
    }

    // S1 = sum u, S2 = sum m u^2, S3 = sum m u^3, u = 1/(z - z_i)
    double s1r[RPL], s1i[RPL], s2r[RPL], s2i[RPL], s3r[RPL], s3i[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) s1r[r] = s1i[r] = s2r[r] = s2i[r] = s3r[r] = s3i[r] = 0.0;

#pragma unroll 2
    for (int i = 0; i < n_stars; ++i) {
        const double2 s = stars[i];
        const double mi = EQUAL ? 0.0 : mass[i];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double dx = zr[r] - s.x;
            const double dy = zi[r] - s.y;
            const double inv = rcp_refined<RCP_STAR>(fma(dx, dx, dy * dy));
            // u = ux - i uy = conj(d) / |d|^2
            const double ux = dx * inv;
            const double uy = dy * inv;
            s1r[r] += ux;
            s1i[r] -= uy;
            // u^2 = vx + i vy
            const double vx = fma(ux, ux, -uy * uy);
            const double vy = -2.0 * ux * uy;
            // u^3 = u^2 u
            const double tx = fma(vx, ux, vy * uy);
            const double ty = fma(vy, ux, -vx * uy);
            if (EQUAL) {
                s2r[r] += vx;
                s2i[r] += vy;
                s3r[r] += tx;
                s3i[r] += ty;
            } else {
                s2r[r] = fma(mi, vx, s2r[r]);
                s2i[r] = fma(mi, vy, s2i[r]);
                s3r[r] = fma(mi, tx, s3r[r]);
                s3i[r] = fma(mi, ty, s3i[r]);
            }
        }
    }

    // R = sum_{r != k} 1/(z_k - z_r) over the front's current iterate
    double Rr[RPL], Ri[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) Rr[r] = Ri[r] = 0.0;
    const int own_lo = k0, own_hi = min(k0 + 64 * RPL, n_r);
#pragma unroll 2
    for (int j = 0; j < own_lo; ++j) {
        const double2 o = zsrc[j];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double dx = zr[r] - o.x, dy = zi[r] - o.y;
            const double inv = rcp_refined<RCP_ROOT>(fma(dx, dx, dy * dy));
            Rr[r] = fma(dx, inv, Rr[r]);
            Ri[r] = fma(-dy, inv, Ri[r]);
        }
    }
    for (int j = own_lo; j < own_hi; ++j) {
        const double2 o = zsrc[j];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double dx = zr[r] - o.x, dy = zi[r] - o.y;
            const double inv = rcp_refined<RCP_ROOT>(fma(dx, dx, dy * dy));
            const bool self = j == k0 + r * 64 + lane;
            Rr[r] = self ? Rr[r] : fma(dx, inv, Rr[r]);
            Ri[r] = self ? Ri[r] : fma(-dy, inv, Ri[r]);
        }
    }
#pragma unroll 2
    for (int j = own_hi; j < n_r; ++j) {
        const double2 o = zsrc[j];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const double dx = zr[r] - o.x, dy = zi[r] - o.y;
            const double inv = rcp_refined<RCP_ROOT>(fma(dx, dx, dy * dy));
            Rr[r] = fma(dx, inv, Rr[r]);
            Ri[r] = fma(-dy, inv, Ri[r]);
        }
    }

    const double2 e = etab[row];
    const bool boundary = fronts[f].bnd_slot >= 0 && row == fronts[f].end_row;
    double2 *__restrict__ bnd_row = bnd + (int64_t)max(fronts[f].bnd_slot, 0) * n_r;
    int n_after = 0, n_upd = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int k = k0 + r * 64 + lane;
        if (EQUAL) {   // every mass equals m0: the sums above left it out
            s2r[r] *= m0;
            s2i[r] *= m0;
            s3r[r] *= m0;
            s3i[r] *= m0;
        }
        // F = gamma + S2 - (1 - kappa_s) e^{-i phi}, F' = -2 S3
        const double Fr = gamma + s2r[r] - e.x, Fi = s2i[r] - e.y;
        const double Fpr = -2.0 * s3r[r], Fpi = -2.0 * s3i[r];
        // Aberth step: 1 / (F'/F + 2 S1 - R) = F / (F' + F (2 S1 - R))
        const double Gr = 2.0 * s1r[r] - Rr[r], Gi = 2.0 * s1i[r] - Ri[r];
        const double Dr = Fpr + (Fr * Gr - Fi * Gi);
        const double Di = Fpi + (Fr * Gi + Fi * Gr);
        const double den = Dr * Dr + Di * Di;
        const double stepr = (Fr * Dr + Fi * Di) / den;
        const double stepi = (Fi * Dr - Fr * Di) / den;
        double nr = zr[r] - stepr, ni = zi[r] - stepi;
        const double aF = sqrt(Fr * Fr + Fi * Fi);
        bool flag = (stepr * stepr + stepi * stepi < tol_step2) || (aF * (aF + 2.0 * a1) < tol_mu);
        if (!isfinite(nr) || !isfinite(ni)) {
            // the iterate hit a star or two roots met: nudge it off, keep iterating
            nr = zr[r] + 1e-7 * (1 + (k & 7));
            ni = zi[r] + 1e-7 * (1 + (k >> 3 & 7));
            flag = false;
        }
        const bool upd = act[r];
        const bool still = upd && !flag;
        n_after += __popcll(__ballot(still));
        n_upd += __popcll(__ballot(upd));
        if (valid[r]) {
            if (upd) {
                nxt[base_f + k] = make_double2(nr, ni);
                if (flag) {
                    flagrow[base_f + k] = row;
                    if (boundary) {
                        bnd_row[k] = make_double2(nr, ni);
                    } else {
                        out_re[(int64_t)row * n_r + k] = nr;
                        out_im[(int64_t)row * n_r + k] = ni;
                    }
                }
            } else {
                nxt[base_f + k] = make_double2(zr[r], zi[r]);
            }
        }
    }
    if (lane == 0) {
        if (n_after) atomicAdd(&counts[f], n_after);
        if (n_upd) atomicAdd(updates, (unsigned long long)n_upd);
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
    const int64_t target_waves = 1024 * 8;
    int64_t want = ceil_div(target_waves, 2 * waves_per_front);
    want = std::min<int64_t>(want, std::max<int64_t>(1, m / 150));
    want = std::min<int64_t>(want, MAX_FRONTS / 2);
    want = std::max<int64_t>(want, 1);
    const int64_t half = m / 2;
    for (int64_t s = want; s >= 1; --s)
        if (half % s == 0) return (int)s;
    return 1;
}

template <int RPL, bool EQUAL>
static void launch_sweep(Ctx *c, int n_fronts, int bpf, const double2 *cur, double2 *nxt,
                         const double2 *etab, double a1, double tol_step2, double tol_mu,
                         int32_t n_r, double *out_re, double *out_im)
{
    hipLaunchKernelGGL((aberth_sweep_f64<RPL, EQUAL>), dim3(n_fronts * bpf), dim3(64), 0,
                       c->stream, c->stars.as<double2>(), c->mass.as<double>(), c->mass0,
                       (int32_t)c->n, cur, nxt, c->flagrow.as<int32_t>(), c->fronts.as<Front>(), etab, c->gamma,
                       a1, tol_step2, tol_mu, n_r, bpf, out_re, out_im, c->bnd.as<double2>(),
                       c->counts.as<int32_t>(),
                       &c->control.as<Control>()->updates);
}

mlcc_status find_critical_curves_fp64(Ctx *c, const mlcc_cc_params *p, double *roots_re,
                                      double *roots_im, int32_t *chain_next,
                                      mlcc_cc_stats *stats)
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
                launch_sweep<RPL, true>(c, F, bpf, cur, nxt, etab, a1, tol_step2, p->tol_inv_mu,
                                        (int32_t)n_r, roots_re, roots_im);
            else
                launch_sweep<RPL, false>(c, F, bpf, cur, nxt, etab, a1, tol_step2, p->tol_inv_mu,
                                         (int32_t)n_r, roots_re, roots_im);
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
            for (int s = 1; s < S; ++s)
                MLCC_TRY(relabel_rows(c, roots_re, roots_im, n_r, s * L + 1, (s + 1) * L + 1,
                                      perm + (int64_t)s * n_r));
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
