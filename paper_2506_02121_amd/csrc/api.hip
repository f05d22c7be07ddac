// C-ABI entry points: argument validation, context and memory management.
// The arithmetic lives in aberth.hip, chains.hip, caustics.hip,
// crossings.hip and edt.hip.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <vector>

#include "mlcc_internal.h"

namespace mlcc {

static thread_local std::string g_error = "no error";

mlcc_status fail(mlcc_status s, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return s;
}

void clear_error() { g_error = "no error"; }

mlcc_status DevBuf::reserve(size_t n)
{
    if (n <= bytes && p) return MLCC_OK;
    release();
    size_t want = std::max<size_t>(n, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(MLCC_ERR_NOMEM, "hipMalloc(%zu bytes): %s", want, hipGetErrorString(e));
    }
    bytes = want;
    return MLCC_OK;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

mlcc_status check_device_ptr(const Ctx *c, const void *p, const char *what)
{
    if (!p) return fail(MLCC_ERR_INVALID, "%s is NULL", what);
    hipPointerAttribute_t a;
    memset(&a, 0, sizeof a);
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MLCC_ERR_INVALID, "%s (%p) is not device memory", what, p);
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
        return fail(MLCC_ERR_INVALID, "%s (%p) is not device memory (type %d)", what, p,
                    (int)a.type);
    if (a.device != c->device)
        return fail(MLCC_ERR_INVALID, "%s lives on device %d, context on device %d", what,
                    a.device, c->device);
    return MLCC_OK;
}

mlcc_status ensure_pinned(Ctx *c, size_t bytes)
{
    if (c->pinned && c->pinned_bytes >= bytes) return MLCC_OK;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    void *p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MLCC_ERR_NOMEM, "hipHostMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    c->pinned = p;
    c->pinned_bytes = bytes;
    return MLCC_OK;
}

static mlcc_status use_device(const Ctx *c)
{
    MLCC_HIP(hipSetDevice(c->device));
    return MLCC_OK;
}

static mlcc_status check_grid(const mlcc_grid *g, bool square)
{
    if (!g) return fail(MLCC_ERR_INVALID, "grid is NULL");
    if (g->nx < 1 || g->ny < 1) return fail(MLCC_ERR_INVALID, "grid needs nx, ny >= 1");
    if (!(g->half_width > 0) || !(g->half_height > 0) || !std::isfinite(g->half_width) ||
        !std::isfinite(g->half_height) || !std::isfinite(g->center_re) ||
        !std::isfinite(g->center_im))
        return fail(MLCC_ERR_INVALID, "grid extents must be finite and positive");
    if ((int64_t)g->nx * g->ny > ((int64_t)1 << 31))
        return fail(MLCC_ERR_INVALID, "grid larger than 2^31 pixels");
    if (square) {
        double hx = (2.0 * g->half_width) / g->nx, hy = (2.0 * g->half_height) / g->ny;
        if (!(std::fabs(hx - hy) <= 1e-9 * hx))
            return fail(MLCC_ERR_INVALID, "pixels must be square (hx=%.17g, hy=%.17g)", hx, hy);
    }
    return MLCC_OK;
}

// The sheet polynomial of a rectangular field.  App. B gives d alpha_s / d zbar
// as -kappa_star i / pi sum_{j=1..t} (1/j) (zbar/c)^j (1 + (-1)^j)
// (1 - e^{2 i Arg(c) j}) + kappa_star - 4 kappa_star Arg(c) / pi (the power-t term
// vanishes for odd t).  Only even j survive, and with c = |c| e^{i th},
// (1 - e^{2 i th j}) / c^j = -2 i sin(j th) / |c|^j, so its conjugate is the
// real-coefficient polynomial
//   d0 + sum_{j = 2, 4, ..., t-1} d_j z^j,  d_j = -(4 kappa_star / pi) sin(j th) / (j |c|^j),
//   d0 = kappa_star (1 - 4 th / pi).
// Integrating d alpha_s / d zbar (and d alpha_s / dz = -kappa_star) from the
// origin, where the sheet's deflection vanishes by symmetry, gives alpha_s =
// -kappa_star z + d0 conj(z) + sum_j d_j conj(z)^(j+1) / (j+1).
SheetPoly sheet_poly(const RealHost &h)
{
    SheetPoly p;
    if (h.t <= 0) return p;
    const double th = std::atan2(h.c2, h.c1), ac = std::hypot(h.c1, h.c2);
    p.d0 = h.kappa_star * (1.0 - 4.0 * th / M_PI);
    p.n = (h.t - 1) / 2;
    p.n_extra = h.t - 1;
    p.seed_r = ac;
    for (int k = 1; k <= p.n; ++k) {
        const int j = 2 * k;
        p.d[k - 1] = -(4.0 * h.kappa_star / M_PI) * std::sin(j * th) / (j * std::pow(ac, j));
        p.dmap[k - 1] = p.d[k - 1] / (j + 1);
    }
    return p;
}

// (t - 1) Arg(c) must stay at least 10% of pi away from a multiple of pi, or
// the leading coefficient of the sheet polynomial (~ sin((t-1) Arg c)) nearly
// vanishes and roots escape to infinity (App. B).
static bool arg_rule_ok(int t, double c1, double c2)
{
    if (t < 3) return true;
    const double r = std::fmod((t - 1) * std::atan2(c2, c1), M_PI);
    return r >= 0.1 * M_PI && r <= 0.9 * M_PI;
}

} // namespace mlcc

using namespace mlcc;

extern "C" {

const char *mlcc_last_error(void) { return g_error.c_str(); }

mlcc_status mlcc_create(mlcc_ctx **out, int device, void *hip_stream)
{
    if (!out) return fail(MLCC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    MLCC_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(MLCC_ERR_INVALID, "device %d out of range (%d devices)", device, ndev);
    MLCC_HIP(hipSetDevice(device));
    MLCC_TRY(noalloc_scratch_init(device));
    mlcc_ctx *c = new (std::nothrow) mlcc_ctx();
    if (!c) return fail(MLCC_ERR_NOMEM, "context allocation failed");
    c->impl.device = device;
    c->impl.stream = static_cast<hipStream_t>(hip_stream);
    *out = c;
    clear_error();
    return MLCC_OK;
}

void mlcc_destroy(mlcc_ctx *ctx)
{
    if (!ctx) return;
    Ctx &c = ctx->impl;
    (void)hipSetDevice(c.device);
    (void)hipStreamSynchronize(c.stream);
    DevBuf *bufs[] = {&c.stars, &c.mass, &c.stars4, &c.sheet_d, &c.sheet, &c.iter[0], &c.iter[1],
                      &c.flagrow, &c.fronts, &c.counts, &c.control, &c.fmm_tally, &c.etab,
                      &c.bnd, &c.perm, &c.match_aux, &c.relabel, &c.workflags, &c.vieta, &c.errbuf, &c.vsum,
                      &c.pq, &c.passupd, &c.reals_d, &c.bmap, &c.diff, &c.edt_col,
                      &c.dmask, &c.fmm_cs, &c.fmm_st, &c.fmm_st2, &c.fmm_cf, &c.fmm_cg,
                      &c.fmm_q, &c.fmm_m, &c.fmm_args};
    for (DevBuf *b : bufs) b->release();
    if (c.own_stream) (void)hipStreamDestroy(c.own_stream);
    if (c.pinned) (void)hipHostFree(c.pinned);
    delete ctx;
}

mlcc_status mlcc_set_stream(mlcc_ctx *ctx, void *hip_stream)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    ctx->impl.stream = static_cast<hipStream_t>(hip_stream);
    return MLCC_OK;
}

void mlcc_cc_params_default(mlcc_cc_params *p, int64_t m_steps)
{
    if (!p) return;
    memset(p, 0, sizeof *p);
    p->m_steps = m_steps;
    p->n_subchains = 0;
    p->max_iter_cold = 500;
    p->max_iter_warm = 100;
    p->precision = MLCC_FP64;
    p->tol_step = 1e-9;
    p->tol_inv_mu = 1e-9;
    p->timing = 0;
    p->predictor = 2;
    p->schedule = MLCC_SCHEDULE_PERSISTENT;
}

// Compensated (Neumaier) summation.
struct Neumaier {
    double s = 0.0, c = 0.0;
    void add(double x)
    {
        const double t = s + x;
        c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    double value() const { return s + c; }
};

// Loads one or several star fields (concatenated; field r holds stars
// [off[r], off[r+1])) and the per-field sums the root finder checks rows
// against.
static mlcc_status load_fields(Ctx &c, int32_t n_fields, const int64_t *off, const double *x,
                               const double *y, const double *m, const double *kappa_s,
                               const double *gamma, bool batched, bool rect = false)
{
    MLCC_TRY(use_device(&c));
    if (n_fields < 1 || n_fields > 65536)
        return fail(MLCC_ERR_INVALID, "need 1..65536 fields (got %d)", n_fields);
    if (off[0] != 0) return fail(MLCC_ERR_INVALID, "star_offsets[0] must be 0");
    for (int32_t r = 0; r < n_fields; ++r)
        if (off[r + 1] - off[r] < 1)
            return fail(MLCC_ERR_INVALID, "field %d: need at least one star", r);
    const int64_t n = off[n_fields];
    if (n > (int64_t)1 << 28) return fail(MLCC_ERR_INVALID, "too many stars (%lld)", (long long)n);
    MLCC_TRY(check_device_ptr(&c, x, "x"));
    MLCC_TRY(check_device_ptr(&c, y, "y"));
    MLCC_TRY(check_device_ptr(&c, m, "m"));
    for (int32_t r = 0; r < n_fields; ++r) {
        if (!std::isfinite(kappa_s[r]) || !std::isfinite(gamma[r]))
            return fail(MLCC_ERR_INVALID, "field %d: kappa_s and gamma must be finite", r);
        if (!rect && std::fabs(gamma[r]) == std::fabs(1.0 - kappa_s[r]))
            return fail(MLCC_ERR_INVALID,
                        "field %d: |gamma| == |1 - kappa_s|: gamma - (1-kappa_s) e^{-i phi} "
                        "vanishes on the phase circle", r);
    }
    std::vector<double> hx(n), hy(n), hm(n);
    MLCC_HIP(hipMemcpyAsync(hx.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    MLCC_HIP(hipMemcpyAsync(hy.data(), y, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    MLCC_HIP(hipMemcpyAsync(hm.data(), m, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    MLCC_HIP(hipStreamSynchronize(c.stream));
    std::vector<RealHost> reals(n_fields);
    for (int32_t r = 0; r < n_fields; ++r) {
        const int64_t i0 = off[r], i1 = off[r + 1];
        RealHost &h = reals[r];
        h.star_off = i0;
        h.n = i1 - i0;
        h.kappa_s = kappa_s[r];
        h.gamma = gamma[r];
        h.m0 = hm[i0];
        h.equal = true;
        for (int64_t i = i0; i < i1; ++i) {
            if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || !std::isfinite(hm[i]) ||
                !(hm[i] > 0))
                return fail(MLCC_ERR_INVALID, "star %lld: non-finite position or mass <= 0",
                            (long long)i);
            if (hm[i] != hm[i0]) h.equal = false;
        }
        std::vector<int64_t> idx(h.n);
        for (int64_t i = 0; i < h.n; ++i) idx[i] = i0 + i;
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            return hx[a] < hx[b] || (hx[a] == hx[b] && hy[a] < hy[b]);
        });
        for (int64_t i = 1; i < h.n; ++i)
            if (hx[idx[i]] == hx[idx[i - 1]] && hy[idx[i]] == hy[idx[i - 1]])
                return fail(MLCC_ERR_INVALID, "stars %lld and %lld share a position",
                            (long long)idx[i - 1], (long long)idx[i]);
        // row identities of the root finder: sum z_i, sum z_i^2 (compensated
        // sums), total mass
        Neumaier s1r, s1i, s2r, s2i;
        for (int64_t i = i0; i < i1; ++i) {
            s1r.add(hx[i]);
            s1i.add(hy[i]);
            s2r.add(hx[i] * hx[i] - hy[i] * hy[i]);
            s2i.add(2.0 * hx[i] * hy[i]);
            const double r2 = hx[i] * hx[i] + hy[i] * hy[i];
            h.sum_abs_z += std::sqrt(r2);
            h.sum_abs_z2 += r2;
            h.max_abs_z = std::max(h.max_abs_z, std::sqrt(r2));
            h.mass_total += hm[i];
        }
        h.sum_z = make_double2(s1r.value(), s1i.value());
        h.sum_z2 = make_double2(s2r.value(), s2i.value());
    }
    std::vector<double> xy(2 * n), xym(4 * n);
    for (int64_t i = 0; i < n; ++i) {
        xy[2 * i] = hx[i];
        xy[2 * i + 1] = hy[i];
        xym[4 * i] = hx[i];
        xym[4 * i + 1] = hy[i];
        xym[4 * i + 2] = hm[i];
        xym[4 * i + 3] = 0.0;
    }
    c.hstars.resize(n);
    for (int64_t i = 0; i < n; ++i) c.hstars[i] = make_double4(hx[i], hy[i], hm[i], 0.0);
    MLCC_TRY(c.stars4.reserve(4 * n * sizeof(double)));
    MLCC_TRY(c.stars.reserve(2 * n * sizeof(double)));
    MLCC_TRY(c.mass.reserve(n * sizeof(double)));
    MLCC_HIP(hipMemcpyAsync(c.stars4.p, xym.data(), 4 * n * sizeof(double), hipMemcpyHostToDevice,
                            c.stream));
    MLCC_HIP(hipMemcpyAsync(c.stars.p, xy.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice,
                            c.stream));
    MLCC_HIP(hipMemcpyAsync(c.mass.p, hm.data(), n * sizeof(double), hipMemcpyHostToDevice,
                            c.stream));
    MLCC_HIP(hipStreamSynchronize(c.stream));
    c.reals = std::move(reals);
    c.batched = batched;
    c.rect = false;
    c.n = n;
    c.kappa_s = kappa_s[0];
    c.gamma = gamma[0];
    c.equal_mass = c.reals[0].equal && !batched;
    c.mass0 = hm[0];
    clear_error();
    return MLCC_OK;
}

mlcc_status mlcc_rect_taylor_degree(double kappa_star, double c1, double c2, double s, double eps,
                                    int32_t *t_out)
{
    if (!t_out) return fail(MLCC_ERR_INVALID, "t is NULL");
    if (!(kappa_star > 0) || !(c1 > 0) || !(c2 > 0) || !(s > 1) || !(eps > 0) ||
        !std::isfinite(kappa_star) || !std::isfinite(c1) || !std::isfinite(c2) ||
        !std::isfinite(s))
        return fail(MLCC_ERR_INVALID, "need kappa_star, c1, c2, eps > 0 and s > 1");
    const double ac = std::hypot(c1, c2);
    // App. B: |error| <= kappa_star / pi * 4 / (t + 1) * s^-(t+1) * |c| (s + 1) / (s - 1)
    // where |z| s < |c|; smallest such t, odd, then the Arg rule
    auto bound = [&](int t) {
        return kappa_star / M_PI * 4.0 / (t + 1) * std::pow(s, -(t + 1)) * ac * (s + 1) / (s - 1);
    };
    int t = 1;
    while (bound(t) > eps)
        if (++t > 2 * MAX_SHEET_TERMS + 1)
            return fail(MLCC_ERR_INVALID, "the App. B bound needs t > %d", 2 * MAX_SHEET_TERMS + 1);
    if (!(t & 1)) ++t;
    while (!arg_rule_ok(t, c1, c2)) {
        t += 2;
        if (t > 2 * MAX_SHEET_TERMS + 1)
            return fail(MLCC_ERR_INVALID, "no admissible odd t <= %d", 2 * MAX_SHEET_TERMS + 1);
    }
    *t_out = t;
    clear_error();
    return MLCC_OK;
}

mlcc_status mlcc_set_lenses_rect(mlcc_ctx *ctx, int64_t n, const double *x, const double *y,
                                 const double *m, double kappa_s, double gamma, double kappa_star,
                                 double c1, double c2, int32_t t)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    if (n < 1) return fail(MLCC_ERR_INVALID, "need at least one star (n=%lld)", (long long)n);
    if (n > (int64_t)1 << 28) return fail(MLCC_ERR_INVALID, "too many stars (%lld)", (long long)n);
    if (!(kappa_star > 0) || !(c1 > 0) || !(c2 > 0) || !std::isfinite(kappa_star) ||
        !std::isfinite(c1) || !std::isfinite(c2))
        return fail(MLCC_ERR_INVALID, "need finite kappa_star, c1, c2 > 0");
    if (t < 1 || !(t & 1) || t > 2 * MAX_SHEET_TERMS + 1)
        return fail(MLCC_ERR_INVALID, "t must be odd, 1..%d (got %d)", 2 * MAX_SHEET_TERMS + 1, t);
    if (!arg_rule_ok(t, c1, c2))
        return fail(MLCC_ERR_INVALID,
                    "(t - 1) Arg(c) lies within 10%% of pi of a multiple of pi: the sheet "
                    "polynomial's leading coefficient nearly vanishes; raise t by 2");
    RealHost probe;
    probe.t = t;
    probe.kappa_star = kappa_star;
    probe.c1 = c1;
    probe.c2 = c2;
    if (t == 1) {
        const double g = gamma - sheet_poly(probe).d0;
        if (std::fabs(g) == std::fabs(1.0 - kappa_s))
            return fail(MLCC_ERR_INVALID, "t = 1 and |gamma - d0| == |1 - kappa_s|");
    }
    const int64_t off[2] = {0, n};
    Ctx &c = ctx->impl;
    MLCC_TRY(load_fields(c, 1, off, x, y, m, &kappa_s, &gamma, false, true));
    RealHost &h = c.reals[0];
    h.t = t;
    h.kappa_star = kappa_star;
    h.c1 = c1;
    h.c2 = c2;
    c.rect = true;
    return MLCC_OK;
}

mlcc_status mlcc_num_roots(mlcc_ctx *ctx, int64_t *n_r)
{
    if (!ctx || !n_r) return fail(MLCC_ERR_INVALID, "ctx or n_r is NULL");
    const Ctx &c = ctx->impl;
    if (c.n < 1) return fail(MLCC_ERR_STATE, "call mlcc_set_lenses first");
    int64_t tot = 0;
    for (const RealHost &h : c.reals) tot += 2 * h.n + sheet_poly(h).n_extra;
    *n_r = tot;
    clear_error();
    return MLCC_OK;
}

mlcc_status mlcc_set_lenses(mlcc_ctx *ctx, int64_t n, const double *x, const double *y,
                            const double *m, double kappa_s, double gamma)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    if (n < 1) return fail(MLCC_ERR_INVALID, "need at least one star (n=%lld)", (long long)n);
    if (n > (int64_t)1 << 28) return fail(MLCC_ERR_INVALID, "too many stars (%lld)", (long long)n);
    const int64_t off[2] = {0, n};
    return load_fields(ctx->impl, 1, off, x, y, m, &kappa_s, &gamma, false);
}

mlcc_status mlcc_set_lenses_batched(mlcc_ctx *ctx, int32_t n_fields, const int64_t *star_offsets,
                                    const double *x, const double *y, const double *m,
                                    const double *kappa_s, const double *gamma)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    if (!star_offsets || !kappa_s || !gamma)
        return fail(MLCC_ERR_INVALID, "star_offsets, kappa_s and gamma must be host arrays");
    if (n_fields < 1 || n_fields > 65536)
        return fail(MLCC_ERR_INVALID, "need 1..65536 fields (got %d)", n_fields);
    for (int32_t r = 0; r < n_fields; ++r)
        if (star_offsets[r + 1] - star_offsets[r] < 1 || star_offsets[r + 1] > ((int64_t)1 << 28))
            return fail(MLCC_ERR_INVALID, "star_offsets must start at 0 and strictly increase");
    return load_fields(ctx->impl, n_fields, star_offsets, x, y, m, kappa_s, gamma, true);
}

mlcc_status mlcc_find_critical_curves(mlcc_ctx *ctx, const mlcc_cc_params *params,
                                      double *roots_re, double *roots_im, double *caustics_re,
                                      double *caustics_im, int32_t *chain_next,
                                      mlcc_cc_stats *stats)
{
    if (!ctx || !params) return fail(MLCC_ERR_INVALID, "ctx or params is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    if (c.n < 1) return fail(MLCC_ERR_STATE, "call mlcc_set_lenses first");
    const mlcc_cc_params &p = *params;
    if (p.m_steps < 2 || (p.m_steps & 1))
        return fail(MLCC_ERR_INVALID, "m_steps must be even and >= 2 (got %lld)",
                    (long long)p.m_steps);
    if (p.m_steps > (int64_t)1 << 28) return fail(MLCC_ERR_INVALID, "m_steps too large");
    if (p.n_subchains < 0 || (p.n_subchains > 0 && (p.m_steps / 2) % p.n_subchains))
        return fail(MLCC_ERR_INVALID, "n_subchains=%d must divide m_steps/2=%lld",
                    p.n_subchains, (long long)(p.m_steps / 2));
    if (!(p.tol_step > 0) || !std::isfinite(p.tol_step))
        return fail(MLCC_ERR_INVALID, "tol_step must be positive and finite");
    if (!(p.tol_inv_mu >= 0) || !std::isfinite(p.tol_inv_mu))
        return fail(MLCC_ERR_INVALID, "tol_inv_mu must be >= 0 and finite");
    if (p.max_iter_cold < 0 || p.max_iter_warm < 0)
        return fail(MLCC_ERR_INVALID, "iteration caps must be >= 0");
    if (p.cold_restart_sweeps < 0)
        return fail(MLCC_ERR_INVALID, "cold_restart_sweeps must be >= 0");
    if (p.precision != MLCC_FP64 && p.precision != MLCC_MIXED && p.precision != MLCC_FP64_R32)
        return fail(MLCC_ERR_INVALID, "unknown precision %d", p.precision);
    if (p.predictor < 0 || p.predictor > 2)
        return fail(MLCC_ERR_INVALID, "predictor must be 0, 1 or 2 (got %d)", p.predictor);
    if (p.schedule != MLCC_SCHEDULE_ROUNDS && p.schedule != MLCC_SCHEDULE_PERSISTENT)
        return fail(MLCC_ERR_INVALID, "unknown schedule %d", p.schedule);
    if (p.watchdog_ms < 0 || p.watchdog_ms > 600000)
        return fail(MLCC_ERR_INVALID, "watchdog_ms=%d outside [0, 600000]", p.watchdog_ms);
    if (c.rect && p.precision == MLCC_MIXED)
        return fail(MLCC_ERR_INVALID, "a rectangular field is solved in the FP64 precisions only");
    if (p.star_sums != MLCC_STARS_DIRECT && p.star_sums != MLCC_STARS_FMM)
        return fail(MLCC_ERR_INVALID, "unknown star_sums %d", p.star_sums);
    if (p.fmm_order != 0 && (p.fmm_order < 8 || p.fmm_order > 63))
        return fail(MLCC_ERR_INVALID, "fmm_order must be 0 or 8..63 (got %d)", p.fmm_order);
    MLCC_TRY(check_device_ptr(&c, roots_re, "roots_re"));
    MLCC_TRY(check_device_ptr(&c, roots_im, "roots_im"));
    if ((caustics_re == nullptr) != (caustics_im == nullptr))
        return fail(MLCC_ERR_INVALID, "caustics_re and caustics_im must both be given or both NULL");
    if (caustics_re) {
        MLCC_TRY(check_device_ptr(&c, caustics_re, "caustics_re"));
        MLCC_TRY(check_device_ptr(&c, caustics_im, "caustics_im"));
    }
    if (chain_next) MLCC_TRY(check_device_ptr(&c, chain_next, "chain_next"));
    clear_error();
    return find_critical_curves_impl(&c, &p, roots_re, roots_im, caustics_re, caustics_im,
                                     chain_next, stats);
}

mlcc_status mlcc_find_critical_curves_batched(mlcc_ctx *ctx, const mlcc_cc_params *params,
                                              int64_t *root_offsets, double *roots_re,
                                              double *roots_im, double *caustics_re,
                                              double *caustics_im, int32_t *chain_next,
                                              mlcc_cc_stats *stats)
{
    if (!ctx || !params) return fail(MLCC_ERR_INVALID, "ctx or params is NULL");
    Ctx &c = ctx->impl;
    if (c.reals.empty()) return fail(MLCC_ERR_STATE, "call mlcc_set_lenses_batched first");
    if (root_offsets) {
        const int64_t rows = params->m_steps + 1;
        for (size_t r = 0; r < c.reals.size(); ++r)
            root_offsets[r] = rows * 2 * c.reals[r].star_off;
        root_offsets[c.reals.size()] = rows * 2 * c.n;
    }
    return mlcc_find_critical_curves(ctx, params, roots_re, roots_im, caustics_re, caustics_im,
                                     chain_next, stats);
}

mlcc_status mlcc_map_caustics(mlcc_ctx *ctx, int64_t count, const double *z_re,
                              const double *z_im, double *w_re, double *w_im)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    if (c.n < 1) return fail(MLCC_ERR_STATE, "call mlcc_set_lenses first");
    if (c.batched)
        return fail(MLCC_ERR_STATE, "mlcc_map_caustics needs a single field (mlcc_set_lenses)");
    if (count < 0) return fail(MLCC_ERR_INVALID, "count < 0");
    if (count == 0) return MLCC_OK;
    MLCC_TRY(check_device_ptr(&c, z_re, "z_re"));
    MLCC_TRY(check_device_ptr(&c, z_im, "z_im"));
    MLCC_TRY(check_device_ptr(&c, w_re, "w_re"));
    MLCC_TRY(check_device_ptr(&c, w_im, "w_im"));
    if (w_re == z_re || w_re == z_im || w_im == z_re || w_im == z_im)
        return fail(MLCC_ERR_INVALID, "w may not alias z");
    clear_error();
    return launch_map_caustics(&c, count, z_re, z_im, w_re, w_im);
}

mlcc_status mlcc_caustic_crossings(mlcc_ctx *ctx, int64_t rows, int64_t n_r, const double *w_re,
                                   const double *w_im, const int32_t *chain_next,
                                   const mlcc_grid *grid, int32_t *ncc)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    if (rows < 1 || n_r < 1) return fail(MLCC_ERR_INVALID, "need rows >= 1 and n_r >= 1");
    if (rows > ((int64_t)1 << 40) / n_r) return fail(MLCC_ERR_INVALID, "rows * n_r too large");
    MLCC_TRY(check_grid(grid, false));
    MLCC_TRY(check_device_ptr(&c, w_re, "w_re"));
    MLCC_TRY(check_device_ptr(&c, w_im, "w_im"));
    if (chain_next) MLCC_TRY(check_device_ptr(&c, chain_next, "chain_next"));
    MLCC_TRY(check_device_ptr(&c, ncc, "ncc"));
    clear_error();
    return run_caustic_crossings(&c, rows, n_r, w_re, w_im, chain_next, grid, ncc);
}

mlcc_status mlcc_caustic_crossings_noalloc(mlcc_ctx *ctx, int64_t rows, int64_t n_r,
                                           const double *w_re, const double *w_im,
                                           const int32_t *chain_next, const mlcc_grid *grid,
                                           int32_t *ncc)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    if (rows < 1 || n_r < 1) return fail(MLCC_ERR_INVALID, "need rows >= 1 and n_r >= 1");
    if (rows > ((int64_t)1 << 40) / n_r) return fail(MLCC_ERR_INVALID, "rows * n_r too large");
    MLCC_TRY(check_grid(grid, false));
    MLCC_TRY(check_device_ptr(&c, w_re, "w_re"));
    MLCC_TRY(check_device_ptr(&c, w_im, "w_im"));
    if (chain_next) MLCC_TRY(check_device_ptr(&c, chain_next, "chain_next"));
    MLCC_TRY(check_device_ptr(&c, ncc, "ncc"));
    clear_error();
    return run_caustic_crossings_noalloc(&c, rows, n_r, w_re, w_im, chain_next, grid, ncc);
}

mlcc_status mlcc_caustic_distances(mlcc_ctx *ctx, const mlcc_grid *grid, const int32_t *ncc,
                                   double *dist, uint8_t *border_limited)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    MLCC_TRY(check_grid(grid, true));
    MLCC_TRY(check_device_ptr(&c, ncc, "ncc"));
    MLCC_TRY(check_device_ptr(&c, dist, "dist"));
    if (border_limited) MLCC_TRY(check_device_ptr(&c, border_limited, "border_limited"));
    clear_error();
    return launch_caustic_distances(&c, grid, ncc, dist, border_limited);
}

mlcc_status mlcc_caustic_distances_directional(mlcc_ctx *ctx, const mlcc_grid *grid,
                                               const int32_t *ncc, double angle, double *dist,
                                               uint8_t *border_limited)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    MLCC_TRY(check_grid(grid, true));
    if (!std::isfinite(angle)) return fail(MLCC_ERR_INVALID, "angle must be finite");
    if ((int64_t)grid->nx + grid->ny > 1000000)
        return fail(MLCC_ERR_INVALID, "moving-source distances need nx + ny <= 10^6");
    MLCC_TRY(check_device_ptr(&c, ncc, "ncc"));
    MLCC_TRY(check_device_ptr(&c, dist, "dist"));
    if (border_limited) MLCC_TRY(check_device_ptr(&c, border_limited, "border_limited"));
    clear_error();
    return launch_directional_distances(&c, grid, ncc, angle, dist, border_limited);
}

mlcc_status mlcc_distance_histogram(mlcc_ctx *ctx, int64_t count, const double *dist,
                                    const uint8_t *border_limited, const int32_t *ncc,
                                    int32_t ncc_lo, int32_t n_classes, int32_t n_bins,
                                    double d_max, int64_t *counts)
{
    if (!ctx) return fail(MLCC_ERR_INVALID, "ctx is NULL");
    Ctx &c = ctx->impl;
    MLCC_TRY(use_device(&c));
    if (count < 0) return fail(MLCC_ERR_INVALID, "count < 0");
    if (n_bins < 1 || n_classes < 1 || (int64_t)n_classes * (n_bins + 1) > 8192)
        return fail(MLCC_ERR_INVALID, "need n_bins, n_classes >= 1 and n_classes * (n_bins + 1) "
                                      "<= 8192");
    if (!ncc && n_classes != 1) return fail(MLCC_ERR_INVALID, "n_classes must be 1 without ncc");
    if (!(d_max > 0) || !std::isfinite(d_max)) return fail(MLCC_ERR_INVALID, "d_max must be > 0");
    if (count > 0) {
        MLCC_TRY(check_device_ptr(&c, dist, "dist"));
        MLCC_TRY(check_device_ptr(&c, border_limited, "border_limited"));
        if (ncc) MLCC_TRY(check_device_ptr(&c, ncc, "ncc"));
    }
    MLCC_TRY(check_device_ptr(&c, counts, "counts"));
    clear_error();
    return launch_distance_histogram(&c, count, dist, border_limited, ncc, ncc_lo, n_classes,
                                     n_bins, d_max, counts);
}

} // extern "C"
