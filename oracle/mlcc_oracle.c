/*
 * mlcc_oracle.c -- plain, slow, CPU reference for the critical-curve /
 * caustic / caustic-crossing / distance-map path of
 * "A GPU Code for Finding Microlensing Critical Curves and Caustics"
 * (Weisenbach 2025, arXiv 2506.02121).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP path.  All arithmetic is IEEE double precision (C99 complex), with
 * OpenMP only over independent roots of one Jacobi sweep or independent
 * pixels.
 *
 * Model (paper Sec. 3.1, parametric critical-curve equation, together with
 * App. A: the compensating smooth sheet of a circular field extended to an
 * infinite sheet, so alpha_s(z) = -kappa_star z everywhere, d alpha_s/dz =
 * -kappa_star and d alpha_s/dzbar = 0):
 *
 *   F(z, phi) = gamma + sum_i m_i / (z - z_i)^2 - (1 - kappa_s) e^{-i phi}
 *   F'(z)     = -2 sum_i m_i / (z - z_i)^3
 *   w(z)      = (1 - kappa_s) z + gamma conj(z) - sum_i m_i / conj(z - z_i)
 *
 * with kappa_s = kappa - kappa_star and theta_star = 1.
 *
 * Parity pins for every function here live in tests/ (closed forms,
 * companion-matrix and multiprecision roots, Vieta identities, the vector
 * form of the lens equation, brute force, scipy's exact EDT).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum {
    ORC_OK = 0,
    ORC_ERR_INVALID = -1,
    ORC_ERR_NOT_CONVERGED = -4,
    ORC_ERR_NONFINITE = -6,
    ORC_ERR_MATCH = -7,
};

/* ---------------------------------------------------------------------- */
/* Model                                                                   */
/* ---------------------------------------------------------------------- */

/* The phase grid of Sec. 3.1 / Sec. 4.3: phi_j = 2 pi j / m_steps, rows
 * j = 0..m_steps (both 0 and 2 pi are kept). */
static double phase_of_row(int64_t j, int64_t m_steps)
{
    return (2.0 * M_PI * (double)j) / (double)m_steps;
}

/* (1 - kappa_s) e^{-i phi}: the phase term of the parametric equation. */
static cplx phase_term(double kappa_s, double phi)
{
    return (1.0 - kappa_s) * (cos(phi) - I * sin(phi));
}

typedef struct {
    int64_t n;
    const double *x, *y, *m;
    double kappa_s, gamma;
    /* NULL: the circular field with its sheet extended to infinity (App. A),
     * alpha_s = -kappa_star z.  Else a rectangular field (Sec. 4.2, App. B):
     * sheet = {kappa_star, c1, c2, t}, corner c = c1 + i c2, Taylor degree t
     * (odd), the sheet again extended to infinity (d alpha_s / dz =
     * -kappa_star) and the logarithms truncated at power t. */
    const double *sheet;
} Lens;

/* ---------------------------------------------------------------------- */
/* Rectangular field (Sec. 4.2, App. A, App. B)                             */
/* ---------------------------------------------------------------------- */

static int sheet_t(const double *sh) { return (int)sh[3]; }

/* Roots added by the sheet polynomial: t - 1 for odd t >= 3 (App. B: the
 * power-t term vanishes for odd t), none for t = 1. */
static int64_t sheet_extra_roots(const double *sh)
{
    if (!sh) return 0;
    int t = sheet_t(sh);
    return t >= 3 ? (int64_t)(t - 1) : 0;
}

/* d alpha_s / d zbar of App. B in its first closed form (with arctan):
 *   -kappa_star i / pi [ zbar^t (1 + (-1)^t) (c^-t - cbar^-t)
 *                        + sum_{j=1..t} zbar^j / j (1 + (-1)^j) (c^-j - cbar^-j) ]
 *   + kappa_star - 4 kappa_star arctan(c2 / c1) / pi,
 * and its derivative in zbar. */
static void sheet_dalpha_dzbar(const double *sh, cplx zb, cplx *d1, cplx *d2)
{
    double ks = sh[0];
    cplx c = sh[1] + I * sh[2], cb = conj(c);
    int t = sheet_t(sh);
    cplx acc = 0, accd = 0, zp = 1, zt1 = 1;   /* zp = zbar^(j-1) in the loop */
    for (int j = 1; j <= t; ++j) {
        double sgn = (j & 1) ? -1.0 : 1.0;
        cplx k = (1.0 + sgn) * (1.0 / cpow(c, j) - 1.0 / cpow(cb, j));
        acc += zp * zb / j * k;
        accd += zp * k;
        if (j == t) zt1 = zp;
        zp *= zb;
    }
    /* the separate power-t term; zp = zbar^t, zt1 = zbar^(t-1) */
    {
        double sgn = (t & 1) ? -1.0 : 1.0;
        cplx k = (1.0 + sgn) * (1.0 / cpow(c, t) - 1.0 / cpow(cb, t));
        acc += zp * k;
        accd += (double)t * zt1 * k;
    }
    *d1 = (-ks * I / M_PI) * acc + ks - 4.0 * ks * atan(sh[2] / sh[1]) / M_PI;
    if (d2) *d2 = (-ks * I / M_PI) * accd;
}

/* alpha_s of App. B: the four logarithms Taylor-expanded about the origin
 * and truncated at power t (exact = 0), or (exact = 1) summed in closed
 * form as log(a) + log(1 - zbar/a), the continuation of the series from the
 * origin, valid for |z| < |c|; plus -kappa_star (c + cbar + zbar + z). */
static cplx sheet_alpha(const double *sh, cplx z, int exact)
{
    double ks = sh[0];
    cplx c = sh[1] + I * sh[2];
    cplx zb = conj(z);
    int t = sheet_t(sh);
    cplx a[4] = {c, conj(c), -c, -conj(c)};
    double sgn[4] = {1.0, -1.0, 1.0, -1.0};
    cplx acc = 0;
    for (int q = 0; q < 4; ++q) {
        cplx lg;
        if (exact) {
            lg = clog(a[q]) + clog(1.0 - zb / a[q]);
        } else {
            cplx s = 0, p = 1;
            for (int j = 1; j <= t; ++j) {
                p *= zb / a[q];
                s += p / j;
            }
            lg = clog(a[q]) - s;
        }
        acc += sgn[q] * (a[q] - zb) * lg;
    }
    return (-ks * I / M_PI) * acc - ks * (c + conj(c) + zb + z);
}

/* Start values of the t - 1 extra roots: evenly spread on the circle through
 * the field's corners, |z| = |c|, at angles 2 pi (k + 1/2) / (t - 1). */
static void sheet_seeds(const double *sh, cplx *out)
{
    int64_t e = sheet_extra_roots(sh);
    double r = cabs(sh[1] + I * sh[2]);
    for (int64_t k = 0; k < e; ++k) {
        double a = 2.0 * M_PI * ((double)k + 0.5) / (double)e;
        out[k] = r * (cos(a) + I * sin(a));
    }
}

/* F, F' and S1 = sum 1/(z - z_i) at one point (Sec. 3.1 and Sec. 3.2). */
static void eval_F(const Lens *L, cplx e, cplx z, cplx *F, cplx *Fp, cplx *S1)
{
    cplx s1 = 0, s2 = 0, s3 = 0;
    for (int64_t i = 0; i < L->n; ++i) {
        cplx d = z - (L->x[i] + I * L->y[i]);
        cplx u = 1.0 / d;
        s1 += u;
        s2 += L->m[i] * u * u;
        s3 += L->m[i] * u * u * u;
    }
    *F = L->gamma + s2 - e;
    *Fp = -2.0 * s3;
    *S1 = s1;
    if (L->sheet) {
        /* F = gamma + sum m/(z - z_i)^2 - conj(d alpha_s/d zbar)
         *     - (1 - kappa - d alpha_s/dz) e^{-i phi}, with d alpha_s/dz =
         * -kappa_star, so the last factor is 1 - kappa_s as for the circle
         * (Sec. 3.1); conj(d alpha_s/d zbar) is a polynomial in z whose
         * z-derivative is conj of the zbar-derivative. */
        cplx d1, d2;
        sheet_dalpha_dzbar(L->sheet, conj(z), &d1, &d2);
        *F -= conj(d1);
        *Fp -= conj(d2);
    }
}

/* Neumaier-compensated complex accumulator, used where a sum of many terms
 * is the final output (the lens mapping). */
typedef struct { double s, c; } Neu;
static void neu_add(Neu *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* Lens equation in complex form (Sec. 3.1) with the infinite sheet (App. A):
 * w = (1 - kappa_s) z + gamma conj(z) - sum m_i / (conj(z) - conj(z_i)). */
static cplx lens_map(const Lens *L, cplx z)
{
    Neu sr = {0, 0}, si = {0, 0};
    for (int64_t i = 0; i < L->n; ++i) {
        cplx dbar = conj(z - (L->x[i] + I * L->y[i]));
        cplx t = L->m[i] / dbar;
        neu_add(&sr, creal(t));
        neu_add(&si, cimag(t));
    }
    cplx s = (sr.s + sr.c) + I * (si.s + si.c);
    if (L->sheet) {
        /* w = (1 - kappa) z + gamma conj(z) - sum - alpha_s(z), kappa =
         * kappa_s + kappa_star (Sec. 3.1), alpha_s the truncated App. B form */
        double kappa = L->kappa_s + L->sheet[0];
        return (1.0 - kappa) * z + L->gamma * conj(z) - s - sheet_alpha(L->sheet, z, 0);
    }
    return (1.0 - L->kappa_s) * z + L->gamma * conj(z) - s;
}

/* Inverse magnification (App. C, first line):
 * 1/mu = (1 - kappa_s)^2 - |gamma + sum m_i / conj(z - z_i)^2|^2. */
static double inv_mu(const Lens *L, cplx z)
{
    cplx s = 0;
    for (int64_t i = 0; i < L->n; ++i) {
        cplx dbar = conj(z - (L->x[i] + I * L->y[i]));
        s += L->m[i] / (dbar * dbar);
    }
    cplx g = L->gamma + s;
    if (L->sheet) {
        cplx d1;
        sheet_dalpha_dzbar(L->sheet, conj(z), &d1, NULL);
        g -= d1;   /* dw/dzbar = gamma + sum m/conj(z - z_i)^2 - d alpha_s/d zbar */
    }
    double a = 1.0 - L->kappa_s;
    return a * a - creal(g * conj(g));
}

static int lens_ok(const Lens *L)
{
    if (L->n < 1) return 0;
    for (int64_t i = 0; i < L->n; ++i)
        if (!isfinite(L->x[i]) || !isfinite(L->y[i]) || !isfinite(L->m[i]) || !(L->m[i] > 0))
            return 0;
    if (!isfinite(L->kappa_s) || !isfinite(L->gamma)) return 0;
    if (L->sheet) {
        const double *sh = L->sheet;
        int t = sheet_t(sh);
        if (!(sh[0] > 0) || !(sh[1] > 0) || !(sh[2] > 0) || t < 1 || !(t & 1) ||
            (double)t != sh[3])
            return 0;
        return 1;
    }
    /* c(phi) = gamma - (1 - kappa_s) e^{-i phi} vanishes on the grid when
     * |gamma| = |1 - kappa_s| (App. A footnote); reject that case. */
    if (fabs(fabs(L->gamma) - fabs(1.0 - L->kappa_s)) == 0.0) return 0;
    return 1;
}

int orc_eval_F(int64_t n, const double *x, const double *y, const double *m,
               double kappa_s, double gamma, const double *sheet, double phi,
               int64_t count,
               const double *zr, const double *zi,
               double *Fr, double *Fi, double *Fpr, double *Fpi)
{
    Lens L = {n, x, y, m, kappa_s, gamma, sheet};
    cplx e = phase_term(kappa_s, phi);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        cplx F, Fp, S1;
        eval_F(&L, e, zr[k] + I * zi[k], &F, &Fp, &S1);
        Fr[k] = creal(F); Fi[k] = cimag(F);
        Fpr[k] = creal(Fp); Fpi[k] = cimag(Fp);
    }
    return ORC_OK;
}

int orc_lens_map(int64_t n, const double *x, const double *y, const double *m,
                 double kappa_s, double gamma, const double *sheet, int64_t count,
                 const double *zr, const double *zi, double *wr, double *wi)
{
    Lens L = {n, x, y, m, kappa_s, gamma, sheet};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) {
        cplx w = lens_map(&L, zr[k] + I * zi[k]);
        wr[k] = creal(w); wi[k] = cimag(w);
    }
    return ORC_OK;
}

int orc_inv_mu(int64_t n, const double *x, const double *y, const double *m,
               double kappa_s, double gamma, const double *sheet, int64_t count,
               const double *zr, const double *zi, double *out)
{
    Lens L = {n, x, y, m, kappa_s, gamma, sheet};
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < count; ++k) out[k] = inv_mu(&L, zr[k] + I * zi[k]);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Root finding (Sec. 3.2)                                                 */
/* ---------------------------------------------------------------------- */

/* Cold-start seeds (Sec. 3.2): the star positions shifted by +1 and -1
 * (theta_star = 1) along the real axis; root 2i <- z_i + 1, 2i+1 <- z_i - 1.
 * With the infinite sheet there are exactly n_r = 2N roots.  A rectangular
 * field adds t - 1 roots (App. B), seeded on a circle around the stars
 * (Sec. 3.2), roots 2N .. 2N + t - 2. */
int orc_seeds(int64_t n, const double *x, const double *y, const double *sheet, double *zr,
              double *zi)
{
    for (int64_t i = 0; i < n; ++i) {
        zr[2 * i] = x[i] + 1.0; zi[2 * i] = y[i];
        zr[2 * i + 1] = x[i] - 1.0; zi[2 * i + 1] = y[i];
    }
    int64_t e = sheet_extra_roots(sheet);
    if (e) {
        cplx *ex = malloc(sizeof(cplx) * e);
        sheet_seeds(sheet, ex);
        for (int64_t k = 0; k < e; ++k) { zr[2 * n + k] = creal(ex[k]); zi[2 * n + k] = cimag(ex[k]); }
        free(ex);
    }
    return ORC_OK;
}

/* App. B for callers: d alpha_s / d zbar, and alpha_s truncated (exact = 0)
 * or summed in closed form (exact = 1), at `count` points. */
int orc_rect_dalpha(const double *sheet, int64_t count, const double *zr, const double *zi,
                    double *dr, double *di)
{
    for (int64_t k = 0; k < count; ++k) {
        cplx d1;
        sheet_dalpha_dzbar(sheet, zr[k] - I * zi[k], &d1, NULL);
        dr[k] = creal(d1); di[k] = cimag(d1);
    }
    return ORC_OK;
}

int orc_rect_alpha(const double *sheet, int exact, int64_t count, const double *zr,
                   const double *zi, double *ar, double *ai)
{
    for (int64_t k = 0; k < count; ++k) {
        cplx a = sheet_alpha(sheet, zr[k] + I * zi[k], exact);
        ar[k] = creal(a); ai[k] = cimag(a);
    }
    return ORC_OK;
}

/* Taylor degree for a rectangular field (App. B): the smallest t whose
 * truncation bound (kappa_star / pi) (4 / (t + 1)) s^-(t+1) |c| (s + 1)/(s - 1)
 * is at most eps (for |z| s < |c|), made odd, then raised by 2 until
 * (t - 1) Arg(c) mod pi lies at least 10% of pi away from 0 and from pi.
 * Returns -1 for invalid arguments. */
int orc_rect_taylor_degree(double kappa_star, double c1, double c2, double s, double eps)
{
    if (!(kappa_star > 0) || !(c1 > 0) || !(c2 > 0) || !(s > 1) || !(eps > 0)) return -1;
    double ac = hypot(c1, c2), th = atan2(c2, c1);
    int t = 1;
    while (kappa_star / M_PI * 4.0 / (t + 1) * pow(s, -(t + 1)) * ac * (s + 1) / (s - 1) > eps) {
        if (++t > 100000) return -1;
    }
    if (!(t & 1)) ++t;
    for (int guard = 0; guard < 100000; ++guard, t += 2) {
        double r = fmod((t - 1) * th, M_PI);
        if (r >= 0.1 * M_PI && r <= 0.9 * M_PI) return t;
    }
    return -1;
}

/* Number of roots per phase: 2N, plus t - 1 for a rectangular field. */
int64_t orc_num_roots(int64_t n, const double *sheet)
{
    return 2 * n + sheet_extra_roots(sheet);
}

/* One Aberth-Ehrlich solve for one phase (Sec. 3.2).
 *
 * Every sweep applies, to every root not yet flagged and all at once from
 * the previous iterate (a Jacobi sweep),
 *     z_k <- z_k - 1 / ( P'/P(z_k) - sum_{r != k} 1/(z_k - z_r) ),
 *     P'/P = F'/F + 2 sum_i 1/(z - z_i),
 * and flags the root when the step is below tol_step or when the App. C
 * bound |F| (|F| + 2 |1 - kappa_s|) on |1/mu| (evaluated at the iterate the
 * step started from) is below tol_mu.  The solve stops when every root is
 * flagged.  Flagged roots keep the value of the step that flagged them.
 *
 * After convergence, when `polish` is set, each root takes up to three
 * Newton steps z <- z - F/F' while the step keeps shrinking: the oracle's own
 * refinement toward the exact zero, so that its error is far below the
 * tolerance the GPU path is held to.
 */
int orc_aberth_row(int64_t n, const double *x, const double *y, const double *m,
                   double kappa_s, double gamma, const double *sheet, double phi, int64_t n_r,
                   double *zr, double *zi, double tol_step, double tol_mu,
                   int64_t max_iter, int polish, int64_t *sweeps_out,
                   int64_t *updates_out)
{
    Lens L = {n, x, y, m, kappa_s, gamma, sheet};
    if (!lens_ok(&L) || n_r < 1) return ORC_ERR_INVALID;
    cplx e = phase_term(kappa_s, phi);
    double a1 = fabs(1.0 - kappa_s);
    cplx *z = malloc(sizeof(cplx) * n_r), *zn = malloc(sizeof(cplx) * n_r);
    unsigned char *done = calloc(n_r, 1);
    for (int64_t k = 0; k < n_r; ++k) z[k] = zr[k] + I * zi[k];
    int64_t sweeps = 0, updates = 0;
    int status = ORC_OK;
    for (;;) {
        int64_t active = 0;
        for (int64_t k = 0; k < n_r; ++k) active += !done[k];
        if (active == 0) break;
        if (sweeps >= max_iter) { status = ORC_ERR_NOT_CONVERGED; break; }
        int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
        for (int64_t k = 0; k < n_r; ++k) {
            if (done[k]) { zn[k] = z[k]; continue; }
            cplx F, Fp, S1;
            eval_F(&L, e, z[k], &F, &Fp, &S1);
            cplx R = 0;
            for (int64_t r = 0; r < n_r; ++r)
                if (r != k) R += 1.0 / (z[k] - z[r]);
            cplx step;
            if (F == 0) {
                step = 0;
            } else {
                cplx dlogP = Fp / F + 2.0 * S1;
                step = 1.0 / (dlogP - R);
            }
            zn[k] = z[k] - step;
            double aF = cabs(F);
            if (cabs(zn[k] - z[k]) < tol_step || aF * (aF + 2.0 * a1) < tol_mu) done[k] = 1;
            if (!isfinite(creal(zn[k])) || !isfinite(cimag(zn[k]))) bad = 1;
        }
        updates += active;
        ++sweeps;
        cplx *t = z; z = zn; zn = t;
        if (bad) { status = ORC_ERR_NONFINITE; break; }
    }
    if (status == ORC_OK && polish) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int64_t k = 0; k < n_r; ++k) {
            double prev = INFINITY;
            for (int t = 0; t < 3; ++t) {
                cplx F, Fp, S1;
                eval_F(&L, e, z[k], &F, &Fp, &S1);
                if (F == 0) break;
                cplx s = F / Fp;
                double as = cabs(s);
                if (!(as < prev)) break;
                z[k] -= s;
                prev = as;
            }
        }
    }
    for (int64_t k = 0; k < n_r; ++k) { zr[k] = creal(z[k]); zi[k] = cimag(z[k]); }
    if (sweeps_out) *sweeps_out = sweeps;
    if (updates_out) *updates_out = updates;
    free(z); free(zn); free(done);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Chains (Sec. 4.3)                                                        */
/* ---------------------------------------------------------------------- */

/* One subchain: cold start at row `center`, then grow toward row `lo` and
 * toward row `hi`, each new row seeded with the converged roots of its
 * neighbour (Sec. 3.2 warm start, Sec. 4.3 centre-out growth).  Writes rows
 * lo..hi into out (row-major, (hi - lo + 1) x 2N).  stats: [0] sweeps,
 * [1] root updates, [2] rows that hit the iteration cap, [3] max sweeps in a
 * warm row, [4] sweeps of the cold start. */
int orc_subchain(int64_t n, const double *x, const double *y, const double *m,
                 double kappa_s, double gamma, const double *sheet, int64_t m_steps, int64_t lo,
                 int64_t center, int64_t hi, double tol_step, double tol_mu,
                 int64_t max_iter_cold, int64_t max_iter_warm, int polish,
                 double *out_re, double *out_im, int64_t *stats)
{
    int64_t n_r = orc_num_roots(n, sheet);
    if (lo > center || center > hi || lo < 0 || hi > m_steps) return ORC_ERR_INVALID;
    int64_t st[5] = {0, 0, 0, 0, 0};
    double *cr = out_re + (center - lo) * n_r, *ci = out_im + (center - lo) * n_r;
    orc_seeds(n, x, y, sheet, cr, ci);
    int64_t sw, up;
    int rc = orc_aberth_row(n, x, y, m, kappa_s, gamma, sheet, phase_of_row(center, m_steps), n_r,
                            cr, ci, tol_step, tol_mu, max_iter_cold, polish, &sw, &up);
    st[0] += sw; st[1] += up; st[4] = sw;
    if (rc == ORC_ERR_NOT_CONVERGED) st[2]++;
    else if (rc != ORC_OK) return rc;
    for (int dir = -1; dir <= 1; dir += 2) {
        int64_t end = dir < 0 ? lo : hi;
        for (int64_t j = center + dir; dir < 0 ? j >= end : j <= end; j += dir) {
            double *pr = out_re + (j - dir - lo) * n_r, *pi = out_im + (j - dir - lo) * n_r;
            double *rr = out_re + (j - lo) * n_r, *ri = out_im + (j - lo) * n_r;
            memcpy(rr, pr, sizeof(double) * n_r);
            memcpy(ri, pi, sizeof(double) * n_r);
            rc = orc_aberth_row(n, x, y, m, kappa_s, gamma, sheet, phase_of_row(j, m_steps), n_r,
                                rr, ri, tol_step, tol_mu, max_iter_warm, polish, &sw, &up);
            st[0] += sw; st[1] += up;
            if (sw > st[3]) st[3] = sw;
            if (rc == ORC_ERR_NOT_CONVERGED) st[2]++;
            else if (rc != ORC_OK) return rc;
        }
    }
    if (stats) memcpy(stats, st, sizeof st);
    return st[2] ? ORC_ERR_NOT_CONVERGED : ORC_OK;
}

/* Nearest-neighbour bijection between two copies of one root set (the same
 * phase computed twice).  perm[k] = index in b of the point nearest a[k].
 * Fails when the map is not one-to-one.  maxdist receives the largest
 * matched distance. */
int orc_match(int64_t n, const double *ar, const double *ai, const double *br,
              const double *bi, int32_t *perm, double *maxdist)
{
    double md = 0.0;
#pragma omp parallel for schedule(static) reduction(max : md)
    for (int64_t k = 0; k < n; ++k) {
        double best = INFINITY;
        int64_t bj = -1;
        for (int64_t j = 0; j < n; ++j) {
            double dx = ar[k] - br[j], dy = ai[k] - bi[j];
            double d = dx * dx + dy * dy;
            if (d < best) { best = d; bj = j; }
        }
        perm[k] = (int32_t)bj;
        if (sqrt(best) > md) md = sqrt(best);
    }
    unsigned char *used = calloc(n, 1);
    int ok = 1;
    for (int64_t k = 0; k < n; ++k) {
        if (perm[k] < 0 || used[perm[k]]) { ok = 0; break; }
        used[perm[k]] = 1;
    }
    free(used);
    if (maxdist) *maxdist = md;
    return ok ? ORC_OK : ORC_ERR_MATCH;
}

/* The whole (m_steps + 1) x 2N matrix of Sec. 4.3: n_sub subchains over
 * [0, 2 pi], subchain s covering rows [s L, (s+1) L] with L = m_steps/n_sub
 * (even), grown from its centre row s L + L/2.  A boundary row shared by two
 * subchains is kept from the lower one; the upper subchain's columns are
 * relabelled through the nearest-neighbour bijection of the two copies, so
 * that column k is one continuous chain over rows 0..m_steps.
 * chain_next[k] = column of row 0 matching row m_steps, column k (phase 2 pi
 * equals phase 0, so the two rows hold the same roots): the start of one
 * chain is the end of another.  stats: as orc_subchain, summed. */
int orc_critical_curves(int64_t n, const double *x, const double *y, const double *m,
                        double kappa_s, double gamma, const double *sheet, int64_t m_steps,
                        int64_t n_sub,
                        double tol_step, double tol_mu, int64_t max_iter_cold,
                        int64_t max_iter_warm, int polish, double *roots_re,
                        double *roots_im, int32_t *chain_next, int64_t *stats,
                        double *match_maxdist)
{
    if (m_steps < 2 || (m_steps & 1) || n_sub < 1 || (m_steps / 2) % n_sub) return ORC_ERR_INVALID;
    int64_t n_r = orc_num_roots(n, sheet), L = m_steps / n_sub;
    int64_t tot[5] = {0, 0, 0, 0, 0};
    double md = 0.0;
    double *br = malloc(sizeof(double) * (L + 1) * n_r), *bi = malloc(sizeof(double) * (L + 1) * n_r);
    int32_t *perm = malloc(sizeof(int32_t) * n_r);
    int status = ORC_OK;
    for (int64_t s = 0; s < n_sub; ++s) {
        int64_t lo = s * L, hi = lo + L, c = lo + L / 2;
        int64_t st[5];
        int rc = orc_subchain(n, x, y, m, kappa_s, gamma, sheet, m_steps, lo, c, hi, tol_step,
                              tol_mu,
                              max_iter_cold, max_iter_warm, polish, br, bi, st);
        for (int q = 0; q < 3; ++q) tot[q] += st[q];
        if (st[3] > tot[3]) tot[3] = st[3];
        if (st[4] > tot[4]) tot[4] = st[4];
        if (rc == ORC_ERR_NOT_CONVERGED) status = rc;
        else if (rc != ORC_OK) { status = rc; goto out; }
        if (s == 0) {
            memcpy(roots_re, br, sizeof(double) * (L + 1) * n_r);
            memcpy(roots_im, bi, sizeof(double) * (L + 1) * n_r);
            continue;
        }
        /* perm[k]: column of the stored boundary row matching this
         * subchain's column k. */
        double d;
        rc = orc_match(n_r, br, bi, roots_re + lo * n_r, roots_im + lo * n_r, perm, &d);
        if (d > md) md = d;
        if (rc != ORC_OK) { status = rc; goto out; }
        for (int64_t j = lo + 1; j <= hi; ++j)
            for (int64_t k = 0; k < n_r; ++k) {
                roots_re[j * n_r + perm[k]] = br[(j - lo) * n_r + k];
                roots_im[j * n_r + perm[k]] = bi[(j - lo) * n_r + k];
            }
    }
    if (chain_next) {
        double d;
        int rc = orc_match(n_r, roots_re + m_steps * n_r, roots_im + m_steps * n_r,
                           roots_re, roots_im, chain_next, &d);
        if (d > md) md = d;
        if (rc != ORC_OK) status = rc;
    }
out:
    if (stats) memcpy(stats, tot, sizeof tot);
    if (match_maxdist) *match_maxdist = md;
    free(br); free(bi); free(perm);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Caustic crossings (Sec. 5.1)                                            */
/* ---------------------------------------------------------------------- */

/* The caustics are oriented polygons (clockwise, Sec. 5.1).  N_cc at a pixel
 * centre p is the winding number (Sunday's crossing rule) of those polygons
 * about p, signed so that a clockwise loop around p counts +1: along the
 * horizontal ray from p toward -x, every edge crossing contributes +1 if the
 * edge runs upward and -1 if it runs downward.  Half-open rule: an edge
 * covers the heights Y_lo <= Y < Y_hi of its lower and upper end; a crossing
 * counts when it lies strictly left of p.
 *
 * Exactness: vertices are put on a fixed-point lattice with QBITS bits per
 * pixel, X = rint((x - x0) / hx * 2^QBITS), the same for y; pixel centres
 * are the lattice points ((2c+1) 2^(QBITS-1), (2r+1) 2^(QBITS-1)); all tests
 * are then integer (128-bit) arithmetic. */
#define QBITS 24
#define QLIMIT 9007199254740992.0 /* 2^53: beyond it the lattice is not exact */

typedef struct { int64_t X, Y; } Pt;
typedef __int128 i128;

static int quantise(double v, double v0, double h, int64_t *q)
{
    double s = (v - v0) / h * 16777216.0; /* 2^QBITS */
    if (!isfinite(s) || fabs(s) >= QLIMIT) return 0;
    *q = (int64_t)rint(s);
    return 1;
}

typedef struct {
    double x0, y0, hx, hy;
    int64_t nx, ny;
} PixGrid;

static int make_grid(double cx, double cy, double hw, double hh, int64_t nx, int64_t ny, PixGrid *g)
{
    if (nx < 1 || ny < 1 || !(hw > 0) || !(hh > 0)) return 0;
    g->x0 = cx - hw; g->y0 = cy - hh;
    g->hx = (2.0 * hw) / (double)nx; g->hy = (2.0 * hh) / (double)ny;
    g->nx = nx; g->ny = ny;
    return 1;
}

/* Edge e of the polygon set, as a pair of lattice points: for e < (rows-1)
 * n_r it is (row j, col k) -> (row j+1, col k) with e = j n_r + k; the last
 * n_r edges close the chains, (rows-1, k) -> (0, chain_next[k]) (identity
 * when chain_next is NULL).  Returns 0 on a vertex that cannot be put on the
 * lattice exactly or a bad chain_next entry. */
static int edge_at(int64_t e, int64_t rows, int64_t n_r, const double *wr, const double *wi,
                   const int32_t *chain_next, const PixGrid *g, Pt *a, Pt *b)
{
    int64_t j = e / n_r, k = e % n_r, j2, k2;
    if (j + 1 < rows) { j2 = j + 1; k2 = k; }
    else { j2 = 0; k2 = chain_next ? chain_next[k] : k; }
    if (k2 < 0 || k2 >= n_r) return 0;
    return quantise(wr[j * n_r + k], g->x0, g->hx, &a->X) &&
           quantise(wi[j * n_r + k], g->y0, g->hy, &a->Y) &&
           quantise(wr[j2 * n_r + k2], g->x0, g->hx, &b->X) &&
           quantise(wi[j2 * n_r + k2], g->y0, g->hy, &b->Y);
}

/* Contribution of edge a->b to the winding count of lattice point p. */
static int edge_term(Pt a, Pt b, Pt p)
{
    if (a.Y == b.Y) return 0;
    i128 cr = (i128)(b.X - a.X) * (p.Y - a.Y) - (i128)(b.Y - a.Y) * (p.X - a.X);
    if (a.Y <= p.Y && p.Y < b.Y) return cr < 0 ? 1 : 0;   /* upward, p right of edge */
    if (b.Y <= p.Y && p.Y < a.Y) return cr > 0 ? -1 : 0;  /* downward, p right of edge */
    return 0;
}

/* N_cc by the definition: every pixel against every edge. */
int orc_ncc_pixels(int64_t rows, int64_t n_r, const double *wr, const double *wi,
                   const int32_t *chain_next, double cx, double cy, double hw, double hh,
                   int64_t nx, int64_t ny, int32_t *ncc)
{
    PixGrid g;
    if (!make_grid(cx, cy, hw, hh, nx, ny, &g) || rows < 1 || n_r < 1) return ORC_ERR_INVALID;
    int64_t ne = rows * n_r;
    Pt *a = malloc(sizeof(Pt) * ne), *b = malloc(sizeof(Pt) * ne);
    for (int64_t e = 0; e < ne; ++e)
        if (!edge_at(e, rows, n_r, wr, wi, chain_next, &g, &a[e], &b[e])) {
            free(a); free(b);
            return ORC_ERR_INVALID;
        }
    const int64_t H = (int64_t)1 << (QBITS - 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c) {
            Pt p = {(2 * c + 1) * H, (2 * r + 1) * H};
            int64_t w = 0;
            for (int64_t e = 0; e < ne; ++e) w += edge_term(a[e], b[e], p);
            ncc[r * nx + c] = (int32_t)w;
        }
    free(a); free(b);
    return ORC_OK;
}

/* N_cc at a list of pixels only (same definition, edges streamed), for spot
 * checks of big maps. */
int orc_ncc_at(int64_t rows, int64_t n_r, const double *wr, const double *wi,
               const int32_t *chain_next, double cx, double cy, double hw, double hh,
               int64_t nx, int64_t ny, int64_t count, const int64_t *pix_r,
               const int64_t *pix_c, int64_t *out)
{
    PixGrid g;
    if (!make_grid(cx, cy, hw, hh, nx, ny, &g) || rows < 1 || n_r < 1) return ORC_ERR_INVALID;
    const int64_t H = (int64_t)1 << (QBITS - 1);
    int64_t ne = rows * n_r;
    int bad = 0;
    for (int64_t q = 0; q < count; ++q) out[q] = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        Pt a, b;
        if (!edge_at(e, rows, n_r, wr, wi, chain_next, &g, &a, &b)) { bad = 1; continue; }
        for (int64_t q = 0; q < count; ++q) {
            Pt p = {(2 * pix_c[q] + 1) * H, (2 * pix_r[q] + 1) * H};
            int t = edge_term(a, b, p);
            if (t) {
#pragma omp atomic
                out[q] += t;
            }
        }
    }
    return bad ? ORC_ERR_INVALID : ORC_OK;
}

static int64_t floor_div(i128 a, i128 b) /* b > 0 */
{
    i128 q = a / b;
    if ((a % b) != 0 && a < 0) --q;
    return (int64_t)q;
}

/* The same map built edge by edge (the paper's footnote to Sec. 5.1: loop
 * over the caustic segments and find the pixels each one affects).  For each
 * pixel row an edge crosses, the exact first column whose centre lies
 * strictly right of the crossing gets the edge's sign in a per-row
 * difference array; a running sum along each row gives N_cc. */
int orc_ncc_rows(int64_t rows, int64_t n_r, const double *wr, const double *wi,
                 const int32_t *chain_next, double cx, double cy, double hw, double hh,
                 int64_t nx, int64_t ny, int32_t *ncc)
{
    PixGrid g;
    if (!make_grid(cx, cy, hw, hh, nx, ny, &g) || rows < 1 || n_r < 1) return ORC_ERR_INVALID;
    int64_t ne = rows * n_r;
    int64_t *diff = calloc((size_t)(nx + 1) * ny, sizeof(int64_t));
    const int64_t H = (int64_t)1 << (QBITS - 1);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t e = 0; e < ne; ++e) {
        Pt lo, hi;
        if (!edge_at(e, rows, n_r, wr, wi, chain_next, &g, &lo, &hi)) { bad = 1; continue; }
        int s = 1;
        if (lo.Y == hi.Y) continue;
        if (lo.Y > hi.Y) { Pt t = lo; lo = hi; hi = t; s = -1; }
        /* rows r whose centre height (2r+1) H lies in [lo.Y, hi.Y) */
        int64_t r = floor_div((i128)lo.Y, (i128)2 * H) - 1;
        if (r < 0) r = 0;
        for (; r < ny; ++r) {
            int64_t Yr = (2 * r + 1) * H;
            if (Yr >= hi.Y) break;
            if (Yr < lo.Y) continue;
            i128 dy = (i128)(hi.Y - lo.Y), dx = (i128)(hi.X - lo.X);
            /* crossing x = num / dy; first c with (2c+1) H dy > num */
            i128 num = (i128)lo.X * dy + (i128)(Yr - lo.Y) * dx;
            int64_t q = floor_div(num, (i128)H * dy);
            int64_t c = floor_div((i128)q + 1, 2);
            if (c < 0) c = 0;
            if (c < nx) {
#pragma omp atomic
                diff[r * (nx + 1) + c] += s;
            }
        }
    }
    for (int64_t r = 0; r < ny; ++r) {
        int64_t acc = 0;
        for (int64_t c = 0; c < nx; ++c) {
            acc += diff[r * (nx + 1) + c];
            ncc[r * nx + c] = (int32_t)acc;
        }
    }
    free(diff);
    return bad ? ORC_ERR_INVALID : ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Distance to the nearest caustic (Sec. 5.2, expanding source)            */
/* ---------------------------------------------------------------------- */

/* A caustic pixel is one with a 4-neighbour inside the map whose N_cc
 * differs; the map border is not a caustic. */
int orc_caustic_mask(int64_t nx, int64_t ny, const int32_t *ncc, uint8_t *mask)
{
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c) {
            int32_t v = ncc[r * nx + c];
            int f = 0;
            if (c > 0 && ncc[r * nx + c - 1] != v) f = 1;
            if (c + 1 < nx && ncc[r * nx + c + 1] != v) f = 1;
            if (r > 0 && ncc[(r - 1) * nx + c] != v) f = 1;
            if (r + 1 < ny && ncc[(r + 1) * nx + c] != v) f = 1;
            mask[r * nx + c] = (uint8_t)f;
        }
    return ORC_OK;
}

static void finish_distance(int64_t nx, int64_t ny, const int64_t *d2, double h,
                            double *dist, uint8_t *border_limited)
{
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c) {
            int64_t v = d2[r * nx + c];
            dist[r * nx + c] = v < 0 ? INFINITY : sqrt((double)v) * h;
            if (border_limited) {
                /* twice the distance (in pixels) from the centre to the
                 * nearest map edge */
                int64_t bb = 2 * c + 1;
                if (2 * (nx - c) - 1 < bb) bb = 2 * (nx - c) - 1;
                if (2 * r + 1 < bb) bb = 2 * r + 1;
                if (2 * (ny - r) - 1 < bb) bb = 2 * (ny - r) - 1;
                border_limited[r * nx + c] = (uint8_t)(v < 0 || 4 * v > bb * bb);
            }
        }
}

/* Exact Euclidean distance transform by brute force: every pixel against
 * every caustic pixel, in integer squared pixel distances. */
int orc_edt_brute(int64_t nx, int64_t ny, const int32_t *ncc, double h, double *dist,
                  uint8_t *border_limited, int64_t *d2_out)
{
    uint8_t *mask = malloc((size_t)nx * ny);
    orc_caustic_mask(nx, ny, ncc, mask);
    int64_t nm = 0;
    for (int64_t p = 0; p < nx * ny; ++p) nm += mask[p];
    int64_t *mr = malloc(sizeof(int64_t) * (nm + 1)), *mc = malloc(sizeof(int64_t) * (nm + 1));
    nm = 0;
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c)
            if (mask[r * nx + c]) { mr[nm] = r; mc[nm] = c; ++nm; }
    int64_t *d2 = malloc(sizeof(int64_t) * nx * ny);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < nx * ny; ++p) {
        int64_t r = p / nx, c = p % nx, best = -1;
        for (int64_t q = 0; q < nm; ++q) {
            int64_t d = (r - mr[q]) * (r - mr[q]) + (c - mc[q]) * (c - mc[q]);
            if (best < 0 || d < best) best = d;
        }
        d2[p] = best;
    }
    finish_distance(nx, ny, d2, h, dist, border_limited);
    if (d2_out) memcpy(d2_out, d2, sizeof(int64_t) * nx * ny);
    free(mask); free(mr); free(mc); free(d2);
    return ORC_OK;
}

/* The same transform in two passes, for maps too big for brute force:
 * min over (r', c') of (r - r')^2 + (c - c')^2 = min over c' of
 * [(c - c')^2 + (min over r' in column c' of (r - r')^2)]. */
int orc_edt_twopass(int64_t nx, int64_t ny, const int32_t *ncc, double h, double *dist,
                    uint8_t *border_limited, int64_t *d2_out)
{
    uint8_t *mask = malloc((size_t)nx * ny);
    orc_caustic_mask(nx, ny, ncc, mask);
    int64_t *col = malloc(sizeof(int64_t) * nx * ny); /* column distance, -1 = none */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nx; ++c)
        for (int64_t r = 0; r < ny; ++r) {
            int64_t best = -1;
            for (int64_t r2 = 0; r2 < ny; ++r2)
                if (mask[r2 * nx + c]) {
                    int64_t d = r > r2 ? r - r2 : r2 - r;
                    if (best < 0 || d < best) best = d;
                }
            col[r * nx + c] = best;
        }
    int64_t *d2 = malloc(sizeof(int64_t) * nx * ny);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c) {
            int64_t best = -1;
            for (int64_t c2 = 0; c2 < nx; ++c2) {
                int64_t g = col[r * nx + c2];
                if (g < 0) continue;
                int64_t d = (c - c2) * (c - c2) + g * g;
                if (best < 0 || d < best) best = d;
            }
            d2[r * nx + c] = best;
        }
    finish_distance(nx, ny, d2, h, dist, border_limited);
    if (d2_out) memcpy(d2_out, d2, sizeof(int64_t) * nx * ny);
    free(mask); free(col); free(d2);
    return ORC_OK;
}

/* ---------------------------------------------------------------------- */
/* Moving source (Sec. 5.2, Figs. 5 bottom, 6, 7)                           */
/* ---------------------------------------------------------------------- */

/* Distance a source moving from the centre of pixel p along (ca, sa) (a unit
 * vector; angle from the +y1 axis) travels before its centre enters a
 * caustic pixel (a pixel with a 4-neighbour of different N_cc, as for the
 * expanding source), in units of the pixel size h: the entry parameter of
 * the ray into the pixel's square, the largest of its two near-slab
 * crossings, taken over every caustic pixel whose square the ray passes
 * through (strictly: a ray that only touches a corner does not enter).  0 on
 * a caustic pixel.  If none is entered, the ray's exit from the map and
 * border_limited = 1 (the map border is not a caustic, Fig. 5 caption).
 * Brute force over all caustic pixels; each parameter is one division of an
 * exact half-integer offset. */
static double slab(double lo, double hi, double p, double c, double *tfar)
{
    /* near and far crossing of lo <= p + t c <= hi */
    if (c == 0.0) {
        *tfar = (p > lo && p < hi) ? INFINITY : -INFINITY;
        return (p > lo && p < hi) ? -INFINITY : INFINITY;
    }
    double t1 = (lo - p) / c, t2 = (hi - p) / c;
    *tfar = t1 > t2 ? t1 : t2;
    return t1 < t2 ? t1 : t2;
}

int orc_directional_distance(int64_t nx, int64_t ny, const int32_t *ncc, double h, double ca,
                             double sa, double *dist, uint8_t *border_limited)
{
    if (nx < 1 || ny < 1 || !(h > 0)) return ORC_ERR_INVALID;
    uint8_t *mask = malloc((size_t)(nx * ny));
    orc_caustic_mask(nx, ny, ncc, mask);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < ny; ++r)
        for (int64_t c = 0; c < nx; ++c) {
            const int64_t i = r * nx + c;
            if (mask[i]) { dist[i] = 0.0; border_limited[i] = 0; continue; }
            double best = INFINITY;
            for (int64_t qr = 0; qr < ny; ++qr)
                for (int64_t qc = 0; qc < nx; ++qc) {
                    if (!mask[qr * nx + qc]) continue;
                    double fx, fy;
                    /* the square of pixel q, relative to p's centre */
                    double nxp = slab((double)(qc - c) - 0.5, (double)(qc - c) + 0.5, 0.0, ca, &fx);
                    double nyp = slab((double)(qr - r) - 0.5, (double)(qr - r) + 0.5, 0.0, sa, &fy);
                    double tn = nxp > nyp ? nxp : nyp, tf = fx < fy ? fx : fy;
                    if (tn < tf && tf > 0.0 && tn >= 0.0 && tn < best) best = tn;
                }
            if (best < INFINITY) {
                dist[i] = best * h;
                border_limited[i] = 0;
            } else {
                /* exit from the map [-1/2, nx - 1/2] x [-1/2, ny - 1/2] */
                double fx, fy;
                slab(-0.5 - (double)c, (double)(nx - c) - 0.5, 0.0, ca, &fx);
                slab(-0.5 - (double)r, (double)(ny - r) - 0.5, 0.0, sa, &fy);
                dist[i] = (fx < fy ? fx : fy) * h;
                border_limited[i] = 1;
            }
        }
    free(mask);
    return ORC_OK;
}

/* Histogram of distances (Figs. 6, 7): pixels not border-limited, bin
 * k = floor(d * inv_w) for d * inv_w < n_bins, else the overflow bin n_bins;
 * with ncc given, one row of n_bins + 1 counts per N_cc class ncc_lo ..
 * ncc_lo + n_classes - 1 (pixels of other classes are not counted). */
int orc_distance_histogram(int64_t npix, const double *dist, const uint8_t *border_limited,
                           const int32_t *ncc, int32_t ncc_lo, int32_t n_classes, int32_t n_bins,
                           double inv_w, int64_t *counts)
{
    if (n_bins < 1 || n_classes < 1 || !(inv_w > 0)) return ORC_ERR_INVALID;
    memset(counts, 0, sizeof(int64_t) * (size_t)n_classes * (size_t)(n_bins + 1));
    for (int64_t i = 0; i < npix; ++i) {
        if (border_limited[i]) continue;
        int64_t cls = 0;
        if (ncc) {
            cls = (int64_t)ncc[i] - ncc_lo;
            if (cls < 0 || cls >= n_classes) continue;
        }
        double x = dist[i] * inv_w;
        int64_t k = x < (double)n_bins ? (int64_t)floor(x) : n_bins;
        counts[cls * (n_bins + 1) + k] += 1;
    }
    return ORC_OK;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later parallel regions (n >= 1); returns the number in effect. */
int orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
