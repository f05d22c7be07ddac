/*
 * mlcc.h -- C-ABI of the MI355X (gfx950) library that finds microlensing
 * critical curves and caustics and reduces them to caustic-crossing and
 * distance-to-caustic maps, after Weisenbach (2025), "A GPU Code for Finding
 * Microlensing Critical Curves and Caustics" (arXiv 2506.02121).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers on the context's GPU (for example a
 *    torch tensor's data_ptr()), unless a comment says host.  The library
 *    checks each one with hipPointerGetAttributes and returns
 *    MLCC_ERR_INVALID for host or foreign memory.
 *  - Complex numbers are two float64 planes (structure of arrays): re[], im[].
 *  - Units: theta_star = theta_E = 1; masses in units of M (Sec. 2.1).
 *  - The caller owns every buffer it passes.  The library never frees or
 *    retains caller memory; mlcc_set_lenses copies its inputs.
 *  - Work is enqueued on the context's HIP stream.  Calls marked
 *    "synchronous" return after the stream has drained; the others only
 *    enqueue.  A context is not thread-safe: use one per host thread.
 *  - Errors are return codes; no exception crosses the ABI.  A readable
 *    message for the last failing call on this thread is given by
 *    mlcc_last_error().  On error the outputs are unspecified, except that
 *    MLCC_ERR_NOT_CONVERGED still writes every root it reached and reports
 *    the rest in stats.
 */
#ifndef MLCC_H
#define MLCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlcc_ctx mlcc_ctx;

typedef enum {
    MLCC_OK = 0,
    MLCC_ERR_INVALID = -1,       /* bad argument; nothing was enqueued */
    MLCC_ERR_HIP = -2,           /* a HIP runtime call failed */
    MLCC_ERR_NOMEM = -3,         /* device or pinned allocation failed */
    MLCC_ERR_NOT_CONVERGED = -4, /* an iteration cap was reached */
    MLCC_ERR_STATE = -5,         /* call order violated (e.g. no lenses set) */
    MLCC_ERR_MATCH = -7          /* two copies of one root set did not pair up */
} mlcc_status;

typedef enum {
    MLCC_FP64 = 0, /* the double-precision iteration of Sec. 3.2 and Sec. 4.4: every
                      star term, root-root term, sum, step and cutoff in IEEE double
                      precision.  Each reciprocal 1/|d|^2 is the hardware estimate
                      refined by one Newton step (relative error below 2^-47, against
                      2^-53 for a correctly rounded division); consecutive star terms,
                      and consecutive root-root terms, are taken in groups of eight that
                      share one refined reciprocal of the product of their eight |d|^2 */
    MLCC_MIXED = 1,/* Aberth sweeps in FP32 (FP64 star distances, FP32 sums per tile of
                      64 stars carried in FP64), every root finished by FP64 Newton
                      polish passes that accept a root on the same cutoffs as the
                      Aberth sweeps (on the Newton step), and the two row identities
                      (sum r, sum r^2) per row.  Cold starts:
                      FP32 sweeps until the roots settle, then the polish.  Warm rows:
                      the polish straight from the chain prediction (predictor > 0),
                      else after one FP32 sweep.  A row the polish does not settle
                      gets one FP32 sweep and the polish again, then restarts from
                      its start values with FP64 Aberth sweeps.  With the persistent
                      schedule and the chain predictor a polish pass whose roots are
                      all accepted goes on through up to 7 further rows of its front
                      (multipole star sums; direct sums for fields of at most 160
                      stars); the results are those of one row per pass.  Results
                      meet the same cutoffs as MLCC_FP64. */
    MLCC_FP64_R32 = 2 /* not the paper's precision: MLCC_FP64, except that in warm rows
                      the root-root sum R = sum_{r != k} 1/(z_k - z_r) of the Aberth
                      correction is formed in FP32 (each coordinate split into an FP32
                      pair hi + lo, the distance as (hi_k - hi_r) + (lo_k - lo_r), an
                      FP32 reciprocal, FP32 sums per tile of 64 roots carried in FP64):
                      relative error ~2^-24 per term.  R enters the step only through
                      F (2 S1 - R), which vanishes at a zero of F, so the roots it
                      accepts meet the same FP64 cutoffs; star sums, F, F', the step
                      and the lens map stay FP64, and cold starts are MLCC_FP64's */
} mlcc_precision;

typedef enum {
    MLCC_SCHEDULE_ROUNDS = 0,     /* global rounds: every front's pass, then a control kernel
                                     advancing all fronts; batches of rounds run as hipGraphs;
                                     per-kind kernel times in the stats */
    MLCC_SCHEDULE_PERSISTENT = 1  /* the default: one persistent launch (captured into a
                                     hipGraph and run from it), (front, block) passes
                                     from a device-side queue, each front advanced by the work
                                     group that finishes its pass, no global rounds.  Same
                                     results bit for bit; no front waits for the slowest pass
                                     of a round.  A launch in which no pass finishes for
                                     watchdog_ms (default 5 s) ends with MLCC_ERR_HIP. */
} mlcc_schedule;

typedef enum {
    MLCC_STARS_DIRECT = 0,        /* every star term summed directly (the default) */
    MLCC_STARS_FMM = 1            /* Sec. 4.1: stars binned on a grid; the 3 x 3 cells around a
                                     root summed directly, all others through the cell's local
                                     Taylor expansion (order fmm_order), which is built once per
                                     call from the far stars; in a batched call every field has
                                     its own grid.  The kernels then take each field's stars in
                                     cell order, so the seeds z_i +- 1 are numbered in that order */
} mlcc_star_sums;

/* Create a context on HIP device `device`, enqueuing on `hip_stream` (a
 * hipStream_t; NULL = the legacy default stream).  *out receives the context;
 * release it with mlcc_destroy. */
mlcc_status mlcc_create(mlcc_ctx **out, int device, void *hip_stream);
void mlcc_destroy(mlcc_ctx *ctx);
/* Replace the stream later calls enqueue on. */
mlcc_status mlcc_set_stream(mlcc_ctx *ctx, void *hip_stream);
/* Message for the last failing call on this thread (never NULL; valid until
 * the next call on this thread). */
const char *mlcc_last_error(void);

/*
 * set_lenses -- the lens model of Sec. 2.1 and Sec. 3.1 with the circular
 * field's compensating sheet extended to an infinite sheet (App. A):
 *   w(z)   = (1 - kappa_s) z + gamma conj(z) - sum_i m_i / conj(z - z_i)
 *   F(z,p) = gamma + sum_i m_i / (z - z_i)^2 - (1 - kappa_s) e^{-i p}
 * kappa_s = kappa - kappa_star is the smooth convergence; gamma the real
 * external shear along x1.
 *   n       number of point masses, >= 1
 *   x, y, m device float64[n]: positions and masses (m > 0), all finite,
 *           no two stars at the same position
 * Rejected (MLCC_ERR_INVALID): any of the above, non-finite kappa_s or gamma,
 * and |gamma| == |1 - kappa_s| (then gamma - (1-kappa_s) e^{-i p} vanishes on
 * the phase circle and a critical curve runs off to infinity, App. A
 * footnote).  Copies the inputs; synchronous.
 */
mlcc_status mlcc_set_lenses(mlcc_ctx *ctx, int64_t n, const double *x, const double *y,
                            const double *m, double kappa_s, double gamma);

/*
 * set_lenses_rect -- one rectangular microlens field (Sec. 4.2): stars in
 * [-c1, c1] x [-c2, c2] (not checked), corner c = c1 + i c2, and a smooth
 * sheet of convergence -kappa_star over the rectangle whose deflection has
 * its logarithms Taylor-expanded about the origin to odd degree t and is
 * extended to an infinite sheet for d alpha_s / dz (App. A, App. B).  Then
 *   d alpha_s / dz = -kappa_star,  conj(d alpha_s / d zbar) = d0 + sum_{j=2,4,..,t-1} d_j z^j,
 *   d0  = kappa_star (1 - 4 Arg(c) / pi),
 *   d_j = -(4 kappa_star / pi) sin(j Arg(c)) / (j |c|^j)   (App. B, last form),
 *   F(z,p) = gamma - d0 + sum_i m_i / (z - z_i)^2 - sum_j d_j z^j - (1 - kappa_s) e^{-i p},
 *   w(z)   = (1 - kappa_s) z + (gamma - d0) conj(z) - sum_j d_j conj(z)^(j+1) / (j+1)
 *            - sum_i m_i / conj(z - z_i),
 * and each phase has n_r = 2N + t - 1 roots (mlcc_num_roots): the t - 1
 * extra ones start evenly spread on the circle |z| = |c| (Sec. 3.2), at
 * angles 2 pi (k + 1/2) / (t - 1), k = 0 .. t - 2, after the 2N star seeds.
 * Outside the rectangle the expansion, and the curves found there, are not
 * the field's (App. A).
 *   n, x, y, m       as mlcc_set_lenses
 *   kappa_star       > 0, the sheet's convergence (the stars' mean
 *                    convergence pi sum m_i / (4 c1 c2) for a matched sheet)
 *   c1, c2           > 0
 *   t                odd, 1 .. 129 (mlcc_rect_taylor_degree picks one)
 * Rejected (MLCC_ERR_INVALID): the mlcc_set_lenses conditions (except the
 * |gamma| rule, which applies to gamma - d0 and only for t = 1), even or
 * out-of-range t, and (t - 1) Arg(c) within 10% of pi of a multiple of pi
 * (the leading coefficient nearly vanishes; App. B).  Only the two FP64
 * precisions (MLCC_FP64, MLCC_FP64_R32) solve it.  Copies the inputs;
 * synchronous.
 */
mlcc_status mlcc_set_lenses_rect(mlcc_ctx *ctx, int64_t n, const double *x, const double *y,
                                 const double *m, double kappa_s, double gamma, double kappa_star,
                                 double c1, double c2, int32_t t);

/*
 * rect_taylor_degree -- App. B's choice of t: the smallest t with
 *   (kappa_star / pi) (4 / (t + 1)) s^-(t+1) |c| (s + 1) / (s - 1) <= eps
 * (the bound on the truncation error of alpha_s where |z| s < |c|), made
 * odd, then raised by 2 until (t - 1) Arg(c) mod pi lies in [0.1 pi, 0.9 pi].
 *   s > 1, eps > 0; *t receives the degree.  MLCC_ERR_INVALID if no t up to
 *   129 qualifies.  Host only.
 */
mlcc_status mlcc_rect_taylor_degree(double kappa_star, double c1, double c2, double s,
                                    double eps, int32_t *t);

/* Roots per phase of the current lenses: sum over fields of 2N (+ t - 1 for
 * a rectangular field); the row length of mlcc_find_critical_curves. */
mlcc_status mlcc_num_roots(mlcc_ctx *ctx, int64_t *n_r);

/*
 * set_lenses_batched -- several independent star fields, each with its own
 * stars, kappa_s and gamma (the model of mlcc_set_lenses per field), solved
 * together by one mlcc_find_critical_curves call.  Field r holds stars
 * star_offsets[r] .. star_offsets[r+1]-1 of the concatenated arrays.
 *   n_fields          1 .. 65536
 *   star_offsets      host int64[n_fields + 1]: 0 = star_offsets[0] <
 *                     star_offsets[1] < ... ; total stars <= 2^28
 *   x, y, m           device float64[star_offsets[n_fields]]
 *   kappa_s, gamma    host float64[n_fields]
 * Rejected as for mlcc_set_lenses, field by field (duplicate positions are
 * checked within a field).  Copies the inputs; synchronous.  After it,
 * mlcc_map_caustics refuses (it maps through one field).
 */
mlcc_status mlcc_set_lenses_batched(mlcc_ctx *ctx, int32_t n_fields, const int64_t *star_offsets,
                                    const double *x, const double *y, const double *m,
                                    const double *kappa_s, const double *gamma);

typedef struct {
    int64_t m_steps;       /* phase steps m, even, >= 2: row j <-> phi_j = 2 pi j / m,
                              rows 0..m (Sec. 3.1, Sec. 4.3) */
    int32_t n_subchains;   /* S subchains (Sec. 4.3), each grown from its centre row;
                              must divide m/2.  0 = chosen by the library */
    int32_t max_iter_cold; /* sweep cap for a cold-started row (0 = 500) */
    int32_t max_iter_warm; /* sweep cap for a warm-started row (0 = 100) */
    int32_t precision;     /* mlcc_precision */
    double tol_step;       /* flag a root once |z^{a+1} - z^a| < tol_step; > 0 */
    double tol_inv_mu;     /* ... or once the App. C bound |F|(|F| + 2|1-kappa_s|) on
                              |1/mu| is below tol_inv_mu; 0 disables this test */
    int32_t timing;        /* nonzero: time the root-finder launches with HIP events (the
                              round schedule then launches eagerly, without graphs) */
    int32_t predictor;     /* start of a warm row's first pass, for each root:
                              0 = its value in the previous row (the warm start of
                              Sec. 3.2); 1 = linear, 2 = quadratic extrapolation
                              along its chain from the last 2 / 3 rows of the
                              same subchain (fewer rows are used where fewer
                              exist); the other roots enter that first pass at
                              their previous-row values */
    int32_t schedule;      /* mlcc_schedule */
    int32_t watchdog_ms;   /* MLCC_SCHEDULE_PERSISTENT: the launch gives up, and the call
                              returns MLCC_ERR_HIP, once no pass has finished anywhere for this
                              many milliseconds (0 = 5000; at most 600000) */
    int32_t star_sums;     /* mlcc_star_sums: how the sweeps and the polish sum over the stars
                              (the FP64 sweep's few-root cooperative passes always directly) */
    int32_t fmm_order;     /* MLCC_STARS_FMM: expansion order p, 8..63 (0 = 48); a far star's
                              terms are truncated after ~0.47^(p+1) of their size.  Below
                              p ~ 28 the jumps of F between neighbouring cells exceed what the
                              1e-9 cutoffs resolve, and roots near cell borders may not settle */
    int32_t cold_restart_sweeps; /* an FP64 cold start still unsettled after this many sweeps
                              begins again, once, from the second set of start values (z_i +- i;
                              a rectangular sheet's extra roots turned by half their spacing);
                              0 = 100.  Takes effect only below max_iter_cold */
} mlcc_cc_params;

/* The paper's cutoffs (Sec. 3.2 footnote: 1e-9 and |mu| > 1e9),
 * library-chosen subchains, FP64, quadratic chain predictor (predictor = 0
 * gives the paper's warm start from the previous row), persistent schedule. */
void mlcc_cc_params_default(mlcc_cc_params *p, int64_t m_steps);

typedef struct {
    int64_t sweeps;          /* MLCC_SCHEDULE_ROUNDS: rounds that did work (one round = every
                                pass kind once); MLCC_SCHEDULE_PERSISTENT: passes of the
                                front that made the most */
    int64_t root_updates;    /* FP64 Aberth root updates */
    int64_t root_updates_f32;/* FP32 Aberth root updates (MLCC_MIXED) */
    int64_t polish_updates;  /* FP64 Newton polish updates (MLCC_MIXED) */
    int64_t unconverged;     /* roots still unflagged in rows that hit a cap */
    int64_t rows_capped;     /* rows that hit an iteration cap */
    int64_t rows_fallback;   /* rows that fell back to FP64 Aberth sweeps (MLCC_MIXED) */
    int32_t n_subchains;     /* S actually used */
    int32_t max_row_sweeps;  /* most passes (of any kind) any warm row needed */
    int32_t cold_sweeps;     /* most passes any cold start needed */
    int32_t polls;           /* host polls of the device-side front table */
    double match_maxdist;    /* largest distance between paired duplicate roots */
    double sweep_ms;         /* GPU time of FP64 sweep launches that did work (timing != 0) */
    double sweep_f32_ms;     /* same, FP32 sweep launches */
    double polish_ms;        /* same, polish launches */
    int64_t sweep_launches, sweep_f32_launches, polish_launches;   /* launches that did work */
    double algorithmic_flop; /* FP64 sweeps, FP64 part: root_updates * 29 N (star terms) plus
                                10 (2N - 1) per update whose root-root terms run in FP64
                                (every update of MLCC_FP64; cold starts and the mixed form's
                                restarts otherwise); FMA = 2, add/mul/reciprocal = 1 */
    double algorithmic_flop_f32;    /* FP32 sweeps: root_updates_f32 * (29 N + 10 (2N - 1)) */
    double algorithmic_flop_polish; /* polish: polish_updates * 29 N (star terms only) */
    double persistent_ms;    /* MLCC_SCHEDULE_PERSISTENT: GPU time of the one launch that runs
                                every pass (timing != 0); the per-kind times above stay 0 */
    int64_t persistent_launches;    /* 1 with MLCC_SCHEDULE_PERSISTENT, else 0 */
    double algorithmic_flop_sweep_roots; /* FP64 sweeps, FP32 part: 10 (2N - 1) per update of
                                a warm MLCC_FP64_R32 row (its root-root terms run in FP32);
                                0 for MLCC_FP64 */
    int64_t fmm_near_terms;  /* MLCC_STARS_FMM: star terms summed directly in the updates that
                                took the multipole sums (the 3 x 3 near cells), all pass kinds;
                                0 otherwise */
    int64_t fmm_far_evals;   /* MLCC_STARS_FMM: those updates (one evaluation of a cell's series
                                each); the algorithmic FLOP fields above count such an update as
                                29 per near star term plus 26 p + 20 for the series of order p
                                (8 p more in sweeps of unequal masses).  FP32 sweeps take these
                                sums in FP64: their star part counts in algorithmic_flop, their
                                root terms stay in algorithmic_flop_f32 */
    int64_t cold_restarts;   /* FP64 cold starts still unsettled after cold_restart_sweeps
                                sweeps and begun again
                                from the second set of start values (z_i +- i; a rectangular
                                sheet's extra roots turned by half their spacing) */
} mlcc_cc_stats;

/*
 * find_critical_curves -- all n_r = 2N roots of F(., phi_j) for every row
 * j = 0..m of the phase grid (Sec. 3.1), by parallel Aberth-Ehrlich iteration
 * (Sec. 3.2): every unflagged root takes the step
 *   z <- z - 1 / (F'/F + 2 sum_i 1/(z - z_i) - sum_{r != k} 1/(z - z_r))
 * from the previous iterate of all roots at once, seeded with z_i +- 1 at the
 * centre row of each subchain and with the neighbouring row's roots elsewhere
 * (Sec. 3.2 warm start, Sec. 4.3 centre-out growth and subchains).
 *   roots_re, roots_im  device float64[(m+1) * 2N], row-major: row j holds the
 *                       roots at phi_j.  Column k is one continuous chain over
 *                       rows 0..m (subchain blocks are relabelled through the
 *                       nearest-neighbour pairing of their shared boundary row).
 *   caustics_re, caustics_im
 *                       device float64[(m+1) * 2N] or both NULL: the lens-equation
 *                       image w of every root (the caustics, Sec. 3.1), same
 *                       layout and chains.  Evaluated in the same pass from the
 *                       star sums at the last iterate z and the final step D:
 *                       sum m_i/(z - D - z_i) = sum m_i u_i + D sum m_i u_i^2
 *                       + D^2 sum m_i u_i^3 + O(D^3), with |D| below the cutoffs;
 *                       mlcc_map_caustics gives the same images directly.
 *   chain_next          device int32[2N] or NULL: chain_next[k] = the column
 *                       whose row 0 continues column k's row m (phi = 2 pi and
 *                       phi = 0 give the same roots; Sec. 4.3 footnote).
 *   stats               host, or NULL.
 * With several fields (mlcc_set_lenses_batched), field r with N_r stars and
 * star offset o_r owns the block of (m+1) * 2N_r elements starting at
 * (m+1) * 2 o_r of roots_* and caustics_* (row-major within the block, as
 * above) and the 2N_r entries starting at 2 o_r of chain_next (column
 * indices within the field); the arrays hold (m+1) * 2 * (total stars) and
 * 2 * (total stars) elements.  All fields share one phase grid and one set
 * of parameters; n_subchains = 0 picks one S for all of them.
 * Synchronous.  MLCC_ERR_NOT_CONVERGED if any row hit its cap;
 * MLCC_ERR_MATCH if duplicate rows did not pair one-to-one within 1e-6.
 */
mlcc_status mlcc_find_critical_curves(mlcc_ctx *ctx, const mlcc_cc_params *params,
                                      double *roots_re, double *roots_im, double *caustics_re,
                                      double *caustics_im, int32_t *chain_next,
                                      mlcc_cc_stats *stats);

/*
 * find_critical_curves_batched -- mlcc_find_critical_curves over the fields
 * of mlcc_set_lenses_batched (one field after mlcc_set_lenses), with the
 * layout made explicit: root_offsets (host int64[n_fields + 1], or NULL)
 * receives the first element of each field's (m+1) x 2N_r block in roots_*
 * and caustics_*, root_offsets[n_fields] the total; chain_next of field r
 * starts at 2 star_offsets[r].  Everything else as mlcc_find_critical_curves.
 */
mlcc_status mlcc_find_critical_curves_batched(mlcc_ctx *ctx, const mlcc_cc_params *params,
                                              int64_t *root_offsets, double *roots_re,
                                              double *roots_im, double *caustics_re,
                                              double *caustics_im, int32_t *chain_next,
                                              mlcc_cc_stats *stats);

/*
 * map_caustics -- the lens equation (Sec. 3.1, infinite sheet of App. A) at
 * `count` points: w = (1 - kappa_s) z + gamma conj(z) - sum_i m_i / conj(z - z_i).
 * Applied to the roots it gives the caustics.  z_re, z_im, w_re, w_im:
 * device float64[count]; w may not alias z.  Enqueues only.
 */
mlcc_status mlcc_map_caustics(mlcc_ctx *ctx, int64_t count, const double *z_re,
                              const double *z_im, double *w_re, double *w_im);

/* Pixel grid of the source plane: pixel (r, c) has its centre at
 * (center_re - half_width + (c + 0.5) hx, center_im - half_height + (r + 0.5) hy),
 * hx = 2 half_width / nx, hy = 2 half_height / ny; row 0 is the lowest y. */
typedef struct {
    double center_re, center_im, half_width, half_height;
    int32_t nx, ny;
} mlcc_grid;

/*
 * caustic_crossings -- the number of caustic crossings N_cc at every pixel
 * centre (Sec. 5.1): the winding number of the oriented caustic polygons
 * about the centre, by Sunday's crossing rule evaluated edge by edge (the
 * Sec. 5.1 footnote: loop over segments, not pixels).  Caustics run clockwise
 * (Sec. 5.1), and each edge crossing the ray from the centre toward -x
 * counts +1 when the edge runs upward and -1 when downward, so N_cc >= 0 for
 * closed caustics.  An edge covers heights lo <= y < hi; a crossing counts
 * when strictly left of the centre.  Vertices are put exactly on a lattice of
 * 2^24 points per pixel, X = rint((x - x0) / hx * 2^24), so the predicate is
 * exact integer arithmetic.
 *   w_re, w_im   device float64[rows * n_r], row-major caustic vertices
 *   edges        (row j, col k) -> (row j+1, col k) for j < rows-1, and the
 *                closing edges (rows-1, k) -> (0, chain_next[k])
 *   chain_next   device int32[n_r] or NULL (= identity)
 *   ncc          device int32[ny * nx], row-major
 * MLCC_ERR_INVALID if a vertex is not finite or lies more than 2^29 pixels
 * from the grid, or chain_next holds an index outside [0, n_r).
 * Synchronous.
 */
mlcc_status mlcc_caustic_crossings(mlcc_ctx *ctx, int64_t rows, int64_t n_r,
                                   const double *w_re, const double *w_im,
                                   const int32_t *chain_next, const mlcc_grid *grid,
                                   int32_t *ncc);

/*
 * caustic_crossings_noalloc -- mlcc_caustic_crossings for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result, bit
 * for bit, but the difference map and error word live in a fixed device
 * array of MLCC_NOALLOC_MAX_PIXELS + 64 int32 (16 MiB) that the library holds
 * on each GPU it runs on until the process ends, instead of context memory.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine); the caller passes inputs and outputs as for
 * mlcc_caustic_crossings.  Every call on one GPU shares that GPU's array and
 * clears it first: calls that overlap on one GPU (from several contexts,
 * streams or threads) race and must be serialised by the caller.
 *   arguments     as mlcc_caustic_crossings
 * MLCC_ERR_INVALID if nx * ny > MLCC_NOALLOC_MAX_PIXELS (use
 * mlcc_caustic_crossings), and for every case mlcc_caustic_crossings
 * rejects.  Synchronous.
 */
#define MLCC_NOALLOC_MAX_PIXELS (2048 * 2048)
mlcc_status mlcc_caustic_crossings_noalloc(mlcc_ctx *ctx, int64_t rows, int64_t n_r,
                                           const double *w_re, const double *w_im,
                                           const int32_t *chain_next, const mlcc_grid *grid,
                                           int32_t *ncc);

/*
 * caustic_distances -- distance from every pixel centre to the nearest
 * caustic pixel, for an expanding source (Sec. 5.2: Euclidean distance
 * transform of the N_cc map).  A caustic pixel is one with a 4-neighbour of
 * different N_cc; it gets 0.  The map border is not a caustic (Fig. 5
 * caption), so a pixel may be nearer to the border than to any caustic in
 * the map: border_limited marks those (distance > distance to the map edge).
 * With no caustic pixel at all every distance is +inf and every mark 1.
 * Pixels must be square: |hx - hy| <= 1e-9 hx; distances are in units of hx.
 * nx + ny <= 30000 (MLCC_ERR_INVALID otherwise).
 *   ncc             device int32[ny * nx]
 *   dist            device float64[ny * nx]: sqrt(d2) * hx, d2 the exact
 *                   integer squared pixel distance
 *   border_limited  device uint8[ny * nx] or NULL
 * Enqueues only.
 */
mlcc_status mlcc_caustic_distances(mlcc_ctx *ctx, const mlcc_grid *grid, const int32_t *ncc,
                                   double *dist, uint8_t *border_limited);

/*
 * caustic_distances_directional -- distance to the caustics for a moving source
 * (Sec. 5.2, Fig. 5 bottom): from every pixel centre, the distance travelled
 * along the direction (cos angle, sin angle) (angle from the +y1 axis, in
 * radians) before the source centre enters a caustic pixel (a pixel with a
 * 4-neighbour of different N_cc, as for mlcc_caustic_distances).  A square
 * the path only touches at a corner is not entered; a caustic pixel gets 0.
 * If the path leaves the map first (the border is not a caustic, Fig. 5
 * caption), the distance is the exit distance and border_limited is 1.
 * Square pixels as for mlcc_caustic_distances; nx + ny <= 10^6.
 *   ncc             device int32[ny * nx]
 *   dist            device float64[ny * nx], in units of hx
 *   border_limited  device uint8[ny * nx] or NULL
 * Enqueues only.
 */
mlcc_status mlcc_caustic_distances_directional(mlcc_ctx *ctx, const mlcc_grid *grid,
                                               const int32_t *ncc, double angle, double *dist,
                                               uint8_t *border_limited);

/*
 * distance_histogram -- the distributions of Figs. 6 and 7: counts of pixels
 * by distance (bin k holds k w <= d < (k+1) w, w = d_max / n_bins, computed as
 * floor(d * (n_bins / d_max)); column n_bins counts d >= d_max), skipping
 * border-limited pixels, and with ncc given, by N_cc class (row k holds
 * N_cc = ncc_lo + k; other values are skipped).  P(d | angle) is one call per
 * angle of mlcc_caustic_distances_directional; P(d | N_cc) one call with ncc.
 *   count           pixels
 *   dist, border_limited  device float64[count], uint8[count]
 *   ncc             device int32[count] or NULL (then n_classes = 1)
 *   counts          device int64[n_classes * (n_bins + 1)], overwritten;
 *                   n_classes * (n_bins + 1) <= 8192
 * Enqueues only.
 */
mlcc_status mlcc_distance_histogram(mlcc_ctx *ctx, int64_t count, const double *dist,
                                    const uint8_t *border_limited, const int32_t *ncc,
                                    int32_t ncc_lo, int32_t n_classes, int32_t n_bins,
                                    double d_max, int64_t *counts);

#ifdef __cplusplus
}
#endif

#endif /* MLCC_H */
