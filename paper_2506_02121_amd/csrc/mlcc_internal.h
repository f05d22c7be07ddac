// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mlcc.h"

namespace mlcc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
mlcc_status fail(mlcc_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define MLCC_HIP(expr)                                                                    \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::mlcc::fail(e_ == hipErrorOutOfMemory ? MLCC_ERR_NOMEM : MLCC_ERR_HIP, \
                                "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                                __LINE__);                                                \
    } while (0)

#define MLCC_TRY(expr)                          \
    do {                                        \
        mlcc_status s_ = (expr);                \
        if (s_ != MLCC_OK) return s_;           \
    } while (0)

// ---------------------------------------------------------------------------
// device memory owned by a context
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    // Grow to at least n bytes (contents are not kept).
    mlcc_status reserve(size_t n);
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Per-front control record of the root finder (one per growing end of a
// subchain, see aberth.hip).
struct Front {
    int32_t row;      // row being solved
    int32_t dir;      // -1 toward row 0, +1 toward row m, 0 = cold start at the centre
    int32_t end_row;  // last row this front solves (inclusive)
    int32_t state;    // FRONT_IDLE / FRONT_ACTIVE / FRONT_DONE / FRONT_FAILED
    int32_t sweeps;   // FP64 sweeps spent on the current row
    int32_t src;      // front whose iterate this front reads on its next pass
    int32_t partner;  // cold start: front that takes over the other direction
    int32_t bnd_slot; // >= 0: its end row is a duplicate boundary row, kept here
    int32_t lo, hi;   // rows of the subchain
    int32_t max_warm; // most FP64 sweeps a warm row of this front needed
    int32_t cold;     // sweeps its cold start needed
    int32_t phase;    // PH_F64 / PH_F32 / PH_POLISH: what the next pass does
    int32_t mode;     // phase a new warm row starts in
    int32_t stamp;    // flag value meaning "converged on this row": 4 row + generation
    int32_t passes;   // polish passes spent on the current row
    int32_t real;     // realisation (star field) this front belongs to
    int32_t blk0;     // first block of this front in the launch grid
    int32_t hist;     // finished rows of this subchain behind the current row (<= 3)
    int32_t fresh;    // 1 until the first pass over the current row has run
    int32_t tried;    // mixed mode: TRIED_F32 | TRIED_POLISH done on the current row
    int32_t f32;      // FP32 sweeps on the current row
    int32_t best;     // fewest roots still moving after an FP32 sweep (cold start)
    int32_t stall;    // FP32 sweeps since that count last fell
    int32_t passes_row; // passes of any kind on the current row
    int32_t reseed;   // 1: the next FP64 pass restarts the row from its start values
    int32_t par;      // persistent scheduler: which iterate buffer holds the current values
    int32_t npass;    // passes run by this front (all rows)
    int32_t seedvar;  // cold start: 0 = the seeds z_i +- 1; 1 = the second set (after a stall)
    int64_t it_off;   // first element of its roots in the iterate and flag arrays
};

// Rectangular field: the sheet polynomial (see sheet_poly in api.hip) has at
// most this many terms, so the Taylor degree is at most 2 MAX_SHEET_TERMS + 1.
constexpr int MAX_SHEET_TERMS = 64;

// One star field of a (possibly batched) root-finder call, as the kernels
// see it.
struct Real {
    int64_t star_off;   // first star in the concatenated star arrays
    int64_t out_off;    // first element of its (m+1) x n_r output block
    int64_t bnd_off;    // first element of its duplicate boundary rows
    int32_t n_stars, n_r;
    double m0;          // the common mass (equal-mass kernels)
    double gamma, a, a1;   // shear, 1 - kappa_s, |1 - kappa_s|
    double sz_r, sz_i, sz2_r, sz2_i, M;   // sum z_i, sum z_i^2, sum m_i (row identities)
    double tol1, tol2;  // rounding of the reference values of the two row identities
    int32_t n_poly;     // rectangular field: sheet terms (gamma holds gamma - d0); else 0
    int32_t n_extra;    // roots beyond 2 N: t - 1 for a rectangular field
    int32_t root32;     // MLCC_FP64_R32: warm FP64 rows take the root-root sum in FP32
    int32_t restart;    // FP64 sweeps after which an unsettled cold start begins again
    int32_t xrows;      // persistent mixed form: further rows a polish pass may finish (0: none)
    int32_t pad_;
    int64_t sheet_off;  // its record in the sheet array: d_2..d_{t-1} (n_poly), the lens-map
                        // terms d_2k / (2k + 1) (n_poly), start values of the extra roots
                        // (2 n_extra: re, im)
};

// Host-side description of one star field.
struct RealHost {
    int64_t star_off = 0, n = 0;
    double kappa_s = 0, gamma = 0, m0 = 1;
    bool equal = false;
    double2 sum_z{0, 0}, sum_z2{0, 0};
    double sum_abs_z = 0, sum_abs_z2 = 0, max_abs_z = 0, mass_total = 0;
    // rectangular field (t > 0): sheet of convergence -kappa_star, corner
    // c1 + i c2, Taylor degree t
    int32_t t = 0;
    double kappa_star = 0, c1 = 0, c2 = 0;
};

// The sheet polynomial of a rectangular field, as the kernels use it:
//   conj(d alpha_s / d zbar) = d0 + sum_{k=1..n} d[k-1] z^(2k), d real,
// and in the lens map alpha_s(z) = -kappa_star z + d0 conj(z)
//   + sum_k d[k-1] conj(z)^(2k+1) / (2k+1).
struct SheetPoly {
    int32_t n = 0;          // terms (t - 1) / 2; 0 for a circular field
    int32_t n_extra = 0;    // roots the sheet adds: t - 1
    double d0 = 0;          // constant term (folded into gamma by the caller)
    double seed_r = 0;      // radius of the extra roots' start values, |c|
    double d[MAX_SHEET_TERMS] = {};
    double dmap[MAX_SHEET_TERMS] = {};   // d[k-1] / (2k + 1)
};
SheetPoly sheet_poly(const RealHost &h);
enum { FRONT_IDLE = 0, FRONT_ACTIVE = 1, FRONT_DONE = 2, FRONT_FAILED = 3 };
enum { PH_F64 = 0, PH_F32 = 1, PH_POLISH = 2 };
enum { TRIED_F32 = 1, TRIED_POLISH = 2 };

// Device-side totals of the root finder.
struct Control {
    int32_t active_fronts;            // fronts still IDLE or ACTIVE
    int32_t failed_rows;
    int64_t unconverged;
    unsigned long long updates;       // FP64 Aberth root updates
    unsigned long long updates_f32;   // FP32 Aberth root updates
    unsigned long long polish_updates;
    int64_t rows_fallback;            // rows that fell back to FP64 sweeps
    int64_t live_sweeps;              // rounds that found an active front
    int64_t cold_restarts;            // FP64 cold starts begun again from the second seeds
    unsigned long long star_updates;  // sum over FP64 updates of the field's star count
    unsigned long long star_updates_f32;
    unsigned long long star_updates_polish;
    unsigned long long updates_fast;      // FP64 Aberth updates of warm FP64-mode rows, whose
    unsigned long long star_updates_fast; // root-root terms run in FP32 (and their star counts)
};

// Tallies of the fast-multipole star sums behind the algorithmic FLOP count,
// per pass kind (FMM_T_F64, FMM_T_POLISH, FMM_T_F32): near-field star terms
// (+0), far-field series evaluations (+1) and those evaluations times their
// field's star count (+2).  Work groups add to one of FMM_STRIPES copies, each
// on a cache line of its own, so that the adds of thousands of work groups
// do not queue on one address; the host sums the copies.
constexpr int FMM_STRIPES = 16;
constexpr int FMM_STRIPE_U64 = 16;   // 128 bytes per copy
enum { FMM_T_F64 = 0, FMM_T_POLISH = 3, FMM_T_F32 = 6 };

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;   // rounds of the root finder when `stream` is null

    // lenses: one field (set_lenses) or a batch (set_lenses_batched), stars
    // concatenated
    bool batched = false;
    bool rect = false;  // set_lenses_rect: one rectangular field
    std::vector<RealHost> reals;
    int64_t n = 0;      // total stars
    double kappa_s = 0.0, gamma = 0.0;  // the single field's macro-model
    bool equal_mass = false;
    double mass0 = 1.0; // the common mass when equal_mass
    DevBuf stars;  // double2[n]: (x, y)
    DevBuf mass;   // double[n]
    DevBuf stars4; // double4[n]: (x, y, m, 0)
    DevBuf sheet_d; // double[MAX_SHEET_TERMS]: lens-map terms of a rectangular field's sheet
    DevBuf sheet;   // double[]: the root finder's sheet records (Real::sheet_off)

    // root-finder workspace
    DevBuf iter[2];   // double2[F * n_r]: Jacobi iterates, ping-pong
    DevBuf flagrow;   // int32[F * n_r]: row at which the root was flagged
    DevBuf fronts;    // Front[F]
    DevBuf counts;    // int32[F]: unflagged roots after the last sweep
    DevBuf passupd;   // int32[F]: roots updated by the last round's pass
    DevBuf control;   // Control
    DevBuf fmm_tally; // uint64[FMM_STRIPES * FMM_STRIPE_U64]: multipole tallies
    DevBuf etab;      // double2[m + 1]: (1 - kappa_s) e^{-i phi_j}
    DevBuf bnd;       // double2[(S - 1) * n_r]: duplicate boundary rows
    DevBuf perm;      // int32[(S + 1) * n_r]: pairings and global labels
    DevBuf match_aux; // matching workspace
    DevBuf relabel;   // scratch rows for the in-place relabel
    DevBuf workflags; // int32[poll batch]: phases active in round i
    DevBuf vieta;     // double4[2 * blocks]: per-block row sums and error terms (mixed mode)
    DevBuf errbuf;    // double[F * n_r]: estimated error of each polished root
    DevBuf vsum;      // double4[2 * F]: each front's row sums (mixed mode)
    DevBuf pq;        // persistent scheduler: queue header, task ring, slot sequence, pass counts
    DevBuf reals_d;   // Real[n_real]
    DevBuf bmap;      // int2[blocks]: (front, block within front)

    // crossing / distance workspace
    DevBuf diff;      // int32 per-row difference map, then the crossing kernel's error word
    DevBuf edt_col;   // distance map: caustic-mask words (uint64 per column and band of 64
                      // rows), and the lower-envelope work rows of maps too wide for LDS
    DevBuf dmask;     // uint8 caustic-pixel mask (moving-source distances)
    // fast multipole star sums: the stars sorted by grid cell and each cell's
    // expansions (built by the root finder when asked for)
    std::vector<double4> hstars;   // host copy of the stars (x, y, m, 0)
    DevBuf fmm_cs, fmm_st, fmm_st2, fmm_cf, fmm_cg, fmm_q, fmm_m, fmm_args;

    void *pinned = nullptr; // host-pinned readback area
    size_t pinned_bytes = 0;
};

mlcc_status check_device_ptr(const Ctx *c, const void *p, const char *what);
mlcc_status ensure_pinned(Ctx *c, size_t bytes);

// Entry points implemented per translation unit (argument checks done by the
// caller in api.hip).
mlcc_status find_critical_curves_impl(Ctx *c, const mlcc_cc_params *p, double *roots_re,
                                      double *roots_im, double *caus_re, double *caus_im,
                                      int32_t *chain_next, mlcc_cc_stats *stats);
mlcc_status launch_directional_distances(Ctx *c, const mlcc_grid *grid, const int32_t *ncc,
                                         double angle, double *dist, uint8_t *border_limited);
mlcc_status launch_distance_histogram(Ctx *c, int64_t count, const double *dist,
                                      const uint8_t *border_limited, const int32_t *ncc,
                                      int32_t ncc_lo, int32_t n_classes, int32_t n_bins,
                                      double d_max, int64_t *counts);
mlcc_status launch_map_caustics(Ctx *c, int64_t count, const double *zr, const double *zi,
                                double *wr, double *wi);
mlcc_status run_caustic_crossings(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                  const double *wi, const int32_t *chain_next,
                                  const mlcc_grid *g, int32_t *ncc);
mlcc_status run_caustic_crossings_noalloc(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                          const double *wi, const int32_t *chain_next,
                                          const mlcc_grid *g, int32_t *ncc);
// Looks up, once per device (the device current), the device address of the
// allocation-free crossing map's fixed scratch array (crossings.hip).
mlcc_status noalloc_scratch_init(int device);
mlcc_status launch_caustic_distances(Ctx *c, const mlcc_grid *g, const int32_t *ncc,
                                     double *dist, uint8_t *border_limited);

// Nearest-neighbour pairing of two copies of one root set (chains.hip).
// A job pairs n points a (double2 interleaved, or SoA planes) with n points b
// (SoA planes): perm[k] = index in b nearest a[k].  All jobs run in one
// launch and are checked at once; the call fails with
// MLCC_ERR_MATCH when a pairing is not one-to-one or a pair is further apart
// than tol.  *maxdist receives the largest paired distance.
struct PairJob {
    const double2 *a2;
    const double *a_re, *a_im, *b_re, *b_im;
    int32_t *perm;
    int64_t n;
};
mlcc_status pair_all(Ctx *c, const std::vector<PairJob> &jobs, double tol, double *maxdist);
// Relabel rows [row0, row1) of (re, im) in place: new[j][label[k]] =
// old[j][k]; all jobs in a few chunked launches through context scratch.
struct RelabelJob {
    double *re, *im;
    int64_t n_r, row0, row1;
    const int32_t *label;
};
mlcc_status relabel_all(Ctx *c, const std::vector<RelabelJob> &jobs);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

} // namespace mlcc

struct mlcc_ctx {
    mlcc::Ctx impl;
};
