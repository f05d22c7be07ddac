// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

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
    int32_t sweeps;   // sweeps spent on the current row
    int32_t src;      // front whose iterate this front reads on its next sweep
    int32_t partner;  // cold start: front that takes over the other direction
    int32_t bnd_slot; // >= 0: its end row is a duplicate boundary row, kept here
    int32_t lo, hi;   // rows of the subchain
    int32_t max_warm; // most sweeps a warm row of this front needed
    int32_t cold;     // sweeps its cold start needed
};
enum { FRONT_IDLE = 0, FRONT_ACTIVE = 1, FRONT_DONE = 2, FRONT_FAILED = 3 };

// Device-side totals of the root finder.
struct Control {
    int32_t active_fronts;      // fronts still IDLE or ACTIVE
    int32_t failed_rows;
    int64_t unconverged;
    unsigned long long updates; // root updates
    int64_t live_sweeps;        // sweep launches that found an active front
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;

    // lenses
    int64_t n = 0;
    double kappa_s = 0.0, gamma = 0.0;
    bool equal_mass = false;
    double mass0 = 1.0; // the common mass when equal_mass
    DevBuf stars;  // double2[n]: (x, y)
    DevBuf mass;   // double[n]
    DevBuf stars4; // double4[n]: (x, y, m, 0)

    // root-finder workspace
    DevBuf iter[2];   // double2[F * n_r]: Jacobi iterates, ping-pong
    DevBuf flagrow;   // int32[F * n_r]: row at which the root was flagged
    DevBuf fronts;    // Front[F]
    DevBuf counts;    // int32[F]: unflagged roots after the last sweep
    DevBuf control;   // Control
    DevBuf etab;      // double2[m + 1]: (1 - kappa_s) e^{-i phi_j}
    DevBuf bnd;       // double2[(S - 1) * n_r]: duplicate boundary rows
    DevBuf perm;      // int32[(S + 1) * n_r]: pairings and global labels
    DevBuf match_aux; // matching workspace
    DevBuf relabel;   // scratch rows for the in-place relabel
    DevBuf workflags; // int32[poll batch]: did launch i do work

    // crossing / distance workspace
    DevBuf diff;      // int32 per-row difference map
    DevBuf err;       // int32 error flag
    DevBuf edt_col;   // int32 column distances

    void *pinned = nullptr; // host-pinned readback area
    size_t pinned_bytes = 0;
};

mlcc_status check_device_ptr(const Ctx *c, const void *p, const char *what);
mlcc_status ensure_pinned(Ctx *c, size_t bytes);

// Entry points implemented per translation unit (argument checks done by the
// caller in api.hip).
mlcc_status find_critical_curves_fp64(Ctx *c, const mlcc_cc_params *p, double *roots_re,
                                      double *roots_im, double *caus_re, double *caus_im,
                                      int32_t *chain_next, mlcc_cc_stats *stats);
mlcc_status launch_map_caustics(Ctx *c, int64_t count, const double *zr, const double *zi,
                                double *wr, double *wi);
mlcc_status run_caustic_crossings(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                  const double *wi, const int32_t *chain_next,
                                  const mlcc_grid *g, int32_t *ncc);
mlcc_status launch_caustic_distances(Ctx *c, const mlcc_grid *g, const int32_t *ncc,
                                     double *dist, uint8_t *border_limited);

// Nearest-neighbour pairing of two copies of one root set (chains.hip).
//   a, b: n points each (double2 interleaved for a, SoA planes for b)
//   perm[k] = index in b nearest a[k]; returns MLCC_ERR_MATCH when not 1-1 or
//   when a pair is further apart than tol; *maxdist = largest paired distance.
mlcc_status pair_rows(Ctx *c, int64_t n, const double2 *a, const double *b_re,
                      const double *b_im, int32_t *perm, double tol, double *maxdist);
mlcc_status pair_rows_soa(Ctx *c, int64_t n, const double *a_re, const double *a_im,
                          const double *b_re, const double *b_im, int32_t *perm, double tol,
                          double *maxdist);
// Relabel rows [row0, row1) in place: new[j][label[k]] = old[j][k].
mlcc_status relabel_rows(Ctx *c, double *re, double *im, int64_t n_r, int64_t row0,
                         int64_t row1, const int32_t *label);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

} // namespace mlcc

struct mlcc_ctx {
    mlcc::Ctx impl;
};
