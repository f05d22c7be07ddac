// Caustic-crossing map (Sec. 5.1): N_cc at each pixel centre is the winding
// number of the clockwise caustic polygons about it (Sunday's rule, signed so
// that a clockwise loop counts +1).  Following the Sec. 5.1 footnote the work
// is done per edge, not per pixel: for every pixel row whose centre height an
// edge spans (half-open, lo <= y < hi), the first column whose centre lies
// strictly right of the crossing receives the edge's sign (+1 upward,
// -1 downward) in a per-row difference map; a prefix sum along each row then
// yields N_cc.
//
// Exactness: vertices go on a lattice of 2^24 points per pixel; pixel centres
// are lattice points; the crossing test is a 128-bit integer comparison, and
// the first column is a floating-point estimate corrected by that exact test.
#include <algorithm>
#include <mutex>

#include "mlcc_internal.h"

namespace mlcc {

constexpr int QBITS = 24;
constexpr int64_t HALF = (int64_t)1 << (QBITS - 1); // half a pixel on the lattice
constexpr double QSCALE = 16777216.0;               // 2^QBITS
constexpr double QLIMIT = 9007199254740992.0;       // 2^53

__device__ __forceinline__ bool to_lattice(double v, double v0, double h, int64_t *q)
{
    const double s = (v - v0) / h * QSCALE;
    if (!(fabs(s) < QLIMIT)) return false; // also rejects NaN
    *q = (int64_t)rint(s);
    return true;
}

// floor(a / b) for b > 0
__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && (a < 0)) --q;
    return q;
}

// Edges of one chain (column k) over CROSS_ROWS consecutive rows per lane:
// each vertex is loaded and put on the lattice once and serves as the end of
// one edge and the start of the next; lanes of a work group take adjacent
// columns, so every row's loads are coalesced.
constexpr int CROSS_ROWS = 16;

// Adds the edge (a -> b)'s crossings to the difference map.
__device__ __forceinline__ void edge_crossings(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                                               int32_t nx, int32_t ny,
                                               int32_t *__restrict__ diff)
{
    if (ay == by) return;
    int s = 1;
    if (ay > by) {   // order the ends by height; a downward edge counts -1
        int64_t t = ax; ax = bx; bx = t;
        t = ay; ay = by; by = t;
        s = -1;
    }
    // rows r with (2r+1) HALF in [ay, by)
    int64_t r0 = floor_div64(ay + HALF - 1, 2 * HALF);
    int64_t r1 = floor_div64(by + HALF - 1, 2 * HALF);
    if (r0 < 0) r0 = 0;
    if (r1 > ny) r1 = ny;
    const int64_t dy = by - ay, dx = bx - ax;
    const double slope = (double)dx / (double)dy;
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t yr = (2 * r + 1) * HALF;
        // crossing x = ax + (yr - ay) dx / dy = num / dy
        const __int128 num = (__int128)ax * dy + (__int128)(yr - ay) * dx;
        // column c's centre (2c+1) HALF is strictly right of the crossing
        // iff (2c+1) HALF dy > num
        auto right = [&](int64_t c) {
            return (__int128)(2 * c + 1) * HALF * dy > num;
        };
        const double xc = (double)ax + (double)(yr - ay) * slope;
        double cest = floor((xc / (double)HALF - 1.0) * 0.5) + 1.0;
        cest = fmin(fmax(cest, 0.0), (double)nx);
        int64_t c = (int64_t)cest;
        while (c > 0 && right(c - 1)) --c;
        while (c < nx && !right(c)) ++c;
        if (c < nx) atomicAdd(&diff[r * nx + c], s);
    }
}

// One lane per (column, chunk of CROSS_ROWS rows); work group b covers
// columns 256 (b mod cb) .. + 255 of chunk b / cb (cb = column blocks).
__global__ void __launch_bounds__(256)
crossing_edges(int64_t rows, int64_t n_r, int64_t cb, const double *__restrict__ wr,
               const double *__restrict__ wi, const int32_t *__restrict__ chain_next,
               double x0, double y0, double hx, double hy, int32_t nx, int32_t ny,
               int32_t *__restrict__ diff, int32_t *__restrict__ err)
{
    const int64_t k = (blockIdx.x % cb) * 256 + threadIdx.x;
    if (k >= n_r) return;
    const int64_t j0 = (blockIdx.x / cb) * CROSS_ROWS;
    const int64_t j1 = min(j0 + CROSS_ROWS, rows);
    int64_t ax, ay;
    if (!to_lattice(wr[j0 * n_r + k], x0, hx, &ax) || !to_lattice(wi[j0 * n_r + k], y0, hy, &ay)) {
        atomicOr(err, 1);
        return;
    }
    for (int64_t j = j0; j < j1; ++j) {
        int64_t j2 = j + 1, k2 = k;
        if (j2 == rows) {   // the closing edge: row 0 of the chain that continues this one
            j2 = 0;
            k2 = chain_next ? chain_next[k] : k;
            if (k2 < 0 || k2 >= n_r) {
                atomicOr(err, 2);
                return;
            }
        }
        int64_t bx, by;
        if (!to_lattice(wr[j2 * n_r + k2], x0, hx, &bx) ||
            !to_lattice(wi[j2 * n_r + k2], y0, hy, &by)) {
            atomicOr(err, 1);
            return;
        }
        edge_crossings(ax, ay, bx, by, nx, ny, diff);
        ax = bx;
        ay = by;
    }
}

// Clears n int32 (the difference map and the error word before a call).
__global__ void __launch_bounds__(256) zero_i32(int32_t *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

// Inclusive prefix sum along each row: one 256-lane work-group per row,
// 64-lane wave scans joined through LDS, chunk by chunk.
__global__ void __launch_bounds__(256)
row_prefix(const int32_t *__restrict__ diff, int32_t *__restrict__ ncc, int32_t nx)
{
    __shared__ int32_t wave_tot[4];
    __shared__ int32_t carry;
    const int r = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nx; base += 256) {
        const int c = base + tid;
        int v = c < nx ? diff[(int64_t)r * nx + c] : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(v, off, 64);
            if (lane >= off) v += t;
        }
        if (lane == 63) wave_tot[w] = v;
        __syncthreads();
        int add = carry;
        for (int q = 0; q < w; ++q) add += wave_tot[q];
        v += add;
        if (c < nx) ncc[(int64_t)r * nx + c] = v;
        __syncthreads();
        if (tid == 255) carry = v;
        __syncthreads();
    }
}

// The three launches and the error readback of one crossing map, with the
// difference map (npix int32) and the error word after it in `diff`.
static mlcc_status crossings_into(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                  const double *wi, const int32_t *chain_next,
                                  const mlcc_grid *g, int32_t *ncc, int32_t *diff)
{
    const int64_t nx = g->nx, ny = g->ny;
    const double x0 = g->center_re - g->half_width, y0 = g->center_im - g->half_height;
    const double hx = (2.0 * g->half_width) / (double)nx, hy = (2.0 * g->half_height) / (double)ny;
    const int64_t npix = nx * ny;
    int32_t *err = diff + npix;
    const int64_t cb = ceil_div(n_r, 256);
    const int64_t blocks = cb * ceil_div(rows, CROSS_ROWS);
    if (blocks > 0x7fffffff) return fail(MLCC_ERR_INVALID, "too many edges");
    // one clear of the difference map and the error word (a kernel, not a
    // memset node, so that a captured graph replays it correctly)
    hipLaunchKernelGGL(zero_i32, dim3((unsigned)std::min<int64_t>(ceil_div(npix + 1, 256), 8192)),
                       dim3(256), 0, c->stream, diff, npix + 1);
    hipLaunchKernelGGL(crossing_edges, dim3((unsigned)blocks), dim3(256), 0, c->stream, rows, n_r,
                       cb, wr, wi, chain_next, x0, y0, hx, hy, (int32_t)nx, (int32_t)ny, diff, err);
    hipLaunchKernelGGL(row_prefix, dim3((unsigned)ny), dim3(256), 0, c->stream, diff, ncc,
                       (int32_t)nx);
    MLCC_HIP(hipGetLastError());
    int32_t herr = 0;
    MLCC_HIP(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, c->stream));
    MLCC_HIP(hipStreamSynchronize(c->stream));
    if (herr & 1)
        return fail(MLCC_ERR_INVALID,
                    "a caustic vertex is not finite or lies more than 2^29 pixels from the grid");
    if (herr & 2) return fail(MLCC_ERR_INVALID, "chain_next holds an index outside [0, n_r)");
    return MLCC_OK;
}

mlcc_status run_caustic_crossings(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                  const double *wi, const int32_t *chain_next,
                                  const mlcc_grid *g, int32_t *ncc)
{
    const int64_t npix = (int64_t)g->nx * g->ny;
    MLCC_TRY(c->diff.reserve((size_t)(npix + 64) * sizeof(int32_t)));
    return crossings_into(c, rows, n_r, wr, wi, chain_next, g, ncc, c->diff.as<int32_t>());
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the difference map and the error word live in a
// fixed device array instead of context memory.  In host code `scratch` only
// names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress at context creation and is the one passed to kernels.
// ---------------------------------------------------------------------------

static __device__ __align__(256) int32_t scratch[MLCC_NOALLOC_MAX_PIXELS + 64];

constexpr int MAX_DEVICES = 64;
static std::mutex scratch_mu;
static int32_t *scratch_dev[MAX_DEVICES];   // device address of `scratch`, per device

mlcc_status noalloc_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES)
        return fail(MLCC_ERR_INVALID, "device %d beyond the %d the library supports", device,
                    MAX_DEVICES);
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return MLCC_OK;
    void *p = nullptr;
    MLCC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MLCC_ERR_HIP, "hipGetSymbolAddress gave no address for the scratch array");
    scratch_dev[device] = static_cast<int32_t *>(p);
    return MLCC_OK;
}

mlcc_status run_caustic_crossings_noalloc(Ctx *c, int64_t rows, int64_t n_r, const double *wr,
                                          const double *wi, const int32_t *chain_next,
                                          const mlcc_grid *g, int32_t *ncc)
{
    const int64_t npix = (int64_t)g->nx * g->ny;
    if (npix > MLCC_NOALLOC_MAX_PIXELS)
        return fail(MLCC_ERR_INVALID,
                    "caustic_crossings_noalloc: %lld pixels exceed the fixed scratch of %lld "
                    "(use mlcc_caustic_crossings)",
                    (long long)npix, (long long)MLCC_NOALLOC_MAX_PIXELS);
    int32_t *diff = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mu);
        diff = (c->device >= 0 && c->device < MAX_DEVICES) ? scratch_dev[c->device] : nullptr;
    }
    if (!diff) return fail(MLCC_ERR_STATE, "the scratch array of device %d is not set up", c->device);
    return crossings_into(c, rows, n_r, wr, wi, chain_next, g, ncc, diff);
}

} // namespace mlcc
