// Moving source (Sec. 5.2, Fig. 5 bottom, Figs. 6 and 7): the distance a
// source travels from each pixel centre along a fixed direction before its
// centre enters a caustic pixel (a pixel with a 4-neighbour of different
// N_cc, as for the expanding source), and histograms of such distances.
//
// A ray from a pixel centre crosses the pixel boundaries x = +-1/2, +-3/2, ...
// (relative to its own centre) at t = (a - 1/2)/|cos|, a = 1, 2, ..., and the
// y boundaries likewise; each crossing moves it one pixel in x or in y, and
// both at once where an x and a y crossing coincide (it passes through a
// corner, so squares touched only at the corner are not entered).  The
// sequence of pixel offsets it visits, and the parameter of each step, is
// therefore the same for every start pixel: walk_events builds it once per
// direction, as the merge of the two sorted crossing sequences (each crossing
// one correctly rounded division of an exact half-integer by the direction's
// component, so the distances are reproducible to the bit), together with the
// step at which a ray leaves the map through each column or row boundary.
// directional_walk then checks, for every pixel, the mask at its own start
// plus each offset in turn, sixteen steps per round of independent loads,
// until the first caustic pixel, or until the step that leaves the map (the
// border is not a caustic, Fig. 5 caption): then the distance is the exit
// distance and the pixel is marked border-limited.  Lanes of a wave take
// neighbouring pixels of a row, so every step of the wave reads 64
// consecutive mask bytes.
#include <climits>
#include <cmath>

#include "mlcc_internal.h"

namespace mlcc {

__global__ void __launch_bounds__(256)
caustic_mask_u8(const int32_t *__restrict__ ncc, int32_t nx, int32_t ny, uint8_t *__restrict__ mask)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)nx * ny) return;
    const int r = (int)(p / nx), c = (int)(p - (int64_t)r * nx);
    const int32_t v = ncc[p];
    mask[p] = (uint8_t)((c > 0 && ncc[p - 1] != v) || (c + 1 < nx && ncc[p + 1] != v) ||
                        (r > 0 && ncc[p - nx] != v) || (r + 1 < ny && ncc[p + nx] != v));
}

// The step table of one direction.  Steps are numbered 0, 1, ... in order of
// the ray parameter; step k moves the ray to offset delta[k] (pixels, row-major,
// from the start pixel) at parameter t[k].  exit_x[a] is the step that makes
// the a-th x crossing (a = 1 .. nx), exit_y[b] the step of the b-th y crossing
// (b = 1 .. ny; a y crossing that coincides with an x crossing shares its
// step).  xcnt and xtie are work arrays over the x crossings.
struct WalkTable {
    int64_t *delta;   // [nx + ny + WALK_UNROLL]
    double *t;        // [nx + ny + WALK_UNROLL]
    int32_t *exit_x;  // [nx + 1]
    int32_t *exit_y;  // [ny + 1]
    int32_t *xcnt;    // [nx + 1]: y crossings strictly before x crossing a
    int32_t *xtie;    // [nx + 1]: 1 if a y crossing coincides with x crossing a,
                      //           then the inclusive prefix count of those
};

constexpr int WALK_UNROLL = 16;   // steps per round of loads
constexpr int WALK_TABLE_THREADS = 1024;

// Parameter of the n-th crossing (n >= 1) along one axis, with s the step
// sign, hs = s/2 and comp the direction's component along the axis.
__device__ __forceinline__ double crossing_t(int64_t n, int s, double hs, double comp)
{
    return ((double)((n - 1) * s) + hs) / comp;
}

// Number of crossings n in 1 .. count (along the axis given by s, hs, comp)
// with parameter strictly below v: a first guess from (n - 1/2)/|comp| < v,
// then exact comparisons with the crossing parameters themselves, which
// increase strictly with n.
__device__ __forceinline__ int64_t crossings_below(double v, int64_t count, int s, double hs,
                                                   double comp)
{
    if (count == 0) return 0;
    double g = ceil(fma(v, fabs(comp), 0.5)) - 1.0;
    g = fmin(fmax(g, 0.0), (double)count);
    int64_t c = (int64_t)g;
    while (c < count && crossing_t(c + 1, s, hs, comp) < v) ++c;
    while (c > 0 && !(crossing_t(c, s, hs, comp) < v)) --c;
    return c;
}

__global__ void __launch_bounds__(WALK_TABLE_THREADS)
walk_events(int32_t nx, int32_t ny, double ca, double sa, WalkTable w)
{
    __shared__ int32_t part[WALK_TABLE_THREADS];
    const int tid = threadIdx.x;
    const int sx = ca > 0.0 ? 1 : -1, sy = sa > 0.0 ? 1 : -1;
    const double hx = 0.5 * sx, hy = 0.5 * sy;
    const int64_t ax = ca != 0.0 ? nx : 0, ay = sa != 0.0 ? ny : 0;

    // 1. for every x crossing: the y crossings before it, and a coincident one
    for (int64_t a = 1 + tid; a <= ax; a += WALK_TABLE_THREADS) {
        const double tx = crossing_t(a, sx, hx, ca);
        const int64_t cy = crossings_below(tx, ay, sy, hy, sa);
        w.xcnt[a] = (int32_t)cy;
        w.xtie[a] = (cy < ay && crossing_t(cy + 1, sy, hy, sa) == tx) ? 1 : 0;
    }
    __syncthreads();

    // 2. inclusive prefix count of the coincidences, in place (xtie[0] = 0)
    const int64_t chunk = (ax + WALK_TABLE_THREADS - 1) / WALK_TABLE_THREADS;
    const int64_t lo = 1 + tid * chunk, hi = min(ax, lo + chunk - 1);
    int32_t own = 0;
    for (int64_t a = lo; a <= hi; ++a) own += w.xtie[a];
    part[tid] = own;
    __syncthreads();
    for (int off = 1; off < WALK_TABLE_THREADS; off <<= 1) {
        const int32_t add = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += add;
        __syncthreads();
    }
    int32_t run = part[tid] - own;
    for (int64_t a = lo; a <= hi; ++a) {
        run += w.xtie[a];
        w.xtie[a] = run;
    }
    if (tid == 0) w.xtie[0] = 0;
    __syncthreads();

    // 3. the steps: an x crossing a is preceded by a - 1 x crossings and
    // xcnt[a] y crossings, less the xtie[a - 1] pairs among them that share a
    // step; a y crossing b by b - 1 y and cx x crossings, less xtie[cx]
    for (int64_t a = 1 + tid; a <= ax; a += WALK_TABLE_THREADS) {
        const int32_t before = w.xtie[a - 1];
        const int32_t tie = w.xtie[a] - before;
        const int32_t k = (int32_t)(a - 1) + w.xcnt[a] - before;
        w.exit_x[a] = k;
        w.delta[k] = (int64_t)sy * (w.xcnt[a] + tie) * nx + sx * a;
        w.t[k] = crossing_t(a, sx, hx, ca);
    }
    for (int64_t b = 1 + tid; b <= ay; b += WALK_TABLE_THREADS) {
        const double ty = crossing_t(b, sy, hy, sa);
        const int64_t cx = crossings_below(ty, ax, sx, hx, ca);
        const bool tie = cx < ax && crossing_t(cx + 1, sx, hx, ca) == ty;
        const int32_t k = (int32_t)(b - 1 + cx) - w.xtie[cx];
        w.exit_y[b] = k;
        if (!tie) {
            w.delta[k] = (int64_t)sy * b * nx + sx * cx;
            w.t[k] = ty;
        }
    }
    // padding read by the last round of a walk (never taken as a step)
    const int64_t steps = ax + ay - w.xtie[ax];
    if (tid < WALK_UNROLL) {
        w.delta[steps + tid] = 0;
        w.t[steps + tid] = 0.0;
    }
}

__global__ void __launch_bounds__(256)
directional_walk(const uint8_t *__restrict__ mask, int32_t nx, int32_t ny, int32_t sx, int32_t sy,
                 int32_t has_x, int32_t has_y, const int64_t *__restrict__ delta,
                 const double *__restrict__ tt, const int32_t *__restrict__ exit_x,
                 const int32_t *__restrict__ exit_y, double h, double *__restrict__ dist,
                 uint8_t *__restrict__ border_limited)
{
    const int64_t npix = (int64_t)nx * ny;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t pc = p < npix ? p : npix - 1;   // lanes past the end: the last pixel's bounds
    const int r0 = (int)(pc / nx), c0 = (int)(pc - (int64_t)r0 * nx);
    // the step that leaves the map: through the last column or row boundary
    int32_t ke = INT_MAX;
    if (has_x) ke = exit_x[sx > 0 ? nx - c0 : c0 + 1];
    if (has_y) ke = min(ke, exit_y[sy > 0 ? ny - r0 : r0 + 1]);
    // the wave's earliest exit: rounds that end before it need no per-lane bound
    int32_t kmin = ke;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) kmin = min(kmin, __shfl_xor(kmin, off, 64));
    kmin = __builtin_amdgcn_readfirstlane(kmin);
    if (p >= npix) return;
    if (mask[p]) {
        dist[p] = 0.0;
        if (border_limited) border_limited[p] = 0;
        return;
    }
    // Every load of a round is issued before any is tested.  The lanes still
    // walking are at the same step, so the offsets are read once per wave.
    // In a round that reaches past some lane's exit, a step past it reads
    // the start pixel instead (offset masked to zero; not a caustic pixel).
    int32_t hit = -1;
    for (int32_t k = 0; k < ke; k += WALK_UNROLL) {
        const int32_t ku = __builtin_amdgcn_readfirstlane(k);
        int64_t d[WALK_UNROLL];
        uint8_t m[WALK_UNROLL];
#pragma unroll
        for (int u = 0; u < WALK_UNROLL; ++u) d[u] = delta[ku + u];
        if (ku + WALK_UNROLL <= kmin) {
#pragma unroll
            for (int u = 0; u < WALK_UNROLL; ++u) m[u] = mask[p + d[u]];
        } else {
#pragma unroll
            for (int u = 0; u < WALK_UNROLL; ++u)
                m[u] = mask[p + (d[u] & -(int64_t)(ku + u < ke))];
        }
        int first = WALK_UNROLL;
#pragma unroll
        for (int u = WALK_UNROLL - 1; u >= 0; --u)
            if (m[u]) first = u;
        if (first < WALK_UNROLL) {
            hit = ku + first;
            break;
        }
    }
    const int32_t kk = hit >= 0 ? hit : ke;
    dist[p] = tt[kk] * h;
    if (border_limited) border_limited[p] = hit >= 0 ? 0 : 1;
}

// Counts per (class, bin): bin k = floor(d * inv_w) for d * inv_w < n_bins,
// else the overflow bin n_bins; pixels marked border-limited are skipped;
// with ncc, class = ncc - ncc_lo and pixels outside 0 .. n_classes-1 are
// skipped.  Each work group counts in LDS, then adds its counts to the
// global ones.
constexpr int HIST_PX = 4;          // runs of 64 pixels per wave and round
constexpr int HIST_GROUPS = 1024;   // work groups of the histogram (at most)
__global__ void __launch_bounds__(256)
distance_histogram(int64_t count, const double *__restrict__ dist,
                   const uint8_t *__restrict__ border_limited, const int32_t *__restrict__ ncc,
                   int32_t ncc_lo, int32_t n_classes, int32_t n_bins, double inv_w,
                   unsigned long long *__restrict__ counts)
{
    extern __shared__ uint32_t local[];
    const int nb = n_classes * (n_bins + 1);
    for (int q = threadIdx.x; q < nb; q += 256) local[q] = 0u;
    __syncthreads();
    // Each wave takes HIST_PX runs of 64 consecutive pixels per round and
    // issues all their loads before it counts the first.  Neighbouring
    // pixels mostly fall in few bins: the lanes of a wave that share a bin
    // add their count once, through the lowest of them.
    const int lane = threadIdx.x & 63;
    constexpr int PX = HIST_PX;
    const int wave = threadIdx.x >> 6;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64 * PX; base < count;
         base += (int64_t)gridDim.x * 4 * 64 * PX) {
        double dv[PX];
        uint8_t bv[PX];
        int cv[PX];
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            const int64_t p = min(base + u * 64 + lane, count - 1);
            dv[u] = dist[p];
            bv[u] = border_limited[p];
            cv[u] = ncc ? ncc[p] - ncc_lo : 0;
        }
#pragma unroll
        for (int u = 0; u < PX; ++u) {
            const double x = dv[u] * inv_w;
            const int bin = (base + u * 64 + lane < count && !bv[u] && cv[u] >= 0 &&
                             cv[u] < n_classes)
                                ? cv[u] * (n_bins + 1) + (x < (double)n_bins ? (int)floor(x) : n_bins)
                                : -1;
            unsigned long long left = __ballot(bin >= 0);
            while (left) {
                const int leader = __builtin_ctzll(left);
                const int b = __builtin_amdgcn_readlane(bin, leader);
                const unsigned long long same = __ballot(bin == b) & left;
                if (lane == leader) atomicAdd(&local[b], (uint32_t)__popcll(same));
                left &= ~same;
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += 256)
        if (local[q]) atomicAdd(&counts[q], (unsigned long long)local[q]);
}

__global__ void __launch_bounds__(256) zero_u64(unsigned long long *__restrict__ a, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) a[p] = 0ull;
}

mlcc_status launch_directional_distances(Ctx *c, const mlcc_grid *grid, const int32_t *ncc,
                                         double angle, double *dist, uint8_t *border_limited)
{
    const int32_t nx = grid->nx, ny = grid->ny;
    const int64_t npix = (int64_t)nx * ny;
    const double h = (2.0 * grid->half_width) / (double)nx;
    const double ca = std::cos(angle), sa = std::sin(angle);
    // mask bytes, then the step table (nx + ny <= 10^6 steps at most)
    const size_t steps = (size_t)nx + (size_t)ny + WALK_UNROLL;
    const size_t mask_bytes = ((size_t)npix + 255) & ~(size_t)255;
    const size_t bytes = mask_bytes + steps * (sizeof(int64_t) + sizeof(double)) +
                         4 * ((size_t)std::max(nx, ny) + 1) * sizeof(int32_t);
    MLCC_TRY(c->dmask.reserve(bytes));
    char *base = static_cast<char *>(c->dmask.p);
    uint8_t *mask = reinterpret_cast<uint8_t *>(base);
    WalkTable w;
    w.delta = reinterpret_cast<int64_t *>(base + mask_bytes);
    w.t = reinterpret_cast<double *>(w.delta + steps);
    w.exit_x = reinterpret_cast<int32_t *>(w.t + steps);
    w.exit_y = w.exit_x + ((size_t)nx + 1);
    w.xcnt = w.exit_y + ((size_t)ny + 1);
    w.xtie = w.xcnt + ((size_t)nx + 1);
    const unsigned blocks = (unsigned)ceil_div(npix, 256);
    hipLaunchKernelGGL(caustic_mask_u8, dim3(blocks), dim3(256), 0, c->stream, ncc, nx, ny, mask);
    hipLaunchKernelGGL(walk_events, dim3(1), dim3(WALK_TABLE_THREADS), 0, c->stream, nx, ny, ca,
                       sa, w);
    hipLaunchKernelGGL(directional_walk, dim3(blocks), dim3(256), 0, c->stream, mask, nx, ny,
                       ca > 0.0 ? 1 : -1, sa > 0.0 ? 1 : -1, ca != 0.0 ? 1 : 0, sa != 0.0 ? 1 : 0,
                       w.delta, w.t, w.exit_x, w.exit_y, h, dist, border_limited);
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

mlcc_status launch_distance_histogram(Ctx *c, int64_t count, const double *dist,
                                      const uint8_t *border_limited, const int32_t *ncc,
                                      int32_t ncc_lo, int32_t n_classes, int32_t n_bins,
                                      double d_max, int64_t *counts)
{
    const int64_t nb = (int64_t)n_classes * (n_bins + 1);
    unsigned long long *cu = reinterpret_cast<unsigned long long *>(counts);
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, c->stream, cu,
                       nb);
    if (count > 0) {
        const int64_t groups = std::min<int64_t>(ceil_div(count, 256 * HIST_PX), HIST_GROUPS);
        hipLaunchKernelGGL(distance_histogram, dim3((unsigned)groups), dim3(256),
                           (size_t)nb * sizeof(uint32_t), c->stream, count, dist, border_limited,
                           ncc, ncc_lo, n_classes, n_bins, (double)n_bins / d_max, cu);
    }
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

} // namespace mlcc
