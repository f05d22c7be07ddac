// Moving source (Sec. 5.2, Fig. 5 bottom, Figs. 6 and 7): the distance a
// source travels from each pixel centre along a fixed direction before its
// centre enters a caustic pixel (a pixel with a 4-neighbour of different
// N_cc, as for the expanding source), and histograms of such distances.
//
// One lane per pixel walks the pixels its ray passes through, in order of the
// ray parameter (a grid traversal: the next x or y pixel boundary, whichever
// the ray reaches first; both at once when it meets a pixel corner exactly,
// so squares touched only at a corner are not entered).  Every crossing
// parameter is one division of an exact half-integer offset by the
// direction's component, so the distances are reproducible to the bit.  The
// walk stops at the first caustic pixel, or where the ray leaves the map,
// which is not a caustic (Fig. 5 caption): then the distance is the exit
// distance and the pixel is marked border-limited.  Lanes of a wave take
// neighbouring pixels of a row, whose rays run side by side.
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

__global__ void __launch_bounds__(256)
directional_walk(const uint8_t *__restrict__ mask, int32_t nx, int32_t ny, double h, double ca,
                 double sa, double *__restrict__ dist, uint8_t *__restrict__ border_limited)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)nx * ny) return;
    const int r0 = (int)(p / nx), c0 = (int)(p - (int64_t)r0 * nx);
    if (mask[p]) {
        dist[p] = 0.0;
        if (border_limited) border_limited[p] = 0;
        return;
    }
    const int sx = ca > 0.0 ? 1 : -1, sy = sa > 0.0 ? 1 : -1;
    const double hx = 0.5 * sx, hy = 0.5 * sy;
    int i = c0, j = r0;
    double tx = ca != 0.0 ? hx / ca : INFINITY;
    double ty = sa != 0.0 ? hy / sa : INFINITY;
    double t = 0.0;
    bool hit = false;
    // at most nx + ny steps leave the map
    for (int step = 0; step < nx + ny + 2; ++step) {
        if (tx < ty) {
            i += sx;
            t = tx;
            tx = ((double)(i - c0) + hx) / ca;
        } else if (ty < tx) {
            j += sy;
            t = ty;
            ty = ((double)(j - r0) + hy) / sa;
        } else {   // a pixel corner: step diagonally
            i += sx;
            j += sy;
            t = tx;
            tx = ((double)(i - c0) + hx) / ca;
            ty = ((double)(j - r0) + hy) / sa;
        }
        if (i < 0 || i >= nx || j < 0 || j >= ny) break;
        if (mask[(int64_t)j * nx + i]) {
            hit = true;
            break;
        }
    }
    dist[p] = t * h;
    if (border_limited) border_limited[p] = hit ? 0 : 1;
}

// Counts per (class, bin): bin k = floor(d * inv_w) for d * inv_w < n_bins,
// else the overflow bin n_bins; pixels marked border-limited are skipped;
// with ncc, class = ncc - ncc_lo and pixels outside 0 .. n_classes-1 are
// skipped.  Each work group counts in LDS, then adds its counts to the
// global ones.
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
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < count;
         p += (int64_t)gridDim.x * 256) {
        if (border_limited[p]) continue;
        int cls = 0;
        if (ncc) {
            cls = ncc[p] - ncc_lo;
            if (cls < 0 || cls >= n_classes) continue;
        }
        const double x = dist[p] * inv_w;
        const int k = x < (double)n_bins ? (int)floor(x) : n_bins;
        atomicAdd(&local[cls * (n_bins + 1) + k], 1u);
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
    MLCC_TRY(c->dmask.reserve((size_t)npix));
    const unsigned blocks = (unsigned)ceil_div(npix, 256);
    hipLaunchKernelGGL(caustic_mask_u8, dim3(blocks), dim3(256), 0, c->stream, ncc, nx, ny,
                       c->dmask.as<uint8_t>());
    hipLaunchKernelGGL(directional_walk, dim3(blocks), dim3(256), 0, c->stream,
                       c->dmask.as<uint8_t>(), nx, ny, h, ca, sa, dist, border_limited);
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
        const int64_t groups = std::min<int64_t>(ceil_div(count, 256), 4096);
        hipLaunchKernelGGL(distance_histogram, dim3((unsigned)groups), dim3(256),
                           (size_t)nb * sizeof(uint32_t), c->stream, count, dist, border_limited,
                           ncc, ncc_lo, n_classes, n_bins, (double)n_bins / d_max, cu);
    }
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

} // namespace mlcc
