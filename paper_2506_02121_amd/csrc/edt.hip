// Distance to the nearest caustic for an expanding source (Sec. 5.2): an
// exact Euclidean distance transform of the caustic pixels of the N_cc map.
// A caustic pixel has a 4-neighbour of different N_cc; the map border is not
// a caustic (Fig. 5 caption).
//
// Two separable passes in integer arithmetic:
//  1. columns: g(r, c) = distance in rows to the nearest caustic pixel of
//     column c (one lane per column, a down and an up sweep; coalesced across
//     lanes);
//  2. rows: d2(r, c) = min_q [(c - q)^2 + g(r, q)^2] by the lower envelope of
//     parabolas (Meijster, Roerdink & Hesselink 2000), one work-group per row
//     with the row staged in LDS.
// Output: sqrt(d2) * h, and the border-limited mark 4 d2 > b^2 where b is
// twice the distance (in pixels) from the centre to the nearest map edge.
#include "mlcc_internal.h"

namespace mlcc {

__device__ __forceinline__ bool caustic_pixel(const int32_t *__restrict__ ncc, int r, int c,
                                              int nx, int ny)
{
    const int64_t p = (int64_t)r * nx + c;
    const int32_t v = ncc[p];
    return (c > 0 && ncc[p - 1] != v) || (c + 1 < nx && ncc[p + 1] != v) ||
           (r > 0 && ncc[p - nx] != v) || (r + 1 < ny && ncc[p + nx] != v);
}

__global__ void __launch_bounds__(256)
edt_columns(const int32_t *__restrict__ ncc, int32_t nx, int32_t ny, int32_t ginf,
            int32_t *__restrict__ col, int32_t *__restrict__ any)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nx) return;
    int32_t g = ginf;
    bool seen = false;
    for (int r = 0; r < ny; ++r) {
        if (caustic_pixel(ncc, r, c, nx, ny)) {
            g = 0;
            seen = true;
        } else if (g < ginf) {
            ++g;
        }
        col[(int64_t)r * nx + c] = g;
    }
    if (seen) atomicOr(any, 1);
    g = ginf;
    for (int r = ny - 1; r >= 0; --r) {
        const int64_t p = (int64_t)r * nx + c;
        const int32_t down = col[p];
        if (down == 0) g = 0;
        else if (g < ginf) ++g;
        if (g < down) col[p] = g;
    }
}

template <bool IN_LDS>
__global__ void __launch_bounds__(64)
edt_rows(const int32_t *__restrict__ col, int32_t nx, int32_t ny, double h,
         const int32_t *__restrict__ any, int32_t *__restrict__ work, double *__restrict__ dist,
         uint8_t *__restrict__ border_limited)
{
    extern __shared__ int32_t lds[];
    const int r = blockIdx.x;
    int32_t *g, *s, *t, *d2;
    if (IN_LDS) {
        g = lds;
    } else {
        g = work + (int64_t)r * 4 * nx;
    }
    s = g + nx;
    t = s + nx;
    d2 = t + nx;
    for (int c = threadIdx.x; c < nx; c += 64) g[c] = col[(int64_t)r * nx + c];
    __syncthreads();
    if (threadIdx.x == 0) {
        // f(x, i) = (x - i)^2 + g(i)^2; sep(i, u) = first x at which parabola u
        // is no higher than parabola i (u > i), floor division.
        auto f = [&](int64_t x, int64_t i) { return (x - i) * (x - i) + (int64_t)g[i] * g[i]; };
        auto sep = [&](int64_t i, int64_t u) {
            const int64_t num = u * u - i * i + (int64_t)g[u] * g[u] - (int64_t)g[i] * g[i];
            const int64_t den = 2 * (u - i);
            int64_t q = num / den;
            if ((num % den != 0) && (num < 0)) --q;
            return q;
        };
        int q = 0;
        s[0] = 0;
        t[0] = 0;
        for (int u = 1; u < nx; ++u) {
            while (q >= 0 && f(t[q], s[q]) > f(t[q], u)) --q;
            if (q < 0) {
                q = 0;
                s[0] = u;
            } else {
                const int64_t w = 1 + sep(s[q], u);
                if (w < nx) {
                    ++q;
                    s[q] = u;
                    t[q] = (int32_t)w;
                }
            }
        }
        for (int u = nx - 1; u >= 0; --u) {
            d2[u] = (int32_t)f(u, s[q]);
            if (u == t[q]) --q;
        }
    }
    __syncthreads();
    const bool none = *any == 0;
    for (int c = threadIdx.x; c < nx; c += 64) {
        const int64_t p = (int64_t)r * nx + c;
        const int64_t v = d2[c];
        dist[p] = none ? INFINITY : sqrt((double)v) * h;
        if (border_limited) {
            int64_t b = 2 * c + 1;
            b = min(b, (int64_t)(2 * (nx - c) - 1));
            b = min(b, (int64_t)(2 * r + 1));
            b = min(b, (int64_t)(2 * (ny - r) - 1));
            border_limited[p] = (uint8_t)(none || 4 * v > b * b);
        }
    }
}

mlcc_status launch_caustic_distances(Ctx *c, const mlcc_grid *grid, const int32_t *ncc,
                                     double *dist, uint8_t *border_limited)
{
    const int32_t nx = grid->nx, ny = grid->ny;
    if ((int64_t)nx + ny > 30000)
        return fail(MLCC_ERR_INVALID, "distance maps are limited to nx + ny <= 30000");
    const double h = (2.0 * grid->half_width) / (double)nx;
    const int32_t ginf = nx + ny; // exceeds every real column distance
    const size_t lds_bytes = (size_t)16 * nx;
    const bool in_lds = lds_bytes <= 64 * 1024;
    const size_t col_bytes = (size_t)nx * ny * sizeof(int32_t);
    const size_t work_bytes = in_lds ? 0 : (size_t)16 * nx * ny;
    MLCC_TRY(c->edt_col.reserve(col_bytes + work_bytes + 256));
    MLCC_TRY(c->err.reserve(sizeof(int32_t)));
    int32_t *col = c->edt_col.as<int32_t>();
    int32_t *work = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(c->edt_col.p) + col_bytes);
    int32_t *any = c->err.as<int32_t>();
    MLCC_HIP(hipMemsetAsync(any, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(edt_columns, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, c->stream,
                       ncc, nx, ny, ginf, col, any);
    if (in_lds)
        hipLaunchKernelGGL(edt_rows<true>, dim3((unsigned)ny), dim3(64), lds_bytes, c->stream, col,
                           nx, ny, h, any, work, dist, border_limited);
    else
        hipLaunchKernelGGL(edt_rows<false>, dim3((unsigned)ny), dim3(64), 0, c->stream, col, nx,
                           ny, h, any, work, dist, border_limited);
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

} // namespace mlcc
