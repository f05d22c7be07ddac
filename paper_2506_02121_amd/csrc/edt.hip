// Distance to the nearest caustic for an expanding source (Sec. 5.2): an
// exact Euclidean distance transform of the caustic pixels of the N_cc map.
// A caustic pixel has a 4-neighbour of different N_cc; the map border is not
// a caustic (Fig. 5 caption).
//
// Two kernels in integer arithmetic:
//  1. edt_mask_words: the caustic-pixel mask as one 64-bit word per column
//     and band of 64 rows (bit i = row 64 t + i); one lane per column, one
//     work group per (64 columns, band), so a 2048^2 map runs as 1024 work
//     groups.  Each lane walks its band keeping the rows above and below in
//     registers; left and right neighbours come from the adjacent lanes.
//  2. edt_rows: one work group per row.  The column distance
//     g(r, c) = |r - nearest caustic row of column c| is read off the mask
//     words (the set bit nearest to row r in the band's word, else in the
//     nearest band with one), then
//       d2(r, c) = min_q [(c - q)^2 + g(r, q)^2]
//     is searched outward from q = c: terms with |c - q| >= k are at least
//     k^2, so the search stops once k^2 reaches the best value found; no
//     term is skipped, so the minimum is exact.  A pixel still open after
//     WINDOW steps (a map with few caustics) sends its row to the lower
//     envelope of parabolas (Meijster, Roerdink & Hesselink 2000), which
//     costs O(nx) per row whatever the distances.
// A map with a caustic pixel has one in some column, whose g is finite on
// every row, so a row whose g are all infinite belongs to a map with no
// caustic pixel at all.
// Output: sqrt(d2) * h, and the border-limited mark 4 d2 > b^2 where b is
// twice the distance (in pixels) from the centre to the nearest map edge.
#include "mlcc_internal.h"

namespace mlcc {

// Outward search steps per pixel before a row takes the lower envelope.
constexpr int EDT_WINDOW = 512;
constexpr int EDT_ROW_THREADS = 256;

__global__ void __launch_bounds__(64)
edt_mask_words(const int32_t *__restrict__ ncc, int32_t nx, int32_t ny,
               uint64_t *__restrict__ bits)
{
    const int lane = threadIdx.x;
    const int c = blockIdx.x * 64 + lane;
    const int r0 = blockIdx.y * 64, r1 = min(r0 + 64, ny);
    const bool in = c < nx;
    const int cc = in ? c : nx - 1;   // loads of lanes past the last column stay in bounds
    int32_t cur = ncc[(int64_t)r0 * nx + cc];
    int32_t prev = r0 > 0 ? ncc[(int64_t)(r0 - 1) * nx + cc] : cur;
    uint64_t w = 0;
    for (int r = r0; r < r1; ++r) {
        const int64_t p = (int64_t)r * nx + cc;
        const int32_t next = r + 1 < ny ? ncc[p + nx] : cur;
        int32_t left = __shfl_up(cur, 1, 64);
        int32_t right = __shfl_down(cur, 1, 64);
        if (lane == 0 && cc > 0) left = ncc[p - 1];
        if (lane == 63 && cc + 1 < nx) right = ncc[p + 1];
        const bool edge = (cc > 0 && left != cur) || (cc + 1 < nx && right != cur) ||
                          (r > 0 && prev != cur) || (r + 1 < ny && next != cur);
        if (edge) w |= 1ull << (r - r0);
        prev = cur;
        cur = next;
    }
    if (in) bits[(int64_t)blockIdx.y * nx + c] = w;
}

template <bool IN_LDS>
__global__ void __launch_bounds__(EDT_ROW_THREADS)
edt_rows(const uint64_t *__restrict__ bits, int32_t nx, int32_t ny, double h,
         int32_t *__restrict__ work, double *__restrict__ dist,
         uint8_t *__restrict__ border_limited)
{
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_any, s_open;
    const int r = blockIdx.x;
    const int tid = threadIdx.x;
    int32_t *g = IN_LDS ? lds : work + (int64_t)r * 4 * nx;
    int32_t *s = g + nx, *t = s + nx, *d2 = t + nx;
    const int32_t ginf = nx + ny;   // exceeds every real column distance
    const int band = r >> 6, o = r & 63, nb = (ny + 63) >> 6;
    if (tid == 0) {
        s_any = 0;
        s_open = 0;
    }
    __syncthreads();
    bool any = false;
    for (int c = tid; c < nx; c += EDT_ROW_THREADS) {
        const uint64_t w = bits[(int64_t)band * nx + c];
        int32_t dn = ginf, up = ginf;
        const uint64_t lo = o == 63 ? w : w & ((2ull << o) - 1);   // rows <= r of the band
        if (lo) {
            dn = o - (63 - __clzll(lo));
        } else {
            for (int q = band - 1; q >= 0; --q) {
                const uint64_t v = bits[(int64_t)q * nx + c];
                if (v) {
                    dn = r - (q * 64 + 63 - __clzll(v));
                    break;
                }
            }
        }
        const uint64_t hi = w >> o;   // rows >= r of the band
        if (hi) {
            up = __ffsll((long long)hi) - 1;
        } else {
            for (int q = band + 1; q < nb; ++q) {
                const uint64_t v = bits[(int64_t)q * nx + c];
                if (v) {
                    up = q * 64 + (__ffsll((long long)v) - 1) - r;
                    break;
                }
            }
        }
        const int32_t gc = min(dn, up);
        g[c] = gc;
        any |= gc < ginf;
    }
    if (any) s_any = 1;
    __syncthreads();
    const bool none = s_any == 0;
    if (!none) {
        bool open = false;
        for (int c = tid; c < nx; c += EDT_ROW_THREADS) {
            int32_t best = g[c] * g[c];
            int k = 1;
            for (; k <= EDT_WINDOW; ++k) {
                const int32_t kk = k * k;
                if (kk >= best || (c - k < 0 && c + k >= nx)) break;
                const int32_t a = c - k >= 0 ? g[c - k] : ginf;
                const int32_t b = c + k < nx ? g[c + k] : ginf;
                const int32_t m = min(a, b);
                best = min(best, kk + m * m);
            }
            d2[c] = best;
            open |= k > EDT_WINDOW;
        }
        if (open) s_open = 1;
        __syncthreads();
        if (s_open) {
            if (tid == 0) {
                // f(x, i) = (x - i)^2 + g(i)^2; sep(i, u) = first x at which
                // parabola u is no higher than parabola i (u > i), floor division.
                auto f = [&](int64_t x, int64_t i) {
                    return (x - i) * (x - i) + (int64_t)g[i] * g[i];
                };
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
        }
    }
    for (int c = tid; c < nx; c += EDT_ROW_THREADS) {
        const int64_t p = (int64_t)r * nx + c;
        const int64_t v = none ? 0 : d2[c];
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
    const int32_t bands = (int32_t)ceil_div(ny, 64);
    const size_t lds_bytes = (size_t)16 * nx;
    const bool in_lds = lds_bytes <= 64 * 1024;
    const size_t bits_bytes = (size_t)bands * nx * sizeof(uint64_t);
    const size_t work_bytes = in_lds ? 0 : (size_t)16 * nx * ny;
    MLCC_TRY(c->edt_col.reserve(bits_bytes + work_bytes + 256));
    uint64_t *bits = c->edt_col.as<uint64_t>();
    int32_t *work = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(c->edt_col.p) + bits_bytes);
    hipLaunchKernelGGL(edt_mask_words, dim3((unsigned)ceil_div(nx, 64), (unsigned)bands), dim3(64),
                       0, c->stream, ncc, nx, ny, bits);
    if (in_lds)
        hipLaunchKernelGGL(edt_rows<true>, dim3((unsigned)ny), dim3(EDT_ROW_THREADS), lds_bytes,
                           c->stream, bits, nx, ny, h, work, dist, border_limited);
    else
        hipLaunchKernelGGL(edt_rows<false>, dim3((unsigned)ny), dim3(EDT_ROW_THREADS), 0,
                           c->stream, bits, nx, ny, h, work, dist, border_limited);
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

} // namespace mlcc
