// Distance to the nearest caustic for an expanding source (Sec. 5.2): an
// exact Euclidean distance transform of the caustic pixels of the N_cc map.
// A caustic pixel has a 4-neighbour of different N_cc; the map border is not
// a caustic (Fig. 5 caption).
//
// Two kernels in integer arithmetic:
//  1. edt_mask_words: the caustic-pixel mask as one 64-bit word per column
//     and band of 64 rows (bit i = row 64 t + i); one lane per column and
//     16 rows, one four-wave work group per (64 columns, band), so a 2048^2
//     map runs as 1024 work groups.  Each lane walks its 16 rows keeping the
//     rows above and below in registers; left and right neighbours come from
//     the adjacent lanes.
//  2. edt_rows: one 1024-lane work group per row.  The column distance
//     g(r, c) = |r - nearest caustic row of column c| is read off the mask
//     words (the set bit nearest to row r in the band's word, else in the
//     nearest band with one), then
//       d2(r, c) = min_q [(c - q)^2 + g(r, q)^2]
//     is searched outward from q = c: terms with |c - q| >= k are at least
//     k^2, so the search stops once k^2 reaches the best value found; no
//     term is skipped, so the minimum is exact.  A pixel still open after
//     WINDOW steps (a map with few caustics) takes the lower envelope of
//     parabolas (Meijster, Roerdink & Hesselink 2000): its row builds one
//     envelope per segment of 64 columns, a lane each, and the pixel visits
//     the segments outward from its own until no farther one can hold a
//     lower value.
// A map with a caustic pixel has one in some column, whose g is finite on
// every row, so a row whose g are all infinite belongs to a map with no
// caustic pixel at all.
// Output: sqrt(d2) * h, and the border-limited mark 4 d2 > b^2 where b is
// twice the distance (in pixels) from the centre to the nearest map edge.
#include "mlcc_internal.h"

namespace mlcc {

// Outward search steps per pixel before a row takes the lower envelope.
constexpr int EDT_WINDOW = 512;
constexpr int EDT_ROW_THREADS = 1024;
// maps are limited to nx + ny <= 30000, so a row has at most this many
// 64-column segments
constexpr int EDT_MAX_NX = 30000;
constexpr int EDT_MAX_SEGMENTS = (EDT_MAX_NX + 63) / 64;

// Four waves per work group, each over 16 rows of the band; the partial
// words meet in LDS.
constexpr int EDT_MASK_WAVES = 4;

__global__ void __launch_bounds__(64 * EDT_MASK_WAVES)
edt_mask_words(const int32_t *__restrict__ ncc, int32_t nx, int32_t ny,
               uint64_t *__restrict__ bits)
{
    __shared__ uint64_t part[EDT_MASK_WAVES][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + lane;
    const int band0 = blockIdx.y * 64;
    const int r0 = min(band0 + wave * (64 / EDT_MASK_WAVES), ny);
    const int r1 = min(r0 + 64 / EDT_MASK_WAVES, ny);
    const bool in = c < nx;
    const int cc = in ? c : nx - 1;   // loads of lanes past the last column stay in bounds
    uint64_t w = 0;
    if (r0 < r1) {   // wave-uniform: a wave past the last row only contributes zero
        int32_t cur = ncc[(int64_t)r0 * nx + cc];
        int32_t prev = r0 > 0 ? ncc[(int64_t)(r0 - 1) * nx + cc] : cur;
        for (int r = r0; r < r1; ++r) {
            const int64_t p = (int64_t)r * nx + cc;
            const int32_t next = r + 1 < ny ? ncc[p + nx] : cur;
            int32_t left = __shfl_up(cur, 1, 64);
            int32_t right = __shfl_down(cur, 1, 64);
            if (lane == 0 && cc > 0) left = ncc[p - 1];
            if (lane == 63 && cc + 1 < nx) right = ncc[p + 1];
            const bool edge = (cc > 0 && left != cur) || (cc + 1 < nx && right != cur) ||
                              (r > 0 && prev != cur) || (r + 1 < ny && next != cur);
            if (edge) w |= 1ull << (r - band0);
            prev = cur;
            cur = next;
        }
    }
    part[wave][lane] = w;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int v = 1; v < EDT_MASK_WAVES; ++v) w |= part[v][lane];
        if (in) bits[(int64_t)blockIdx.y * nx + c] = w;
    }
}

template <bool IN_LDS>
__global__ void __launch_bounds__(EDT_ROW_THREADS)
edt_rows(const uint64_t *__restrict__ bits, int32_t nx, int32_t ny, double h,
         int32_t *__restrict__ work, double *__restrict__ dist,
         uint8_t *__restrict__ border_limited)
{
    extern __shared__ int32_t lds[];
    __shared__ int32_t s_any, s_open;
    __shared__ int32_t s_cnt[EDT_MAX_SEGMENTS];   // envelope length per 64-column segment
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
            // four steps per round (eight independent LDS reads); the steps
            // past the exit point are terms of the same minimum, so the
            // result is unchanged
            int k = 1;
            for (; k <= EDT_WINDOW; k += 4) {
                if (k * k >= best || (c - k < 0 && c + k >= nx)) break;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int kk = k + u;
                    const int32_t a = c - kk >= 0 ? g[c - kk] : ginf;
                    const int32_t b = c + kk < nx ? g[c + kk] : ginf;
                    const int32_t m = min(a, b);
                    best = min(best, kk * kk + m * m);
                }
            }
            // an open pixel keeps its best value so far, marked by the sign
            d2[c] = k > EDT_WINDOW ? -best - 1 : best;
            open |= k > EDT_WINDOW;
        }
        if (open) s_open = 1;
        __syncthreads();
        if (s_open) {
            // The open pixels take the lower envelope of the row's parabolas
            // f(x, q) = (x - q)^2 + g(q)^2 (Meijster, Roerdink & Hesselink
            // 2000), built for each segment of 64 columns by one lane: sep(i,
            // u) is the first x at which parabola u is no higher than parabola
            // i (u > i), by floor division.  An open pixel visits the segments
            // outward from its own and stops once the gap to the nearer of the
            // next two reaches its best value; every value it meets is a term
            // of the minimum, so the result is exact.
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
            const int nseg = (nx + 63) >> 6;
            for (int j = tid; j < nseg; j += EDT_ROW_THREADS) {
                const int lo = j << 6, hi = min(lo + 64, nx);
                int32_t *ss = s + lo, *tt = t + lo;
                int q = 0;
                ss[0] = lo;
                tt[0] = 0;
                for (int u = lo + 1; u < hi; ++u) {
                    while (q >= 0 && f(tt[q], ss[q]) > f(tt[q], u)) --q;
                    if (q < 0) {
                        q = 0;
                        ss[0] = u;
                    } else {
                        const int64_t w = 1 + sep(ss[q], u);
                        if (w < nx) {
                            ++q;
                            ss[q] = u;
                            tt[q] = (int32_t)w;
                        }
                    }
                }
                s_cnt[j] = q + 1;
            }
            __syncthreads();
            // segment j's envelope at column x: its last parabola starting at
            // or before x
            auto seg_min = [&](int j, int x) {
                const int32_t *ss = s + (j << 6), *tt = t + (j << 6);
                int lo = 0, hi = s_cnt[j] - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (tt[mid] <= x) lo = mid;
                    else hi = mid - 1;
                }
                return f(x, ss[lo]);
            };
            for (int c = tid; c < nx; c += EDT_ROW_THREADS) {
                if (d2[c] >= 0) continue;
                const int j0 = c >> 6;
                int64_t best = min((int64_t)(-d2[c] - 1), seg_min(j0, c));
                for (int k = 1;; ++k) {
                    const int jl = j0 - k, jr = j0 + k;
                    const bool hl = jl >= 0, hr = jr < nseg;
                    if (!hl && !hr) break;
                    const int64_t gl = hl ? c - ((jl << 6) + 63) : INT64_MAX;
                    const int64_t gr = hr ? (jr << 6) - c : INT64_MAX;
                    const int64_t gap = min(gl, gr);
                    if (gap * gap >= best) break;
                    if (hl && gl * gl < best) best = min(best, seg_min(jl, c));
                    if (hr && gr * gr < best) best = min(best, seg_min(jr, c));
                }
                d2[c] = (int32_t)best;
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
    if ((int64_t)nx + ny > EDT_MAX_NX)
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
    hipLaunchKernelGGL(edt_mask_words, dim3((unsigned)ceil_div(nx, 64), (unsigned)bands),
                       dim3(64 * EDT_MASK_WAVES), 0, c->stream, ncc, nx, ny, bits);
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
