// Joining chains (Sec. 4.3 and its footnote): a row computed twice -- the
// shared boundary of two subchains, or phi = 2 pi against phi = 0 -- holds
// the same root set under two labellings.  Each root of one copy is paired
// with its nearest root of the other copy, the pairing is checked to be
// one-to-one and tight, and blocks of rows are relabelled through it.
//
// Nearest roots through a grid per pairing: the second copy's n points are
// binned into g x g square cells (g = ceil(sqrt(n / 2)), about two points
// per cell) over their bounding box by a count, a scan and a fill; a point of
// the first copy then visits the cells around its own in rings of growing
// Chebyshev radius r and stops once its best squared distance is below the
// square of a lower bound on the distance to every cell outside the rings so
// far (less a margin for the rounding of the cell edges).  Ties go to the
// lower index, so the pairing is the brute-force scan's: the first nearest
// point in index order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "mlcc_internal.h"

namespace mlcc {

struct PairAux {
    int32_t bad;                // pairing not one-to-one
    int32_t pad;
    unsigned long long maxbits; // bit pattern of the largest paired squared distance
};

// A pairing job as the kernels see it: its points start at hits_off in the
// per-point arrays (hits, the grid's point list), its g * g cells at cell_off.
struct PairJobDev {
    const double2 *a2;
    const double *a_re, *a_im, *b_re, *b_im;
    int32_t *perm;
    int64_t n, hits_off, cell_off;
    int32_t g, pad;
};

// Grid of one job: origin, cell width, and a margin for the rounding of the
// cell edges (coordinates are binned by floor((x - x0) / h)).
struct PairGrid {
    double x0, y0, h, margin;
};

__device__ __forceinline__ int grid_cell(double v, double v0, double h, int g)
{
    const double t = floor((v - v0) / h);
    if (!(t >= 0.0)) return 0;   // also a coordinate that is not finite
    return t > (double)(g - 1) ? g - 1 : (int)t;
}

// Bounding box of each job's second copy and its grid (one work group per job).
__global__ void __launch_bounds__(256)
grid_bounds(const PairJobDev *__restrict__ jobs, PairGrid *__restrict__ grids)
{
    __shared__ double red[4][4];
    const PairJobDev J = jobs[blockIdx.x];
    double xl = INFINITY, xh = -INFINITY, yl = INFINITY, yh = -INFINITY;
    for (int64_t j = threadIdx.x; j < J.n; j += 256) {
        const double x = J.b_re[j], y = J.b_im[j];
        xl = fmin(xl, x); xh = fmax(xh, x); yl = fmin(yl, y); yh = fmax(yh, y);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        xl = fmin(xl, __shfl_xor(xl, off, 64)); xh = fmax(xh, __shfl_xor(xh, off, 64));
        yl = fmin(yl, __shfl_xor(yl, off, 64)); yh = fmax(yh, __shfl_xor(yh, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w][0] = xl; red[w][1] = xh; red[w][2] = yl; red[w][3] = yh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < 4; ++q) {
            xl = fmin(xl, red[q][0]); xh = fmax(xh, red[q][1]);
            yl = fmin(yl, red[q][2]); yh = fmax(yh, red[q][3]);
        }
        double h = fmax(xh - xl, yh - yl) / (double)J.g;
        if (!(h > 0.0) || !isfinite(h)) h = 1.0;   // one point, or all equal
        const double x0 = isfinite(xl) ? xl : 0.0, y0 = isfinite(yl) ? yl : 0.0;
        grids[blockIdx.x] = PairGrid{x0, y0, h, 1e-12 * (fabs(x0) + fabs(y0) + J.g * h)};
    }
}

// Points of the second copy per cell (one thread per point).
__global__ void __launch_bounds__(64)
grid_count(const PairJobDev *__restrict__ jobs, const int2 *__restrict__ blk,
           const PairGrid *__restrict__ grids, int32_t *__restrict__ cnt)
{
    const int2 q = blk[blockIdx.x];
    const PairJobDev J = jobs[q.x];
    const int64_t j = (int64_t)q.y * 64 + threadIdx.x;
    if (j >= J.n) return;
    const PairGrid G = grids[q.x];
    const int cx = grid_cell(J.b_re[j], G.x0, G.h, J.g), cy = grid_cell(J.b_im[j], G.y0, G.h, J.g);
    atomicAdd(&cnt[J.cell_off + (int64_t)cy * J.g + cx], 1);
}

// First slot of every cell (exclusive scan of the counts, one work group per
// job); the counts are cleared to serve as the fill's cursors.
__global__ void __launch_bounds__(256)
grid_scan(const PairJobDev *__restrict__ jobs, int32_t *__restrict__ cnt,
          int32_t *__restrict__ start)
{
    __shared__ int32_t wave_tot[4];
    __shared__ int32_t carry;
    const PairJobDev J = jobs[blockIdx.x];
    const int64_t cells = (int64_t)J.g * J.g;
    int32_t *c = cnt + J.cell_off, *st = start + J.cell_off;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < cells; base += 256) {
        const int64_t i = base + tid;
        const int32_t v0 = i < cells ? c[i] : 0;
        int32_t v = v0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t t = __shfl_up(v, off, 64);
            if (lane >= off) v += t;
        }
        if (lane == 63) wave_tot[w] = v;
        __syncthreads();
        int32_t add = carry;
        for (int q = 0; q < w; ++q) add += wave_tot[q];
        v += add;
        if (i < cells) {
            st[i] = v - v0;
            c[i] = 0;
        }
        __syncthreads();
        if (tid == 255) carry = v;
        __syncthreads();
    }
}

// Point list of every cell (one thread per point; order within a cell is
// arbitrary, ties are broken by index in the search).
__global__ void __launch_bounds__(64)
grid_fill(const PairJobDev *__restrict__ jobs, const int2 *__restrict__ blk,
          const PairGrid *__restrict__ grids, const int32_t *__restrict__ start,
          int32_t *__restrict__ cur, int32_t *__restrict__ pts)
{
    const int2 q = blk[blockIdx.x];
    const PairJobDev J = jobs[q.x];
    const int64_t j = (int64_t)q.y * 64 + threadIdx.x;
    if (j >= J.n) return;
    const PairGrid G = grids[q.x];
    const int cx = grid_cell(J.b_re[j], G.x0, G.h, J.g), cy = grid_cell(J.b_im[j], G.y0, G.h, J.g);
    const int64_t cell = J.cell_off + (int64_t)cy * J.g + cx;
    const int32_t slot = atomicAdd(&cur[cell], 1);
    pts[J.hits_off + start[cell] + slot] = (int32_t)j;
}

// One launch for every job: block q works on job blk[q].x, points
// 64 blk[q].y .. +63 of it.  Each lane searches the grid of the other copy
// for its point's nearest; the hit counts and the largest distance go to the
// job's slots.
__global__ void __launch_bounds__(64)
nearest_grid(const PairJobDev *__restrict__ jobs, const int2 *__restrict__ blk,
             const PairGrid *__restrict__ grids, const int32_t *__restrict__ start,
             const int32_t *__restrict__ cnt, const int32_t *__restrict__ pts,
             int32_t *__restrict__ hits, PairAux *__restrict__ aux)
{
    const int2 q = blk[blockIdx.x];
    const PairJobDev J = jobs[q.x];
    const int64_t k = (int64_t)q.y * 64 + threadIdx.x;
    if (k >= J.n) return;
    double ax, ay;
    if (J.a2) {
        const double2 v = J.a2[k];
        ax = v.x;
        ay = v.y;
    } else {
        ax = J.a_re[k];
        ay = J.a_im[k];
    }
    const PairGrid G = grids[q.x];
    const int g = J.g;
    const int cx = grid_cell(ax, G.x0, G.h, g), cy = grid_cell(ay, G.y0, G.h, g);
    const int32_t *st = start + J.cell_off, *ct = cnt + J.cell_off, *pl = pts + J.hits_off;
    double best = INFINITY;
    int bi = -1;
    auto visit = [&](int cj, int ci) {
        const int64_t cell = (int64_t)cj * g + ci;
        const int32_t s0 = st[cell], n0 = ct[cell];
        for (int32_t t = 0; t < n0; ++t) {
            const int32_t p = pl[s0 + t];
            const double dx = ax - J.b_re[p], dy = ay - J.b_im[p];
            const double d = fma(dx, dx, dy * dy);
            if (d < best || (d == best && p < bi)) {
                best = d;
                bi = p;
            }
        }
    };
    for (int r = 0; r < g; ++r) {
        // the cells at Chebyshev distance r from (cx, cy): whole rows at the
        // ring's top and bottom, the two ends of the rows between
        const int j0 = max(cy - r, 0), j1 = min(cy + r, g - 1);
        const int i0 = max(cx - r, 0), i1 = min(cx + r, g - 1);
        for (int cj = j0; cj <= j1; ++cj) {
            if (cj == cy - r || cj == cy + r) {
                for (int ci = i0; ci <= i1; ++ci) visit(cj, ci);
            } else {
                if (cx - r >= 0) visit(cj, cx - r);
                if (r > 0 && cx + r <= g - 1) visit(cj, cx + r);
            }
        }
        // lower bound on the distance to any point in a cell outside radius r
        double L = INFINITY;
        if (cx + r + 1 < g) L = fmin(L, G.x0 + (cx + r + 1) * G.h - ax);
        if (cx - r > 0) L = fmin(L, ax - (G.x0 + (cx - r) * G.h));
        if (cy + r + 1 < g) L = fmin(L, G.y0 + (cy + r + 1) * G.h - ay);
        if (cy - r > 0) L = fmin(L, ay - (G.y0 + (cy - r) * G.h));
        if (L == INFINITY) break;   // every cell visited
        const double Lm = L - G.margin;
        if (Lm > 0.0 && best <= Lm * Lm) break;
    }
    J.perm[k] = bi;
    if (bi < 0) {
        atomicOr(&aux[q.x].bad, 1);
        return;
    }
    atomicAdd(&hits[J.hits_off + bi], 1);
    // non-negative doubles order like their bit patterns
    atomicMax(&aux[q.x].maxbits, (unsigned long long)__double_as_longlong(best));
}

// Every point of the second copy must be hit exactly once.
__global__ void check_hits_jobs(const int64_t *__restrict__ hits_off, int32_t n_jobs,
                                const int32_t *__restrict__ hits, int64_t total,
                                PairAux *__restrict__ aux)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total || hits[t] == 1) return;
    int lo = 0, hi = n_jobs - 1;   // last job with hits_off <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (hits_off[mid] <= t) lo = mid; else hi = mid - 1;
    }
    atomicOr(&aux[lo].bad, 1);
}

mlcc_status pair_all(Ctx *c, const std::vector<PairJob> &jobs, double tol, double *maxdist)
{
    if (maxdist) *maxdist = 0.0;
    if (jobs.empty()) return MLCC_OK;
    const int32_t nj = (int32_t)jobs.size();
    std::vector<PairJobDev> jd(nj);
    std::vector<int64_t> hoff(nj);
    std::vector<int2> blk;
    int64_t total = 0, cells = 0;
    for (int32_t i = 0; i < nj; ++i) {
        const PairJob &j = jobs[i];
        if (j.n > 0x7fffffff) return fail(MLCC_ERR_INVALID, "row too long to pair");
        // about two points per cell
        const int32_t g = (int32_t)std::min<double>(
            4096.0, std::max(1.0, std::ceil(std::sqrt((double)j.n / 2.0))));
        jd[i] = PairJobDev{j.a2, j.a_re, j.a_im, j.b_re, j.b_im, j.perm, j.n, total, cells, g, 0};
        hoff[i] = total;
        for (int64_t q = 0; q < ceil_div(j.n, 64); ++q) blk.push_back(make_int2(i, (int)q));
        total += j.n;
        cells += (int64_t)g * g;
    }
    // device layout: aux[nj] | hits[total] | counts[cells] | jobs[nj] | hits_off[nj] |
    // blk[...] | grids[nj] | starts[cells] | points[total]
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_hits = al(nj * sizeof(PairAux));
    const size_t o_cnt = al(o_hits + (size_t)total * sizeof(int32_t));
    const size_t o_jobs = al(o_cnt + (size_t)cells * sizeof(int32_t));
    const size_t o_hoff = al(o_jobs + nj * sizeof(PairJobDev));
    const size_t o_blk = al(o_hoff + nj * sizeof(int64_t));
    const size_t o_grid = al(o_blk + blk.size() * sizeof(int2));
    const size_t o_start = al(o_grid + nj * sizeof(PairGrid));
    const size_t o_pts = al(o_start + (size_t)cells * sizeof(int32_t));
    const size_t bytes = o_pts + (size_t)total * sizeof(int32_t);
    MLCC_TRY(c->match_aux.reserve(bytes));
    char *base = static_cast<char *>(c->match_aux.p);
    PairAux *aux = reinterpret_cast<PairAux *>(base);
    int32_t *hits = reinterpret_cast<int32_t *>(base + o_hits);
    int32_t *cnt = reinterpret_cast<int32_t *>(base + o_cnt);
    const PairJobDev *djobs = reinterpret_cast<const PairJobDev *>(base + o_jobs);
    const int2 *dblk = reinterpret_cast<const int2 *>(base + o_blk);
    PairGrid *grids = reinterpret_cast<PairGrid *>(base + o_grid);
    int32_t *starts = reinterpret_cast<int32_t *>(base + o_start);
    int32_t *pts = reinterpret_cast<int32_t *>(base + o_pts);
    MLCC_HIP(hipMemsetAsync(base, 0, o_jobs, c->stream));   // aux, hits, counts
    MLCC_HIP(hipMemcpyAsync(base + o_jobs, jd.data(), nj * sizeof(PairJobDev),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(base + o_hoff, hoff.data(), nj * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(base + o_blk, blk.data(), blk.size() * sizeof(int2),
                            hipMemcpyHostToDevice, c->stream));
    const unsigned nb = (unsigned)blk.size();
    hipLaunchKernelGGL(grid_bounds, dim3((unsigned)nj), dim3(256), 0, c->stream, djobs, grids);
    hipLaunchKernelGGL(grid_count, dim3(nb), dim3(64), 0, c->stream, djobs, dblk, grids, cnt);
    hipLaunchKernelGGL(grid_scan, dim3((unsigned)nj), dim3(256), 0, c->stream, djobs, cnt, starts);
    hipLaunchKernelGGL(grid_fill, dim3(nb), dim3(64), 0, c->stream, djobs, dblk, grids, starts,
                       cnt, pts);
    hipLaunchKernelGGL(nearest_grid, dim3(nb), dim3(64), 0, c->stream, djobs, dblk, grids, starts,
                       cnt, pts, hits, aux);
    hipLaunchKernelGGL(check_hits_jobs, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                       c->stream, reinterpret_cast<const int64_t *>(base + o_hoff), nj, hits,
                       total, aux);
    MLCC_HIP(hipGetLastError());
    std::vector<PairAux> h(nj);
    MLCC_HIP(hipMemcpyAsync(h.data(), aux, nj * sizeof(PairAux), hipMemcpyDeviceToHost, c->stream));
    // (the host vectors above stay alive until this synchronisation)
    MLCC_HIP(hipStreamSynchronize(c->stream));
    double md = 0.0;
    for (int32_t i = 0; i < nj; ++i) {
        double d2;
        memcpy(&d2, &h[i].maxbits, sizeof d2);
        const double d = std::sqrt(d2);
        md = std::max(md, d);
        if (h[i].bad)
            return fail(MLCC_ERR_MATCH, "duplicate rows of %lld roots do not pair one-to-one",
                        (long long)jobs[i].n);
        if (!(d <= tol))
            return fail(MLCC_ERR_MATCH, "duplicate rows pair at distance %.3g > %.3g", d, tol);
    }
    if (maxdist) *maxdist = md;
    return MLCC_OK;
}

// A run of rows of one array whose columns are relabelled: new[b][label[k]]
// = old[b][k] for b < rows.  `elem0` is its first element in the chunk's
// scratch.
struct RelabelSeg {
    double *re, *im;
    const int32_t *label;
    int64_t n_r, rows, elem0;
};

__device__ __forceinline__ int find_seg(const RelabelSeg *segs, int nseg, int64_t t)
{
    int lo = 0, hi = nseg - 1;   // last segment with elem0 <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].elem0 <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void relabel_scatter(const RelabelSeg *__restrict__ segs, int32_t nseg, int64_t total,
                                double *__restrict__ sre, double *__restrict__ sim)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const RelabelSeg g = segs[find_seg(segs, nseg, t)];
    const int64_t e = t - g.elem0, b = e / g.n_r, k = e - b * g.n_r;
    const int64_t to = g.elem0 + b * g.n_r + g.label[k];
    sre[to] = g.re[e];
    sim[to] = g.im[e];
}

__global__ void relabel_back(const RelabelSeg *__restrict__ segs, int32_t nseg, int64_t total,
                             const double *__restrict__ sre, const double *__restrict__ sim)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const RelabelSeg g = segs[find_seg(segs, nseg, t)];
    const int64_t e = t - g.elem0;
    g.re[e] = sre[t];
    g.im[e] = sim[t];
}

// In place through LDS, one work group per row and plane when a row fits:
// the row is read coalesced, scattered into LDS by its labels, and written
// back coalesced.  Segments count rows here (elem0 = first row).
// (1024 lanes per work group: a long row leaves room for one work group per
// CU, so its loads need many lanes in flight.)
constexpr int RELABEL_THREADS = 1024;

__global__ void __launch_bounds__(RELABEL_THREADS)
relabel_rows_lds(const RelabelSeg *__restrict__ segs, int32_t nseg)
{
    extern __shared__ double row[];
    const int64_t t = blockIdx.x;
    const RelabelSeg g = segs[find_seg(segs, nseg, t)];
    double *p = (blockIdx.y ? g.im : g.re) + (t - g.elem0) * g.n_r;
    for (int64_t k = threadIdx.x; k < g.n_r; k += RELABEL_THREADS) row[g.label[k]] = p[k];
    __syncthreads();
    for (int64_t k = threadIdx.x; k < g.n_r; k += RELABEL_THREADS) p[k] = row[k];
}

static mlcc_status relabel_lds(Ctx *c, const std::vector<RelabelJob> &jobs, int64_t max_nr)
{
    std::vector<RelabelSeg> segs;
    int64_t rows = 0;
    for (const RelabelJob &j : jobs) {
        if (j.row1 <= j.row0) continue;
        segs.push_back(RelabelSeg{j.re + j.row0 * j.n_r, j.im + j.row0 * j.n_r, j.label, j.n_r,
                                  j.row1 - j.row0, rows});
        rows += j.row1 - j.row0;
    }
    if (rows == 0) return MLCC_OK;
    if (rows > 0x7fffffff) return fail(MLCC_ERR_INVALID, "too many rows to relabel");
    MLCC_TRY(c->relabel.reserve(segs.size() * sizeof(RelabelSeg)));
    RelabelSeg *dsegs = c->relabel.as<RelabelSeg>();
    MLCC_HIP(hipMemcpyAsync(dsegs, segs.data(), segs.size() * sizeof(RelabelSeg),
                            hipMemcpyHostToDevice, c->stream));
    const size_t lds = (size_t)max_nr * sizeof(double);
    hipLaunchKernelGGL(relabel_rows_lds, dim3((unsigned)rows, 2), dim3(RELABEL_THREADS), lds,
                       c->stream, dsegs, (int32_t)segs.size());
    MLCC_HIP(hipGetLastError());
    // the segment table is read by the kernel: keep it until it is done
    MLCC_HIP(hipStreamSynchronize(c->stream));
    return MLCC_OK;
}

mlcc_status relabel_all(Ctx *c, const std::vector<RelabelJob> &jobs)
{
    if (jobs.empty()) return MLCC_OK;
    int64_t max_nr = 0;
    for (const RelabelJob &j : jobs) max_nr = std::max(max_nr, j.n_r);
    int lds_max = 0;
    MLCC_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    if (max_nr >= 1 && (size_t)max_nr * sizeof(double) <= (size_t)lds_max) {
        if ((size_t)max_nr * sizeof(double) > 65536)
            MLCC_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&relabel_rows_lds),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(max_nr * sizeof(double))));
        return relabel_lds(c, jobs, max_nr);
    }
    const int64_t budget = (int64_t)16 << 20;   // elements per chunk (256 MiB of scratch)
    // split the jobs into chunks of whole rows, at most `budget` elements each
    std::vector<RelabelSeg> segs;
    std::vector<std::pair<size_t, int64_t>> chunks;   // (first segment, elements)
    int64_t fill = 0;
    size_t first = 0;
    for (const RelabelJob &j : jobs) {
        if (j.n_r < 1 || j.n_r > budget)
            return fail(MLCC_ERR_INVALID, "row of %lld roots too long to relabel",
                        (long long)j.n_r);
        int64_t r = j.row0;
        while (r < j.row1) {
            if (fill + j.n_r > budget) {
                chunks.emplace_back(first, fill);
                first = segs.size();
                fill = 0;
            }
            const int64_t nb = std::min<int64_t>(j.row1 - r, (budget - fill) / j.n_r);
            segs.push_back(RelabelSeg{j.re + r * j.n_r, j.im + r * j.n_r, j.label, j.n_r, nb, fill});
            fill += nb * j.n_r;
            r += nb;
        }
    }
    if (fill) chunks.emplace_back(first, fill);
    int64_t max_fill = 0;
    for (auto &ch : chunks) max_fill = std::max(max_fill, ch.second);
    const size_t seg_bytes = (segs.size() * sizeof(RelabelSeg) + 255) & ~(size_t)255;
    MLCC_TRY(c->relabel.reserve(seg_bytes + (size_t)2 * max_fill * sizeof(double)));
    char *base = static_cast<char *>(c->relabel.p);
    RelabelSeg *dsegs = reinterpret_cast<RelabelSeg *>(base);
    double *sre = reinterpret_cast<double *>(base + seg_bytes), *sim = sre + max_fill;
    MLCC_HIP(hipMemcpyAsync(dsegs, segs.data(), segs.size() * sizeof(RelabelSeg),
                            hipMemcpyHostToDevice, c->stream));
    for (size_t i = 0; i < chunks.size(); ++i) {
        const size_t s0 = chunks[i].first;
        const size_t s1 = i + 1 < chunks.size() ? chunks[i + 1].first : segs.size();
        const int64_t tot = chunks[i].second;
        const unsigned g = (unsigned)ceil_div(tot, 256);
        hipLaunchKernelGGL(relabel_scatter, dim3(g), dim3(256), 0, c->stream, dsegs + s0,
                           (int32_t)(s1 - s0), tot, sre, sim);
        hipLaunchKernelGGL(relabel_back, dim3(g), dim3(256), 0, c->stream, dsegs + s0,
                           (int32_t)(s1 - s0), tot, sre, sim);
    }
    MLCC_HIP(hipGetLastError());
    // the segment table is read by the kernels: keep it until they are done
    MLCC_HIP(hipStreamSynchronize(c->stream));
    return MLCC_OK;
}

} // namespace mlcc
