// Joining chains (Sec. 4.3 and its footnote): a row computed twice -- the
// shared boundary of two subchains, or phi = 2 pi against phi = 0 -- holds
// the same root set under two labellings.  Each root of one copy is paired
// with its nearest root of the other copy (brute force: every lane scans the
// other copy through wave-uniform scalar loads), the pairing is checked to be
// one-to-one and tight, and blocks of rows are relabelled through it.
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

// A pairing job as the kernels see it.
struct PairJobDev {
    const double2 *a2;
    const double *a_re, *a_im, *b_re, *b_im;
    int32_t *perm;
    int64_t n, hits_off;
};

// One launch for every job: block q works on job blk_job[q], points
// 64 blk_idx[q] .. +63 of it.  Each lane scans the other copy and keeps the
// nearest point; the hit counts and the largest distance go to the job's
// slots.
__global__ void __launch_bounds__(64)
nearest_jobs(const PairJobDev *__restrict__ jobs, const int2 *__restrict__ blk,
             int32_t *__restrict__ hits, PairAux *__restrict__ aux)
{
    const int2 q = blk[blockIdx.x];
    const PairJobDev J = jobs[q.x];
    const int64_t k = (int64_t)q.y * 64 + threadIdx.x;
    double ax = 0.0, ay = 0.0;
    if (k < J.n) {
        if (J.a2) {
            const double2 v = J.a2[k];
            ax = v.x;
            ay = v.y;
        } else {
            ax = J.a_re[k];
            ay = J.a_im[k];
        }
    }
    double best = INFINITY;
    int bi = -1;
    for (int j = 0; j < (int)J.n; ++j) {
        const double dx = ax - J.b_re[j], dy = ay - J.b_im[j];
        const double d = fma(dx, dx, dy * dy);
        if (d < best) {
            best = d;
            bi = j;
        }
    }
    if (k >= J.n) return;
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
    int64_t total = 0;
    for (int32_t i = 0; i < nj; ++i) {
        const PairJob &j = jobs[i];
        if (j.n > 0x7fffffff) return fail(MLCC_ERR_INVALID, "row too long to pair");
        jd[i] = PairJobDev{j.a2, j.a_re, j.a_im, j.b_re, j.b_im, j.perm, j.n, total};
        hoff[i] = total;
        for (int64_t q = 0; q < ceil_div(j.n, 64); ++q) blk.push_back(make_int2(i, (int)q));
        total += j.n;
    }
    // device layout: aux[nj] | hits[total] | jobs[nj] | hits_off[nj] | blk[...]
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_hits = al(nj * sizeof(PairAux));
    const size_t o_jobs = al(o_hits + (size_t)total * sizeof(int32_t));
    const size_t o_hoff = al(o_jobs + nj * sizeof(PairJobDev));
    const size_t o_blk = al(o_hoff + nj * sizeof(int64_t));
    const size_t bytes = o_blk + blk.size() * sizeof(int2);
    MLCC_TRY(c->match_aux.reserve(bytes));
    char *base = static_cast<char *>(c->match_aux.p);
    PairAux *aux = reinterpret_cast<PairAux *>(base);
    int32_t *hits = reinterpret_cast<int32_t *>(base + o_hits);
    MLCC_HIP(hipMemsetAsync(base, 0, o_jobs, c->stream));
    MLCC_HIP(hipMemcpyAsync(base + o_jobs, jd.data(), nj * sizeof(PairJobDev),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(base + o_hoff, hoff.data(), nj * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->stream));
    MLCC_HIP(hipMemcpyAsync(base + o_blk, blk.data(), blk.size() * sizeof(int2),
                            hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(nearest_jobs, dim3((unsigned)blk.size()), dim3(64), 0, c->stream,
                       reinterpret_cast<const PairJobDev *>(base + o_jobs),
                       reinterpret_cast<const int2 *>(base + o_blk), hits, aux);
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

mlcc_status relabel_all(Ctx *c, const std::vector<RelabelJob> &jobs)
{
    if (jobs.empty()) return MLCC_OK;
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
