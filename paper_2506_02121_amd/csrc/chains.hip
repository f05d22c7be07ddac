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

template <bool INTERLEAVED>
__global__ void __launch_bounds__(64)
nearest_kernel(int32_t n, const double2 *__restrict__ a2, const double *__restrict__ a_re,
               const double *__restrict__ a_im, const double *__restrict__ b_re,
               const double *__restrict__ b_im, int32_t *__restrict__ perm,
               int32_t *__restrict__ hits, PairAux *__restrict__ aux)
{
    const int k = blockIdx.x * 64 + threadIdx.x;
    double ax = 0.0, ay = 0.0;
    if (k < n) {
        if (INTERLEAVED) {
            const double2 a = a2[k];
            ax = a.x;
            ay = a.y;
        } else {
            ax = a_re[k];
            ay = a_im[k];
        }
    }
    double best = INFINITY;
    int bi = -1;
    for (int j = 0; j < n; ++j) {
        const double dx = ax - b_re[j], dy = ay - b_im[j];
        const double d = fma(dx, dx, dy * dy);
        if (d < best) {
            best = d;
            bi = j;
        }
    }
    if (k >= n) return;
    perm[k] = bi;
    if (bi < 0) {
        atomicOr(&aux->bad, 1);
        return;
    }
    atomicAdd(&hits[bi], 1);
    // non-negative doubles order like their bit patterns
    atomicMax(&aux->maxbits, (unsigned long long)__double_as_longlong(best));
}

__global__ void check_hits(int32_t n, const int32_t *__restrict__ hits, PairAux *__restrict__ aux)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && hits[k] != 1) atomicOr(&aux->bad, 1);
}

mlcc_status pair_all(Ctx *c, const std::vector<PairJob> &jobs, double tol, double *maxdist)
{
    if (maxdist) *maxdist = 0.0;
    if (jobs.empty()) return MLCC_OK;
    int64_t total = 0;
    for (const PairJob &j : jobs) {
        if (j.n > 0x7fffffff) return fail(MLCC_ERR_INVALID, "row too long to pair");
        total += j.n;
    }
    const size_t aux_bytes = jobs.size() * sizeof(PairAux);
    MLCC_TRY(c->match_aux.reserve(aux_bytes + (size_t)total * sizeof(int32_t)));
    PairAux *aux = c->match_aux.as<PairAux>();
    int32_t *hits = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(c->match_aux.p) + aux_bytes);
    MLCC_HIP(hipMemsetAsync(c->match_aux.p, 0, aux_bytes + (size_t)total * sizeof(int32_t),
                            c->stream));
    int64_t off = 0;
    for (size_t i = 0; i < jobs.size(); ++i) {
        const PairJob &j = jobs[i];
        const unsigned blocks = (unsigned)ceil_div(j.n, 64);
        if (j.a2)
            hipLaunchKernelGGL(nearest_kernel<true>, dim3(blocks), dim3(64), 0, c->stream,
                               (int32_t)j.n, j.a2, nullptr, nullptr, j.b_re, j.b_im, j.perm,
                               hits + off, aux + i);
        else
            hipLaunchKernelGGL(nearest_kernel<false>, dim3(blocks), dim3(64), 0, c->stream,
                               (int32_t)j.n, nullptr, j.a_re, j.a_im, j.b_re, j.b_im, j.perm,
                               hits + off, aux + i);
        hipLaunchKernelGGL(check_hits, dim3((unsigned)ceil_div(j.n, 256)), dim3(256), 0,
                           c->stream, (int32_t)j.n, hits + off, aux + i);
        off += j.n;
    }
    MLCC_HIP(hipGetLastError());
    std::vector<PairAux> h(jobs.size());
    MLCC_HIP(hipMemcpyAsync(h.data(), aux, aux_bytes, hipMemcpyDeviceToHost, c->stream));
    MLCC_HIP(hipStreamSynchronize(c->stream));
    double md = 0.0;
    for (size_t i = 0; i < jobs.size(); ++i) {
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

// scratch[b][label[k]] = src[b][k] for nb rows
__global__ void scatter_rows(int64_t n_r, int64_t nb, const double *__restrict__ src_re,
                             const double *__restrict__ src_im, const int32_t *__restrict__ label,
                             double *__restrict__ dst_re, double *__restrict__ dst_im)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_r * nb) return;
    const int64_t b = t / n_r, k = t - b * n_r;
    const int64_t to = b * n_r + label[k];
    dst_re[to] = src_re[t];
    dst_im[to] = src_im[t];
}

mlcc_status relabel_rows(Ctx *c, double *re, double *im, int64_t n_r, int64_t row0,
                         int64_t row1, const int32_t *label)
{
    if (row1 <= row0) return MLCC_OK;
    const int64_t budget = (int64_t)64 << 20; // bytes of scratch
    int64_t B = std::max<int64_t>(1, budget / (2 * (int64_t)sizeof(double) * n_r));
    B = std::min<int64_t>(B, row1 - row0);
    MLCC_TRY(c->relabel.reserve((size_t)2 * B * n_r * sizeof(double)));
    double *sre = c->relabel.as<double>(), *sim = sre + B * n_r;
    for (int64_t r = row0; r < row1; r += B) {
        const int64_t nb = std::min<int64_t>(B, row1 - r);
        const int64_t tot = nb * n_r;
        hipLaunchKernelGGL(scatter_rows, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                           c->stream, n_r, nb, re + r * n_r, im + r * n_r, label, sre, sim);
        MLCC_HIP(hipGetLastError());
        MLCC_HIP(hipMemcpyAsync(re + r * n_r, sre, tot * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream));
        MLCC_HIP(hipMemcpyAsync(im + r * n_r, sim, tot * sizeof(double), hipMemcpyDeviceToDevice,
                                c->stream));
    }
    return MLCC_OK;
}

} // namespace mlcc
