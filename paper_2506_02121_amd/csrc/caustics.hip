// Caustic mapping: the lens equation of Sec. 3.1 in complex form, with the
// compensating sheet extended to infinity (App. A), evaluated at arbitrary
// points (the critical-curve roots give the caustics):
//   w = (1 - kappa_s) z + gamma conj(z) - sum_i m_i / conj(z - z_i),
// and m_i / conj(d) = m_i d / |d|^2.  A rectangular field (Sec. 4.2, App. B)
// adds its sheet's Taylor terms: gamma becomes gamma - d0 and
//   w -= sum_k d_2k conj(z)^(2k+1) / (2k+1).
// One lane per point; star tiles stream through LDS, and groups of eight
// star terms share one refined reciprocal.
#include <type_traits>

#include "mlcc_internal.h"
#include "term_groups.h"

namespace mlcc {

// Reciprocals in the lens map take two Newton steps (about an ulp; the
// root finder's accept test needs only one), shared by groups of star terms
// as in the root finder.
constexpr int RCP_MAP = 2;

// G consecutive star terms m_i d / |d|^2 added to (sr, si).
template <bool EQUAL, int G, class T>
__device__ __forceinline__ void add_map_group(double &sr, double &si, double x, double y,
                                              const T *r)
{
    double dx[G], dy[G], q[G], iq[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        dx[j] = x - r[j].x;
        dy[j] = y - r[j].y;
        q[j] = fma(dx[j], dx[j], dy[j] * dy[j]);
    }
    rcp_group<G, RCP_MAP>(q, iq);
#pragma unroll
    for (int j = 0; j < G; ++j) {
        double v = iq[j];
        if constexpr (!EQUAL) v *= r[j].z;
        sr = fma(v, dx[j], sr);
        si = fma(v, dy[j], si);
    }
}

template <bool EQUAL>
__global__ void __launch_bounds__(64)
map_caustics_f64(const typename std::conditional<EQUAL, double2, double4>::type *__restrict__ stars,
                 double m0, int32_t n_stars, int64_t count, const double *__restrict__ zr,
                 const double *__restrict__ zi, double *__restrict__ wr,
                 double *__restrict__ wi, double a, double gamma,
                 const double *__restrict__ pmap, int32_t n_poly)
{
    using T = typename std::conditional<EQUAL, double2, double4>::type;
    __shared__ T tiles[128];
    const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool valid = k < count;
    const double x = valid ? zr[k] : 0.0;
    const double y = valid ? zi[k] : 0.0;
    double sr = 0.0, si = 0.0;
    stream_tiles_grouped(stars, n_stars, tiles, [&](auto g, const T *r) {
        add_map_group<EQUAL, decltype(g)::value>(sr, si, x, y, r);
    });
    if (EQUAL) {   // every mass equals m0
        sr *= m0;
        si *= m0;
    }
    if (n_poly > 0) {   // + conj(sum_k pmap_k z^(2k+1)), subtracted below with the stars
        const double w2r = x * x - y * y, w2i = 2.0 * x * y;
        double pr = pmap[n_poly - 1], pi = 0.0;
        for (int k = n_poly - 2; k >= 0; --k) {
            const double tr = pr * w2r - pi * w2i + pmap[k];
            pi = pr * w2i + pi * w2r;
            pr = tr;
        }
        // z^3 (...) : multiply by z^2 then z
        const double qr = pr * w2r - pi * w2i, qi = pr * w2i + pi * w2r;
        sr += qr * x - qi * y;
        si -= qr * y + qi * x;   // the conjugate's imaginary part enters with a sign flip
    }
    if (valid) {
        wr[k] = fma(a, x, gamma * x) - sr;
        wi[k] = fma(a, y, -gamma * y) - si;
    }
}

mlcc_status launch_map_caustics(Ctx *c, int64_t count, const double *zr, const double *zi,
                                double *wr, double *wi)
{
    const int64_t blocks = ceil_div(count, 64);
    if (blocks > 0x7fffffff) return fail(MLCC_ERR_INVALID, "count too large");
    const double a = 1.0 - c->kappa_s;
    const SheetPoly sp = sheet_poly(c->reals[0]);
    const double gamma = c->gamma - sp.d0;
    const double *pmap = nullptr;
    if (sp.n > 0) {
        MLCC_TRY(c->sheet_d.reserve(sizeof sp.dmap));
        MLCC_HIP(hipMemcpyAsync(c->sheet_d.p, sp.dmap, sizeof sp.dmap, hipMemcpyHostToDevice,
                                c->stream));
        pmap = c->sheet_d.as<double>();
    }
    if (c->equal_mass)
        hipLaunchKernelGGL(map_caustics_f64<true>, dim3((unsigned)blocks), dim3(64), 0, c->stream,
                           c->stars.as<double2>(), c->mass0, (int32_t)c->n, count, zr, zi, wr, wi,
                           a, gamma, pmap, sp.n);
    else
        hipLaunchKernelGGL(map_caustics_f64<false>, dim3((unsigned)blocks), dim3(64), 0,
                           c->stream, c->stars4.as<double4>(), c->mass0, (int32_t)c->n, count,
                           zr, zi, wr, wi, a, gamma, pmap, sp.n);
    MLCC_HIP(hipGetLastError());
    return MLCC_OK;
}

} // namespace mlcc
