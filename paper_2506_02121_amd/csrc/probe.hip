// Measured vector-ALU rate of the device, the reference beside the published
// peaks in the roofline of the root-finder kernels: eight independent FMA
// chains per lane, enough waves to fill every SIMD, timed with HIP events.
#include <cmath>

#include "mlcc_internal.h"

namespace mlcc {

namespace {

constexpr int PROBE_CHAINS = 8;
constexpr int PROBE_THREADS = 256;

template <class T>
__global__ void __launch_bounds__(PROBE_THREADS) fma_chains(T *__restrict__ out, int iters, T a, T b)
{
    T x[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = (T)(threadIdx.x & 15) * (T)0.001 + (T)c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) x[c] = fma(x[c], a, b);
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += x[c];
    out[blockIdx.x * PROBE_THREADS + threadIdx.x] = s;
}

template <class T>
mlcc_status run_probe(int device, double *tflops)
{
    MLCC_HIP(hipSetDevice(device));
    int cus = 0;
    MLCC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    if (cus < 1) return fail(MLCC_ERR_HIP, "device reports no compute units");
    const int blocks = cus * 8;   // 8 waves of 64 per SIMD
    const int iters = 1 << 16;
    T *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mlcc_status st = MLCC_OK;
    float ms = 0.f;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && st == MLCC_OK)
            st = fail(MLCC_ERR_HIP, "probe: %s", hipGetErrorString(e));
        return e == hipSuccess;
    };
    if (chk(hipMalloc(&out, (size_t)blocks * PROBE_THREADS * sizeof(T))) &&
        chk(hipStreamCreate(&s)) && chk(hipEventCreate(&e0)) && chk(hipEventCreate(&e1))) {
        // one untimed launch (clocks, code load), then four timed ones
        hipLaunchKernelGGL(fma_chains<T>, dim3(blocks), dim3(PROBE_THREADS), 0, s, out, iters / 4,
                           (T)0.999999, (T)1e-6);
        chk(hipGetLastError());
        chk(hipEventRecord(e0, s));
        for (int r = 0; r < 4; ++r)
            hipLaunchKernelGGL(fma_chains<T>, dim3(blocks), dim3(PROBE_THREADS), 0, s, out, iters,
                               (T)0.999999, (T)1e-6);
        chk(hipGetLastError());
        chk(hipEventRecord(e1, s));
        if (chk(hipEventSynchronize(e1))) chk(hipEventElapsedTime(&ms, e0, e1));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    if (out) (void)hipFree(out);
    if (st != MLCC_OK) return st;
    if (!(ms > 0.f)) return fail(MLCC_ERR_HIP, "probe: no elapsed time");
    const double flop = 4.0 * 2.0 * PROBE_CHAINS * (double)iters * blocks * PROBE_THREADS;
    *tflops = flop / (ms * 1e-3) / 1e12;
    return MLCC_OK;
}

}  // namespace

}  // namespace mlcc

using namespace mlcc;

extern "C" mlcc_status mlcc_measure_valu_peak(int device, int kind, double *tflops)
{
    clear_error();
    if (!tflops) return fail(MLCC_ERR_INVALID, "tflops is NULL");
    if (kind == 0) return run_probe<double>(device, tflops);
    if (kind == 1) return run_probe<float>(device, tflops);
    return fail(MLCC_ERR_INVALID, "unknown kind %d (0 = FP64 FMA, 1 = FP32 FMA)", kind);
}
