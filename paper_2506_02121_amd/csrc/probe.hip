// Measured vector-ALU rate of the device: a measurement aid for the
// benchmark's rooflines, not part of the method and not on the library's
// C-ABI.  Built into its own library (libvalu_probe.so) with the same
// compiler flags as libmlcc.so.  Eight independent FMA chains per lane,
// enough waves to fill every SIMD, timed with HIP events.
//
//   int valu_probe_fma_tflops(int device, int kind, double *tflops)
//     kind 0 = FP64 v_fma_f64, 1 = FP32 v_fma_f32 (unpacked); writes the rate
//     in TFLOP/s (FMA = 2 FLOP).  Returns 0, -1 for a bad argument, or the
//     hipError_t of the first HIP call that failed.  Runs ~0.1 s of kernels on
//     a stream of its own (allocates and frees 2 MB); synchronous.
#include <hip/hip_runtime.h>

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
int run_probe(int device, double *tflops)
{
    hipError_t first = hipSuccess;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && first == hipSuccess) first = e;
        return e == hipSuccess;
    };
    int cus = 0;
    if (!chk(hipSetDevice(device)) ||
        !chk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)))
        return (int)first;
    if (cus < 1) return -1;
    const int blocks = cus * 8;   // 8 waves of 64 per SIMD
    const int iters = 1 << 16;
    T *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
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
    if (first != hipSuccess) return (int)first;
    if (!(ms > 0.f)) return -1;
    const double flop = 4.0 * 2.0 * PROBE_CHAINS * (double)iters * blocks * PROBE_THREADS;
    *tflops = flop / (ms * 1e-3) / 1e12;
    return 0;
}

}  // namespace

extern "C" int valu_probe_fma_tflops(int device, int kind, double *tflops)
{
    if (!tflops) return -1;
    if (kind == 0) return run_probe<double>(device, tflops);
    if (kind == 1) return run_probe<float>(device, tflops);
    return -1;
}
