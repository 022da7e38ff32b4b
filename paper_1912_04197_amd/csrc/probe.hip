// Achievable vector FMA rate of the device, the measured ceiling beside the
// datasheet one for the rooflines of the walk and the direct sum (both are
// bound by plain VALU arithmetic). Every lane runs kChains independent fused
// multiply-add chains, so issue, not latency, limits the rate.
#include <cmath>

#include "bhx_impl.h"

namespace {

constexpr int kChains = 8;
constexpr int kProbeThreads = 256;
constexpr int kWavesPerSimd = 8;

template <typename T>
__global__ __launch_bounds__(kProbeThreads) void k_fma_probe(int64_t iters, T mul, T add,
                                                             T *__restrict__ sink)
{
    T a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; c++) a[c] = T(threadIdx.x + c) * T(1e-3);
#pragma unroll 4
    for (int64_t i = 0; i < iters; i++) {
#pragma unroll
        for (int c = 0; c < kChains; c++) a[c] = std::fma(a[c], mul, add);
    }
    T s = T(0);
#pragma unroll
    for (int c = 0; c < kChains; c++) s += a[c];
    sink[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

template <typename T>
hipError_t probe(hipStream_t s, int64_t iters, double *tflops)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // 4 SIMDs per compute unit, kWavesPerSimd wavefronts of 64 lanes on each
    const int blocks = cus * 4 * kWavesPerSimd * 64 / kProbeThreads;
    T *sink = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipMalloc(&sink, (size_t)blocks * kProbeThreads * sizeof(T));
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) {
        const T mul = T(0.999999), add = T(1e-7);
        k_fma_probe<T><<<blocks, kProbeThreads, 0, s>>>(iters / 8 + 1, mul, add, sink);  // warm-up
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(ev[0], s);
        if (e == hipSuccess) {
            k_fma_probe<T><<<blocks, kProbeThreads, 0, s>>>(iters, mul, add, sink);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e == hipSuccess) {
            const double fmas = (double)blocks * kProbeThreads * kChains * (double)iters;
            *tflops = ms > 0.f ? 2.0 * fmas / (ms * 1e-3) / 1e12 : 0.0;
        }
    }
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    if (sink) {
        const hipError_t f = hipStreamSynchronize(s);
        (void)hipFree(sink);
        if (e == hipSuccess) e = f;
    }
    return e;
}

}  // namespace

extern "C" bh_status bh_probe_fma(void *hip_stream, int32_t precision, int64_t iters,
                                  double *tflops)
{
    if (!tflops || iters < 1 || iters > (int64_t)1 << 24) return BH_E_INVALID;  // <= about 2 s
    if (precision != BH_FP64 && precision != BH_FP32C) return BH_E_INVALID;
    *tflops = 0.0;
    const hipStream_t s = (hipStream_t)hip_stream;
    const hipError_t e = precision == BH_FP64 ? probe<double>(s, iters, tflops)
                                              : probe<float>(s, iters, tflops);
    if (e == hipErrorOutOfMemory) return BH_E_OOM;
    return e == hipSuccess ? BH_OK : BH_E_HIP;
}
