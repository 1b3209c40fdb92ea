// Throughput probes of the gfx950 units that bound the path: single- and
// double-precision FMA, the single-precision transcendentals the Voigt
// evaluation issues (v_exp_f32, v_log_f32, v_rcp_f32), a mix of them with
// FMAs in the proportion of a wing term, and a device-memory copy.  They give
// the measured denominators of the roofline beside the nominal peaks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/lrt.h"
#include "lrt_device.h"

namespace lrt {

namespace {

constexpr int kChains = 8;          // independent dependency chains per lane
constexpr int kProbeThreads = 256;

// One lane-op per chain per iteration; every result is kept live through the
// final sum so nothing is dead code.
template <int KIND>
__global__ __launch_bounds__(kProbeThreads) void probe_valu_kernel(float a, float b, int32_t iters, float *out)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = a + (float)(threadIdx.x + c) * 1e-3f;
#pragma unroll 4
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (KIND == LRT_PROBE_FMA_F32) x[c] = fmaf(x[c], a, b);
            if constexpr (KIND == LRT_PROBE_EXP_F32) x[c] = __builtin_amdgcn_exp2f(-fabsf(x[c]));
            if constexpr (KIND == LRT_PROBE_LOG_F32) x[c] = __builtin_amdgcn_logf(fabsf(x[c]));
            if constexpr (KIND == LRT_PROBE_RCP_F32) x[c] = __builtin_amdgcn_rcpf(x[c]);
            if constexpr (KIND == LRT_PROBE_MIX_F32) {
                // 3 transcendentals and 10 other VALU operations, the shape of
                // one wing term of the accumulation: 13 lane-ops
                const float y = fmaf(x[c], a, -b);
                const float d1 = fmaf(y, y, 1.0f);
                const float p = __builtin_amdgcn_exp2f(2.25f * __builtin_amdgcn_logf(fabsf(y)));
                const float d2 = fmaf(p, 0.021f, 1.0f);
                const float num = fmaf(a, d2, -(b * d1));
                const float P = num * __builtin_amdgcn_rcpf(d1 * d2);
                x[c] = fmaf(P, a, fmaf(P, b, x[c]));
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 12345.678f) out[0] = s;   // never true for these inputs; keeps the chains live
}

__global__ __launch_bounds__(kProbeThreads) void probe_fma64_kernel(double a, double b, int32_t iters, double *out)
{
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = a + (double)(threadIdx.x + c) * 1e-3;
#pragma unroll 4
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (s == 12345.678) out[0] = s;
}

__global__ __launch_bounds__(kProbeThreads) void probe_copy_kernel(const float4 *__restrict__ src,
                                                                   float4 *__restrict__ dst, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace
}  // namespace lrt

using namespace lrt;

extern "C" lrt_status lrt_probe(int device, int kind, double *rate, double *ms)
{
    if (!rate || kind < LRT_PROBE_FMA_F32 || kind > LRT_PROBE_COPY) return LRT_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return LRT_E_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return LRT_E_DEVICE;
    // 8 waves per SIMD on every CU: 32 waves of 64 lanes per CU
    const int blocks = prop.multiProcessorCount * 8;
    const int32_t iters = 16384;
    void *buf = nullptr, *src = nullptr;
    const int64_t copy_bytes = (int64_t)4 << 30;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lrt_status st = LRT_OK;
    float t = 0.0f;
    auto launch = [&]() -> hipError_t {
        switch (kind) {
        case LRT_PROBE_FMA_F32:
            hipLaunchKernelGGL(probe_valu_kernel<LRT_PROBE_FMA_F32>, dim3(blocks), dim3(kProbeThreads), 0, nullptr,
                               0.999f, 1e-3f, iters, (float *)buf);
            break;
        case LRT_PROBE_EXP_F32:
            hipLaunchKernelGGL(probe_valu_kernel<LRT_PROBE_EXP_F32>, dim3(blocks), dim3(kProbeThreads), 0, nullptr,
                               0.999f, 1e-3f, iters, (float *)buf);
            break;
        case LRT_PROBE_LOG_F32:
            hipLaunchKernelGGL(probe_valu_kernel<LRT_PROBE_LOG_F32>, dim3(blocks), dim3(kProbeThreads), 0, nullptr,
                               3.0f, 1e-3f, iters, (float *)buf);
            break;
        case LRT_PROBE_RCP_F32:
            hipLaunchKernelGGL(probe_valu_kernel<LRT_PROBE_RCP_F32>, dim3(blocks), dim3(kProbeThreads), 0, nullptr,
                               1.5f, 1e-3f, iters, (float *)buf);
            break;
        case LRT_PROBE_MIX_F32:
            hipLaunchKernelGGL(probe_valu_kernel<LRT_PROBE_MIX_F32>, dim3(blocks), dim3(kProbeThreads), 0, nullptr,
                               0.37f, 0.011f, iters / 8, (float *)buf);
            break;
        case LRT_PROBE_FMA_F64:
            hipLaunchKernelGGL(probe_fma64_kernel, dim3(blocks), dim3(kProbeThreads), 0, nullptr, 0.999, 1e-3, iters,
                               (double *)buf);
            break;
        default:
            hipLaunchKernelGGL(probe_copy_kernel, dim3(blocks * 16), dim3(kProbeThreads), 0, nullptr,
                               (const float4 *)src, (float4 *)buf, copy_bytes / 16);
            break;
        }
        return hipGetLastError();
    };
    const size_t bytes = kind == LRT_PROBE_COPY ? (size_t)copy_bytes : 64;
    if (hipMalloc(&buf, bytes) != hipSuccess) return LRT_E_OOM;
    if (kind == LRT_PROBE_COPY && (hipMalloc(&src, bytes) != hipSuccess || hipMemset(src, 0, bytes) != hipSuccess)) {
        st = LRT_E_OOM;
        goto done;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess || launch() != hipSuccess ||
        hipEventRecord(e0, nullptr) != hipSuccess || launch() != hipSuccess || hipEventRecord(e1, nullptr) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        st = LRT_E_DEVICE;
        goto done;
    }
    {
        const double sec = (double)t * 1e-3;
        const double lanes = (double)blocks * kProbeThreads;
        double ops;
        if (kind == LRT_PROBE_COPY) ops = 2.0 * (double)copy_bytes;   // bytes read + written
        else if (kind == LRT_PROBE_MIX_F32) ops = lanes * (iters / 8) * kChains * 13.0;
        else ops = lanes * iters * kChains;
        *rate = ops / sec;
        if (ms) *ms = t;
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (buf) (void)hipFree(buf);
    if (src) (void)hipFree(src);
    return st;
}
