// Measurement helper: the VALU issue rate the device reaches on long runs of independent
// vector instructions, the ceiling against which the search kernels' instruction rates
// are reported (their packed-FP16 tests, FP32 arithmetic and integer bit work).
//
// Each lane runs kChains independent dependency chains of one instruction kind, unrolled,
// so the issue logic never waits for a result; enough wavefronts are launched to give every
// SIMD several of them. The kernel's VALU instruction count is known from its source (one
// instruction per operation, checked against SQ_INSTS_VALU in the committed profile).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nnps.h"

namespace nnps {

typedef _Float16 ph2 __attribute__((ext_vector_type(2)));

constexpr int kChains = 16;
constexpr int kProbeThreads = 256;

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads)
k_probe_valu(int iters, uint32_t seed, uint32_t* __restrict__ sink)
{
    const uint32_t t = threadIdx.x + blockIdx.x * blockDim.x + seed;
    if constexpr (KIND == 0) {  // packed FP16 fma: one v_pk_fma_f16 per operation
        ph2 acc[kChains];
        const ph2 m = ph2{static_cast<_Float16>(0.999f), static_cast<_Float16>(0.998f)};
        const ph2 c = ph2{static_cast<_Float16>(1e-3f), static_cast<_Float16>(2e-3f)};
#pragma unroll
        for (int k = 0; k < kChains; ++k)
            acc[k] = ph2{static_cast<_Float16>(static_cast<float>((t + k) & 7)), static_cast<_Float16>(0.5f)};
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) acc[k] = __builtin_elementwise_fma(acc[k], m, c);
        }
        ph2 s = acc[0];
#pragma unroll
        for (int k = 1; k < kChains; ++k) s += acc[k];
        if (s.x == static_cast<_Float16>(-1.0f)) sink[0] = t;  // never true; keeps the chains alive
    } else if constexpr (KIND == 1) {  // FP32 fma: one v_fma_f32 per operation
        float acc[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = static_cast<float>((t + k) & 7);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) acc[k] = __builtin_fmaf(acc[k], 0.999f, 1e-3f);
        }
        float s = acc[0];
#pragma unroll
        for (int k = 1; k < kChains; ++k) s += acc[k];
        if (s == -1.0f) sink[0] = t;
    } else {  // 32-bit integer: one v_xad (xor-add) style op per operation
        uint32_t acc[kChains];
#pragma unroll
        for (int k = 0; k < kChains; ++k) acc[k] = t * (2u * k + 1u);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) acc[k] = (acc[k] ^ 0x9E3779B9u) + static_cast<uint32_t>(k);
        }
        uint32_t s = acc[0];
#pragma unroll
        for (int k = 1; k < kChains; ++k) s ^= acc[k];
        if (s == 0xFFFFFFFFu) sink[0] = t;
    }
}

}  // namespace nnps

extern "C" nnps_status nnps_probe_valu_rate(int32_t device, int32_t kind, double* rate, int64_t* insts_per_wave)
{
    using namespace nnps;
    if (!rate || kind < 0 || kind > 2) return NNPS_EINVAL;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return NNPS_EDEVICE;
    nnps_status st = NNPS_OK;
    hipDeviceProp_t prop;
    uint32_t* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int iters = 4096;
    do {
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) { st = NNPS_EDEVICE; break; }
        if (hipMalloc(&sink, 64) != hipSuccess) { st = NNPS_ENOMEM; break; }
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { st = NNPS_EDEVICE; break; }
        // 8 wavefronts per SIMD (4 SIMDs per CU), four times over
        const int grid = prop.multiProcessorCount * 4 * 8 * 4 / (kProbeThreads / 64);
        auto launch = [&]() {
            if (kind == 0) hipLaunchKernelGGL(k_probe_valu<0>, dim3(grid), dim3(kProbeThreads), 0, nullptr, iters, 1u, sink);
            else if (kind == 1) hipLaunchKernelGGL(k_probe_valu<1>, dim3(grid), dim3(kProbeThreads), 0, nullptr, iters, 1u, sink);
            else hipLaunchKernelGGL(k_probe_valu<2>, dim3(grid), dim3(kProbeThreads), 0, nullptr, iters, 1u, sink);
        };
        launch();  // warm-up
        if (hipEventRecord(e0, nullptr) != hipSuccess) { st = NNPS_EDEVICE; break; }
        launch();
        if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipGetLastError() != hipSuccess) {
            st = NNPS_EDEVICE;
            break;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f) { st = NNPS_EDEVICE; break; }
        // the timed loop's VALU instructions per wavefront (the set-up and reduction around
        // it are a few dozen more, below 0.1 % of these)
        const int64_t per_wave = static_cast<int64_t>(iters) * kChains;
        const double waves = static_cast<double>(grid) * (kProbeThreads / 64);
        *rate = waves * static_cast<double>(per_wave) / (ms * 1e-3);
        if (insts_per_wave) *insts_per_wave = per_wave;
    } while (false);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (sink) (void)hipFree(sink);
    if (prev >= 0) (void)hipSetDevice(prev);
    return st;
}
