// Measurement probe: the attainable (non-packed) vector FMA rate in FP64 and FP32,
// a measured ceiling for the apply kernels beside the published peak.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace pa {
namespace {

constexpr int kProbeChains = 8;   // independent FMA chains per lane

// Every lane runs kProbeChains dependent chains of iters FMAs each and writes the
// sum of its chains to out[global lane] (so the work is not optimised away).
template <typename T>
__global__ void __launch_bounds__(256) fma_probe_kernel(T* __restrict__ out, const int iters, const T a, const T b) {
    const int gid = blockIdx.x * 256 + threadIdx.x;
    T v[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) v[k] = T(gid % 1024 + k) * T(1e-3);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) v[k] = fma(v[k], a, b);
    }
    T s = T(0);
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += v[k];
    out[gid] = s;
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" int pa_probe_fma(void* out, int dtype, int blocks, int iters, void* hip_stream) {
    if (!out) return fail(PA_EINVAL, "out is NULL");
    if (dtype != PA_F64 && dtype != PA_F32) return fail(PA_EINVAL, "dtype %d is not PA_F64/PA_F32", dtype);
    if (blocks < 1 || iters < 1) return fail(PA_EINVAL, "blocks and iters must be >= 1");
    const hipStream_t s = (hipStream_t)hip_stream;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(fma_probe_kernel<double>, dim3(blocks), dim3(256), 0, s, (double*)out, iters,
                           0.999999999, 1e-9);
    else
        hipLaunchKernelGGL(fma_probe_kernel<float>, dim3(blocks), dim3(256), 0, s, (float*)out, iters, 0.9999f,
                           1e-4f);
    PA_HIP(hipGetLastError());
    return PA_OK;
}
