// Streaming vector kernels (HBM-bound): fills, Dirichlet fix-ups, apply preparation.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace pa {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    return (int)(b < 1 ? 1 : b);
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ y, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = v;
}

__device__ __forceinline__ void node_pos(int node, const Geom& g, int& gx, int& gy, int& gz) {
    gx = node % g.Nx;
    const int r = node / g.Nx;
    gy = r % g.Ny;
    gz = r / g.Ny;
}

template <typename T>
__global__ void set_clamped_kernel(T* __restrict__ y, Geom g, T v) {
    for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < g.Nn; node += gridDim.x * blockDim.x) {
        int gx, gy, gz;
        node_pos(node, g, gx, gy, gz);
        if (clamped_node(g.clamp, gx, gy, gz, g)) {
            y[node] = v;
            y[(size_t)g.Nn + node] = v;
            y[2 * (size_t)g.Nn + node] = v;
        }
    }
}

template <typename T>
__global__ void apply_prep_kernel(const T* __restrict__ x, T* __restrict__ y, Geom g, int add) {
    for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < g.Nn; node += gridDim.x * blockDim.x) {
        int gx, gy, gz;
        node_pos(node, g, gx, gy, gz);
        const bool cl = clamped_node(g.clamp, gx, gy, gz, g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t i = (size_t)c * g.Nn + node;
            if (cl)
                y[i] = add ? y[i] + x[i] : x[i];
            else if (!add)
                y[i] = T(0);
        }
    }
}

}  // namespace

int launch_fill(void* y, int dtype, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return PA_OK;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, (double*)y, n, v);
    else
        hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, (float*)y, n, (float)v);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

int launch_set_clamped(void* y, int dtype, const Geom& g, double v, hipStream_t s) {
    if (!g.clamp) return PA_OK;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(set_clamped_kernel<double>, dim3(grid_for(g.Nn)), dim3(kBlock), 0, s, (double*)y, g, v);
    else
        hipLaunchKernelGGL(set_clamped_kernel<float>, dim3(grid_for(g.Nn)), dim3(kBlock), 0, s, (float*)y, g,
                           (float)v);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

int launch_apply_prep(const void* x, void* y, int dtype, const Geom& g, int add, hipStream_t s) {
    if (add && !g.clamp) return PA_OK;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(apply_prep_kernel<double>, dim3(grid_for(g.Nn)), dim3(kBlock), 0, s, (const double*)x,
                           (double*)y, g, add);
    else
        hipLaunchKernelGGL(apply_prep_kernel<float>, dim3(grid_for(g.Nn)), dim3(kBlock), 0, s, (const float*)x,
                           (float*)y, g, add);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

}  // namespace pa
