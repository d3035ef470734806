// Unfused forms of the elasticity apply, for the cumulative ablation of the
// paper's optimization stages (Sec. 4.1-4.4 and its ablation table) measured on
// this GPU.  Every variant computes the same y = A x (FP64) in three passes with
// operator-wide arrays in HBM between them, as the baseline PA dataflow does
// (Alg. 1):
//   gradient pass: reference displacement gradients at every quadrature point
//                  -> QVec_grad [NE][Q^3][3][3];
//   stress pass:   physical gradient J^{-T} g, strain, stress with the weighted
//                  w*detJ*lambda, w*detJ*mu, Q = sigma J^{-T} (eq. 7) -> QVec_sigma;
//   action pass:   contraction of QVec_sigma with the test-function gradients
//                  -> element vectors, then a fixed-order assembly into y.
// The gradient and action passes are either dense (every basis function at
// every quadrature point, O(D^3 Q^3) per element, with the basis-gradient table
// streamed from memory) or sum-factorized (X/Y/Z sweeps through LDS, one
// workgroup per few elements); the stress pass uses full 3x3 tensors or the Voigt
// form.
// The fused variant (the fusion stage, Sec. 4.2, Alg. 2) runs the same three
// sum-factorized/Voigt passes inside one kernel, element by element: each
// workgroup stages its elements' quadrature-point data (the per-element el_QVec of
// the paper, 9 words per point) in a buffer of its own, rewrites it in place with
// the stress, and contracts it back, then the same fixed-order assembly.  What it
// lacks against the production apply is the slice-wise organisation (Sec. 4.5):
// gradients held in registers per quadrature column instead of a staged array, x
// read and y written straight from and to the L-vectors.
#include <hip/hip_runtime.h>

#include <vector>

#include "apply_kernel.h"
#include "internal.h"
#include "kernels.h"

namespace pa {

struct AblationBuffers {
    double* qg = nullptr;     // [NE][Q^3][3 comp][3 ref dir]
    double* qs = nullptr;     // [NE][Q^3][3 comp][3 ref dir]
    double* ev = nullptr;     // [NE][3][D^3]
    double* dphi = nullptr;   // [D^3][Q^3][3]: d phi_a / d xi_m at point alpha
    double* tab = nullptr;    // B[D][Q] | G[D][Q] | w[Q]
};

void free_ablation(AblationBuffers* b) {
    if (!b) return;
    for (double* p : {b->qg, b->qs, b->ev, b->dphi, b->tab})
        if (p) (void)hipFree(p);
    delete b;
}

namespace {

constexpr int kAbT = 256;   // threads of the per-element (sum-factorized) kernels

// ---------------------------------------------------------------- dense passes
template <int P, int Q>
__global__ void __launch_bounds__(256)
grad_dense_kernel(const double* __restrict__ x, const double* __restrict__ dphi, double* __restrict__ qg,
                  const Geom g) {
    constexpr int D = P + 1, D3 = D * D * D, Q3 = Q * Q * Q;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.NE * Q3) return;
    const int e = (int)(t / Q3), al = (int)(t % Q3);
    const int ex = e % g.nx, r = e / g.nx, ey = r % g.ny, ez = r / g.ny;
    const size_t NN = (size_t)g.Nn;
    double gr[3][3] = {};
    for (int a = 0; a < D3; ++a) {
        const int ix = a % D, iy = (a / D) % D, iz = a / (D * D);
        const int gx = ex * P + ix, gy = ey * P + iy, gz = ez * P + iz;
        if (g.clamp && clamped_node(g.clamp, gx, gy, gz, g)) continue;   // read as 0
        const int node = gx + g.Nx * (gy + g.Ny * gz);
        const double* dp = dphi + ((size_t)a * Q3 + al) * 3;
        const double d0 = dp[0], d1 = dp[1], d2 = dp[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double xv = x[c * NN + node];
            gr[c][0] += xv * d0;
            gr[c][1] += xv * d1;
            gr[c][2] += xv * d2;
        }
    }
    double* o = qg + t * 9;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 3; ++m) o[c * 3 + m] = gr[c][m];
}

template <int P, int Q>
__global__ void __launch_bounds__(256)
action_dense_kernel(const double* __restrict__ qs, const double* __restrict__ dphi, double* __restrict__ ev,
                    const Geom g) {
    constexpr int D = P + 1, D3 = D * D * D, Q3 = Q * Q * Q;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)g.NE * D3) return;
    const int e = (int)(t / D3), a = (int)(t % D3);
    double s[3] = {0.0, 0.0, 0.0};
    const double* q = qs + (size_t)e * Q3 * 9;
    const double* dp = dphi + (size_t)a * Q3 * 3;
    for (int al = 0; al < Q3; ++al) {
        const double d0 = dp[al * 3], d1 = dp[al * 3 + 1], d2 = dp[al * 3 + 2];
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += q[al * 9 + c * 3] * d0 + q[al * 9 + c * 3 + 1] * d1 + q[al * 9 + c * 3 + 2] * d2;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) ev[((size_t)e * 3 + c) * D3 + a] = s[c];
}

// ---------------------------------------------------------------- stress pass
// One quadrature point: in[c*3+m] = d u_c / d xi_m -> out[c*3+m] = Q_{c,m} = sum_i sigma_{c,i}
// (J^{-1})_{m,i}, sigma from the weighted w*detJ*lambda, w*detJ*mu (eq. 7); in may equal out.
template <bool VOIGT>
__device__ __forceinline__ void point_stress(const double* __restrict__ d, double W, const double* in, double* out) {
    double Ji[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Ji[k] = d[k];
    const double lam = W * d[9], mu = W * d[10];
    double du[3][3];   // du[c][i] = d u_c / d x_i
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            du[c][i] = Ji[0 * 3 + i] * in[c * 3] + Ji[1 * 3 + i] * in[c * 3 + 1] + Ji[2 * 3 + i] * in[c * 3 + 2];
    double s[3][3];
    if (VOIGT) {
        // six independent stress components
        const double div = du[0][0] + du[1][1] + du[2][2];
        const double ld = lam * div, m2 = mu + mu;
        s[0][0] = ld + m2 * du[0][0];
        s[1][1] = ld + m2 * du[1][1];
        s[2][2] = ld + m2 * du[2][2];
        s[0][1] = s[1][0] = mu * (du[0][1] + du[1][0]);
        s[0][2] = s[2][0] = mu * (du[0][2] + du[2][0]);
        s[1][2] = s[2][1] = mu * (du[1][2] + du[2][1]);
    } else {
        // full tensors: eps = (grad u + grad u^T) / 2, sigma = lambda tr(eps) I + 2 mu eps
        double eps[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) eps[i][j] = 0.5 * (du[i][j] + du[j][i]);
        const double tr = eps[0][0] + eps[1][1] + eps[2][2];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) s[i][j] = (i == j ? lam * tr : 0.0) + 2.0 * mu * eps[i][j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 3; ++m) out[c * 3 + m] = s[c][0] * Ji[m * 3 + 0] + s[c][1] * Ji[m * 3 + 1] + s[c][2] * Ji[m * 3 + 2];
}

template <int Q, bool VOIGT>
__global__ void __launch_bounds__(256)
stress_kernel(const double* __restrict__ ed, const double* __restrict__ tab, const double* __restrict__ qg,
              double* __restrict__ qs, const int64_t npts, const int DQ) {
    constexpr int Q3 = Q * Q * Q;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    const int64_t e = t / Q3;
    const int al = (int)(t % Q3);
    const double* w = tab + 2 * DQ;
    const double W = w[al % Q] * w[(al / Q) % Q] * w[al / (Q * Q)];
    double in[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) in[k] = qg[t * 9 + k];
    point_stress<VOIGT>(ed + e * kEdStride, W, in, qs + t * 9);
}

// ---------------------------------------------------------------- sum-factorized passes
// Several elements per workgroup (enough to occupy its threads in every sweep);
// per component: X sweep on lines (iz, iy) read from the L-vector, Y sweep on
// lines (iz, qx), Z sweep on columns (qy, qx).
template <int P, int Q>
struct AbCfg {
    static constexpr int D = P + 1;
    static constexpr int WORK = (D * D > D * Q ? (D * D > Q * Q ? D * D : Q * Q) : (D * Q > Q * Q ? D * Q : Q * Q));
    static constexpr int E = kAbT / WORK > 0 ? kAbT / WORK : 1;
};

// Gradient pass of the elements e0 .. e0+E-1: for each component, X sweep from the
// L-vector into U, Y sweep into S, Z sweep into qg[e][alpha][c*3+m] (the element's slice
// of an array with 9 words per point).  U and S are the workgroup's LDS tiles.
template <int P, int Q, int E>
__device__ void grad_sf(const double* __restrict__ x, const double* __restrict__ tab, double* __restrict__ qg,
                        const Geom& g, int e0, double (*U)[2][P + 1][P + 1][Q], double (*S)[3][P + 1][Q][Q]) {
    constexpr int D = P + 1, Q3 = Q * Q * Q;
    const double* B = tab;
    const double* G = tab + D * Q;
    const int tid = threadIdx.x;
    const size_t NN = (size_t)g.Nn;
    for (int c = 0; c < 3; ++c) {
        for (int w = tid; w < E * D * D; w += kAbT) {
            const int el = w / (D * D), l = w % (D * D), e = e0 + el;
            if (e >= g.NE) continue;
            const int ex = e % g.nx, r = e / g.nx, ey = r % g.ny, ez = r / g.ny;
            const int iz = l / D, iy = l % D;
            double xv[D];
#pragma unroll
            for (int ix = 0; ix < D; ++ix) {
                const int gx = ex * P + ix, gy = ey * P + iy, gz = ez * P + iz;
                xv[ix] = (g.clamp && clamped_node(g.clamp, gx, gy, gz, g))
                             ? 0.0 : x[c * NN + gx + g.Nx * (gy + g.Ny * gz)];
            }
            for (int k = 0; k < Q; ++k) {
                double u = 0.0, v = 0.0;
#pragma unroll
                for (int ix = 0; ix < D; ++ix) {
                    u += xv[ix] * B[ix * Q + k];
                    v += xv[ix] * G[ix * Q + k];
                }
                U[el][0][iz][iy][k] = u;
                U[el][1][iz][iy][k] = v;
            }
        }
        __syncthreads();
        for (int w = tid; w < E * D * Q; w += kAbT) {
            const int el = w / (D * Q), iz = (w % (D * Q)) / Q, qx = w % Q;
            for (int k = 0; k < Q; ++k) {
                double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int iy = 0; iy < D; ++iy) {
                    s0 += U[el][1][iz][iy][qx] * B[iy * Q + k];
                    s1 += U[el][0][iz][iy][qx] * G[iy * Q + k];
                    s2 += U[el][0][iz][iy][qx] * B[iy * Q + k];
                }
                S[el][0][iz][k][qx] = s0;
                S[el][1][iz][k][qx] = s1;
                S[el][2][iz][k][qx] = s2;
            }
        }
        __syncthreads();
        for (int w = tid; w < E * Q * Q; w += kAbT) {
            const int el = w / (Q * Q), qy = (w % (Q * Q)) / Q, qx = w % Q, e = e0 + el;
            if (e >= g.NE) continue;
            for (int k = 0; k < Q; ++k) {
                double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
                for (int iz = 0; iz < D; ++iz) {
                    g0 += S[el][0][iz][qy][qx] * B[iz * Q + k];
                    g1 += S[el][1][iz][qy][qx] * B[iz * Q + k];
                    g2 += S[el][2][iz][qy][qx] * G[iz * Q + k];
                }
                double* o = qg + ((size_t)e * Q3 + qx + Q * (qy + Q * k)) * 9 + c * 3;
                o[0] = g0;
                o[1] = g1;
                o[2] = g2;
            }
        }
        __syncthreads();
    }
}

// Action pass of the elements e0 .. e0+E-1: for each component, backward Z from
// qs[e][alpha][c*3+m] into T, backward Y into R, backward X into the element vectors ev.
template <int P, int Q, int E>
__device__ void action_sf(const double* __restrict__ qs, const double* __restrict__ tab, double* __restrict__ ev,
                          const Geom& g, int e0, double (*T)[3][P + 1][Q][Q], double (*R)[2][P + 1][P + 1][Q]) {
    constexpr int D = P + 1, D3 = D * D * D, Q3 = Q * Q * Q;
    const double* B = tab;
    const double* G = tab + D * Q;
    const int tid = threadIdx.x;
    for (int c = 0; c < 3; ++c) {
        for (int w = tid; w < E * Q * Q; w += kAbT) {
            const int el = w / (Q * Q), qy = (w % (Q * Q)) / Q, qx = w % Q, e = e0 + el;
            if (e >= g.NE) continue;
            const double* q = qs + (size_t)e * Q3 * 9;
            for (int iz = 0; iz < D; ++iz) {
                double t0 = 0.0, t1 = 0.0, t2 = 0.0;
                for (int k = 0; k < Q; ++k) {
                    const double* qq = q + (size_t)(qx + Q * (qy + Q * k)) * 9 + c * 3;
                    t0 += qq[0] * B[iz * Q + k];
                    t1 += qq[1] * B[iz * Q + k];
                    t2 += qq[2] * G[iz * Q + k];
                }
                T[el][0][iz][qy][qx] = t0;
                T[el][1][iz][qy][qx] = t1;
                T[el][2][iz][qy][qx] = t2;
            }
        }
        __syncthreads();
        for (int w = tid; w < E * D * Q; w += kAbT) {
            const int el = w / (D * Q), iz = (w % (D * Q)) / Q, qx = w % Q;
            for (int iy = 0; iy < D; ++iy) {
                double r0 = 0.0, r12 = 0.0;
                for (int k = 0; k < Q; ++k) {
                    r0 += T[el][0][iz][k][qx] * B[iy * Q + k];
                    r12 += T[el][1][iz][k][qx] * G[iy * Q + k] + T[el][2][iz][k][qx] * B[iy * Q + k];
                }
                R[el][0][iz][iy][qx] = r0;
                R[el][1][iz][iy][qx] = r12;
            }
        }
        __syncthreads();
        for (int w = tid; w < E * D * D; w += kAbT) {
            const int el = w / (D * D), l = w % (D * D), e = e0 + el;
            if (e >= g.NE) continue;
            const int iz = l / D, iy = l % D;
            for (int ix = 0; ix < D; ++ix) {
                double y = 0.0;
                for (int k = 0; k < Q; ++k)
                    y += R[el][0][iz][iy][k] * G[ix * Q + k] + R[el][1][iz][iy][k] * B[ix * Q + k];
                ev[((size_t)e * 3 + c) * D3 + ix + D * (iy + D * iz)] = y;
            }
        }
        __syncthreads();
    }
}

template <int P, int Q>
__global__ void __launch_bounds__(kAbT)
grad_sf_kernel(const double* __restrict__ x, const double* __restrict__ tab, double* __restrict__ qg, const Geom g) {
    constexpr int D = P + 1, E = AbCfg<P, Q>::E;
    __shared__ double U[E][2][D][D][Q];    // x-contracted: B (value), G (derivative)
    __shared__ double S[E][3][D][Q][Q];    // y-contracted: (G_x B_y), (B_x G_y), (B_x B_y)
    grad_sf<P, Q, E>(x, tab, qg, g, blockIdx.x * E, U, S);
}

template <int P, int Q>
__global__ void __launch_bounds__(kAbT)
action_sf_kernel(const double* __restrict__ qs, const double* __restrict__ tab, double* __restrict__ ev,
                 const Geom g) {
    constexpr int D = P + 1, E = AbCfg<P, Q>::E;
    __shared__ double T[E][3][D][Q][Q];    // after backward Z: channels m = 0, 1 (B_z), 2 (G_z)
    __shared__ double R[E][2][D][D][Q];    // after backward Y: G_x channel, B_x channel
    action_sf<P, Q, E>(qs, tab, ev, g, blockIdx.x * E, T, R);
}

// The fusion stage: gradient, Voigt stress and action of a workgroup's elements in one
// kernel.  qv holds each element's quadrature-point data (9 words per point): the gradient
// pass writes it, the stress rewrites it in place, the action pass reads it; it is written
// and read back by the same workgroup only.  The two passes' LDS tiles share storage.
template <int P, int Q>
__global__ void __launch_bounds__(kAbT)
fused_unstaged_kernel(const double* __restrict__ x, const double* __restrict__ ed, const double* __restrict__ tab,
                      double* __restrict__ qv, double* __restrict__ ev, const Geom g) {
    constexpr int D = P + 1, Q3 = Q * Q * Q, E = AbCfg<P, Q>::E;
    __shared__ double S[E][3][D][Q][Q];    // Y-pass output, then backward Z output
    __shared__ double U[E][2][D][D][Q];    // X-pass output, then backward Y output
    const int e0 = blockIdx.x * E;
    grad_sf<P, Q, E>(x, tab, qv, g, e0, U, S);
    const double* w = tab + 2 * D * Q;
    for (int t = threadIdx.x; t < E * Q3; t += kAbT) {
        const int el = t / Q3, al = t % Q3, e = e0 + el;
        if (e >= g.NE) continue;
        double* pt = qv + ((size_t)e * Q3 + al) * 9;
        double in[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) in[k] = pt[k];
        point_stress<true>(ed + (size_t)e * kEdStride, w[al % Q] * w[(al / Q) % Q] * w[al / (Q * Q)], in, pt);
    }
    __syncthreads();
    action_sf<P, Q, E>(qv, tab, ev, g, e0, S, U);
}

// ---------------------------------------------------------------- assembly
// y at every node: the sum of its elements' entries in a fixed (z, y, x) order;
// clamped nodes get y = x.
template <int P>
__global__ void __launch_bounds__(256)
assemble_kernel(const double* __restrict__ x, double* __restrict__ y, const double* __restrict__ ev, const Geom g) {
    constexpr int D = P + 1, D3 = D * D * D;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.Nn) return;
    const int gx = node % g.Nx, r = node / g.Nx, gy = r % g.Ny, gz = r / g.Ny;
    const size_t NN = (size_t)g.Nn;
    double acc[3] = {0.0, 0.0, 0.0};
    if (g.clamp && clamped_node(g.clamp, gx, gy, gz, g)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = x[c * NN + node];
    } else {
        const int gg[3] = {gx, gy, gz}, nn[3] = {g.nx, g.ny, g.nz};
        int e_[3][2], l_[3][2];
        bool v_[3][2];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int qd = gg[a] / P, rr = gg[a] % P;
            if (rr != 0) {
                e_[a][0] = qd; l_[a][0] = rr; v_[a][0] = true;
                e_[a][1] = qd; l_[a][1] = rr; v_[a][1] = false;
            } else {
                e_[a][0] = qd - 1; l_[a][0] = P; v_[a][0] = qd > 0;
                e_[a][1] = qd; l_[a][1] = 0; v_[a][1] = qd < nn[a];
            }
        }
#pragma unroll
        for (int kz = 0; kz < 2; ++kz)
#pragma unroll
            for (int ky = 0; ky < 2; ++ky)
#pragma unroll
                for (int kx = 0; kx < 2; ++kx) {
                    if (!(v_[0][kx] && v_[1][ky] && v_[2][kz])) continue;
                    const int e = e_[0][kx] + g.nx * (e_[1][ky] + g.ny * e_[2][kz]);
                    const int a = l_[0][kx] + D * (l_[1][ky] + D * l_[2][kz]);
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += ev[((size_t)e * 3 + c) * D3 + a];
                }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c * NN + node] = acc[c];
}

int64_t blocks_for(int64_t n) { return (n + 255) / 256; }

template <int P, int Q>
int run_variant(pa_op* op, AblationBuffers* b, const Geom& g, const double* x, double* y, int variant) {
    constexpr int D = P + 1, D3 = D * D * D, Q3 = Q * Q * Q;
    hipStream_t s = op->stream;
    const int64_t npts = (int64_t)g.NE * Q3;
    if (variant == PA_VARIANT_FUSED_UNSTAGED) {
        hipLaunchKernelGGL((fused_unstaged_kernel<P, Q>), dim3((g.NE + AbCfg<P, Q>::E - 1) / AbCfg<P, Q>::E),
                           dim3(kAbT), 0, s, x, (const double*)op->ed, b->tab, b->qg, b->ev, g);
        PA_HIP(hipGetLastError());
        hipLaunchKernelGGL((assemble_kernel<P>), dim3(blocks_for(g.Nn)), dim3(256), 0, s, x, y, b->ev, g);
        PA_HIP(hipGetLastError());
        return PA_OK;
    }
    if (variant == PA_VARIANT_UNFUSED_DENSE)
        hipLaunchKernelGGL((grad_dense_kernel<P, Q>), dim3(blocks_for(npts)), dim3(256), 0, s, x, b->dphi, b->qg, g);
    else
        hipLaunchKernelGGL((grad_sf_kernel<P, Q>), dim3((g.NE + AbCfg<P, Q>::E - 1) / AbCfg<P, Q>::E), dim3(kAbT), 0,
                           s, x, b->tab, b->qg, g);
    PA_HIP(hipGetLastError());
    if (variant == PA_VARIANT_UNFUSED_SF_VOIGT)
        hipLaunchKernelGGL((stress_kernel<Q, true>), dim3(blocks_for(npts)), dim3(256), 0, s, (const double*)op->ed,
                           b->tab, b->qg, b->qs, npts, D * Q);
    else
        hipLaunchKernelGGL((stress_kernel<Q, false>), dim3(blocks_for(npts)), dim3(256), 0, s, (const double*)op->ed,
                           b->tab, b->qg, b->qs, npts, D * Q);
    PA_HIP(hipGetLastError());
    if (variant == PA_VARIANT_UNFUSED_DENSE)
        hipLaunchKernelGGL((action_dense_kernel<P, Q>), dim3(blocks_for((int64_t)g.NE * D3)), dim3(256), 0, s, b->qs,
                           b->dphi, b->ev, g);
    else
        hipLaunchKernelGGL((action_sf_kernel<P, Q>), dim3((g.NE + AbCfg<P, Q>::E - 1) / AbCfg<P, Q>::E), dim3(kAbT),
                           0, s, b->qs, b->tab, b->ev, g);
    PA_HIP(hipGetLastError());
    hipLaunchKernelGGL((assemble_kernel<P>), dim3(blocks_for(g.Nn)), dim3(256), 0, s, x, y, b->ev, g);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

template <int P>
int run_p(pa_op* op, AblationBuffers* b, const Geom& g, const double* x, double* y, int variant) {
    switch (op->q - op->p) {
        case 2: return run_variant<P, P + 2>(op, b, g, x, y, variant);
    }
    return fail(PA_EUNSUPPORTED, "ablation variants are built for q = p + 2 only");
}

int prepare(pa_op* op) {
    if (op->abl) return PA_OK;
    const int p = op->p, q = op->q, D = p + 1, D3 = D * D * D, Q3 = q * q * q;
    AblationBuffers* b = new (std::nothrow) AblationBuffers();
    if (!b) return fail(PA_ENOMEM, "host allocation failed");
    const size_t npts = (size_t)op->NE * Q3;
    if (hipMalloc(&b->qg, npts * 9 * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->qs, npts * 9 * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->ev, (size_t)op->NE * 3 * D3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->dphi, (size_t)D3 * Q3 * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&b->tab, (size_t)(2 * D * q + q) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        free_ablation(b);
        return fail(PA_ENOMEM, "device allocation of the ablation work arrays failed");
    }
    const Tables& t = op->tab;
    std::vector<double> tab(2 * D * q + q);
    for (int i = 0; i < D * q; ++i) {
        tab[i] = t.B[i];
        tab[D * q + i] = t.G[i];
    }
    for (int k = 0; k < q; ++k) tab[2 * D * q + k] = t.w[k];
    // dense reference basis gradients: d phi_a / d xi_m at alpha = (qx, qy, qz)
    std::vector<double> dphi((size_t)D3 * Q3 * 3);
    for (int a = 0; a < D3; ++a) {
        const int ix = a % D, iy = (a / D) % D, iz = a / (D * D);
        for (int al = 0; al < Q3; ++al) {
            const int qx = al % q, qy = (al / q) % q, qz = al / (q * q);
            const double bx = t.B[ix * q + qx], by = t.B[iy * q + qy], bz = t.B[iz * q + qz];
            const double gx = t.G[ix * q + qx], gy = t.G[iy * q + qy], gz = t.G[iz * q + qz];
            double* o = &dphi[((size_t)a * Q3 + al) * 3];
            o[0] = gx * by * bz;
            o[1] = bx * gy * bz;
            o[2] = bx * by * gz;
        }
    }
    hipError_t e = hipMemcpy(b->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->dphi, dphi.data(), dphi.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_ablation(b);
        return fail(PA_EHIP, "upload failed: %s", hipGetErrorString(e));
    }
    op->abl = b;
    return PA_OK;
}

}  // namespace

// The production fused kernel with its pointwise stage at the q^3 Gauss points (the form
// before the collocated regrouping).  Its skeleton buffer holds every element's boundary
// nodes; at p = 1 the operator's own buffer is sized for the linear-element tiles, so a work
// array (NE q^3 9 words, far more than NE 24) stands in for it.
template <int P>
int run_fused_quadrature(pa_op* op, AblationBuffers* b, const Geom& g, const double* x, double* y) {
    ApplyLaunch L;
    L.g = g;
    L.x = x;
    L.y = y;
    L.sk = (P == 1 && op->lin) ? (void*)b->qg : op->sk;
    L.ed = op->ed;
    L.tab = &op->tab;
    L.add = 0;
    L.lin = false;
    L.stream = op->stream;
    return launch_apply_typed<P, P + 2, double>(L);
}

int apply_variant(pa_op* op, const void* x, void* y, int flags, int variant) {
    if (variant == PA_VARIANT_FUSED) return apply_op(op, x, y, flags);
    if (variant != PA_VARIANT_UNFUSED_DENSE && variant != PA_VARIANT_UNFUSED_SF &&
        variant != PA_VARIANT_UNFUSED_SF_VOIGT && variant != PA_VARIANT_FUSED_UNSTAGED &&
        variant != PA_VARIANT_FUSED_QUADRATURE)
        return fail(PA_EINVAL, "unknown variant %d", variant);
    if (op->dtype != PA_F64) return fail(PA_EUNSUPPORTED, "the unfused variants are FP64 only");
    if (flags & PA_ADD) return fail(PA_EUNSUPPORTED, "the unfused variants overwrite y (no PA_ADD)");
    int rc = prepare(op);
    if (rc) return rc;
    const Geom g = make_geom(op->mesh, op->p, !(flags & PA_UNCONSTRAINED));
    if (g.NE == 0) return PA_OK;
    const double* xd = (const double*)x;
    double* yd = (double*)y;
    AblationBuffers* b = op->abl;
    if (variant == PA_VARIANT_FUSED_QUADRATURE) {
        if (op->q != op->p + 2) return fail(PA_EUNSUPPORTED, "ablation variants are built for q = p + 2 only");
        switch (op->p) {
            case 1: return run_fused_quadrature<1>(op, b, g, xd, yd);
            case 2: return run_fused_quadrature<2>(op, b, g, xd, yd);
            case 3: return run_fused_quadrature<3>(op, b, g, xd, yd);
            case 4: return run_fused_quadrature<4>(op, b, g, xd, yd);
            case 5: return run_fused_quadrature<5>(op, b, g, xd, yd);
            case 6: return run_fused_quadrature<6>(op, b, g, xd, yd);
            case 7: return run_fused_quadrature<7>(op, b, g, xd, yd);
            case 8: return run_fused_quadrature<8>(op, b, g, xd, yd);
        }
        return fail(PA_EUNSUPPORTED, "p = %d", op->p);
    }
    switch (op->p) {
        case 1: return run_p<1>(op, b, g, xd, yd, variant);
        case 2: return run_p<2>(op, b, g, xd, yd, variant);
        case 3: return run_p<3>(op, b, g, xd, yd, variant);
        case 4: return run_p<4>(op, b, g, xd, yd, variant);
        case 5: return run_p<5>(op, b, g, xd, yd, variant);
        case 6: return run_p<6>(op, b, g, xd, yd, variant);
        case 7: return run_p<7>(op, b, g, xd, yd, variant);
        case 8: return run_p<8>(op, b, g, xd, yd, variant);
    }
    return fail(PA_EUNSUPPORTED, "p = %d", op->p);
}

}  // namespace pa

using namespace pa;

extern "C" int pa_elast_apply_variant(pa_op_t* op, const void* x, void* y, int flags, int variant) {
    if (!op || !x || !y) return fail(PA_EINVAL, "NULL argument");
    if (x == y) return fail(PA_EINVAL, "x and y must not alias");
    if (flags & ~(PA_UNCONSTRAINED | PA_ADD)) return fail(PA_EINVAL, "unknown flags 0x%x", flags);
    if (variant != PA_VARIANT_FUSED && (op->mat != PA_MAT_ELEM_ISO || op->geo != PA_GEOM_AFFINE))
        return fail(PA_EUNSUPPORTED, "the unfused variants take per-element Lame parameters on the affine box");
    return apply_variant(op, x, y, flags, variant);
}
