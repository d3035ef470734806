// Fused matrix-free apply of the linear-elasticity operator on affine hexahedra.
//
// One kernel performs, per element (paper Sec. 4.2 macro-kernel fusion, Sec. 4.4
// sum factorization, Sec. 4.5 Voigt stress and backward sweeps):
//   gather x_e (restriction G)                    -> LDS tile [3][D^3]
//   forward X:  u = sum_ix x B, v = sum_ix x G    -> LDS [2][D][D][Q]
//   forward Y:  (v B, u G, u B) over iy            -> LDS [3][D][Q][Q]
//   forward Z:  over iz into a register column per (qx,qy): 3 comps x 3 dirs x Q
//   pointwise:  grad = J^{-T} ref-grad; Voigt sigma with w*detJ*lambda, w*detJ*mu;
//               Q_{c,m} = sum_i sigma_{c,i} J^{-1}_{m,i}   (in place in registers)
//   backward Z (registers -> LDS), Y, X (m-channels summed where B/G coincide),
//   scatter-add into y (G^T) with hardware FP atomics.
//
// Design for gfx950: the 1D tables B, G, w are kernel arguments (kernarg segment),
// so every contraction reads them with scalar loads as wave-uniform SGPR operands
// of the FMAs; lanes map to distinct 1D lines, each lane contracting a whole line
// with its inputs in VGPRs (no per-FMA LDS traffic).  LDS only transposes data
// between the X, Y and Z passes.  Several elements share a workgroup at low p so
// that the (qx,qy) columns fill 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"

namespace pa {

template <typename T, int D, int Q>
struct Tab1D {
    T B[D * Q];
    T G[D * Q];
    T w[Q];
};

template <typename T, int D, int Q>
inline Tab1D<T, D, Q> make_tab(const Tables& t) {
    Tab1D<T, D, Q> r;
    for (int i = 0; i < D * Q; ++i) { r.B[i] = (T)t.B[i]; r.G[i] = (T)t.G[i]; }
    for (int k = 0; k < Q; ++k) r.w[k] = (T)t.w[k];
    return r;
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

// Elements per workgroup: fill 64-lane waves with the E*Q*Q quadrature columns while
// keeping the workgroup's LDS at or below 64 KiB.
template <int P, int Q, typename T>
struct ApplyCfg {
    static constexpr int D = P + 1;
    static constexpr int QQ = Q * Q;
    static constexpr int LDS_ELEM = 3 * D * D * D + 2 * D * D * Q + 3 * D * Q * Q;  // words / element
    static constexpr int pickE() {
        int bestE = 1;
        double bestU = 0.0;
        for (int E = 1; E * QQ <= 256; ++E) {
            if (E > 1 && E * LDS_ELEM * (int)sizeof(T) > 65536) break;
            int nt = ((E * QQ + 63) / 64) * 64;
            double u = double(E * QQ) / nt;
            if (u > bestU + 0.02) { bestU = u; bestE = E; }
        }
        return bestE;
    }
    static constexpr int E = pickE();
    static constexpr int NT = ((E * QQ + 63) / 64) * 64;
};

// Consecutive workgroups are dealt round-robin to the 8 XCDs; remap so that each
// XCD receives a contiguous range of element blocks (shared faces stay in one L2).
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, k = b >> 3;
    const int start = xcd * per + (xcd < rem ? xcd : rem);
    return start + k;
}

template <int P, int Q, typename T>
__global__ void __launch_bounds__((ApplyCfg<P, Q, T>::NT))
pa_apply_kernel(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ ed,
                const Tab1D<T, P + 1, Q> tab, const Geom g) {
    using C = ApplyCfg<P, Q, T>;
    constexpr int D = P + 1, E = C::E, NT = C::NT, QQ = Q * Q;
    constexpr int D3 = D * D * D;
    constexpr int XS = 3 * D3;          // gather/scatter tile per element
    constexpr int US = 2 * D * D * Q;   // X-pass output per element
    constexpr int SS = 3 * D * Q * Q;   // Y-pass output per element
    __shared__ T Xs[E * XS];
    __shared__ T Us[E * US];
    __shared__ T Ss[E * SS];

    const int tid = threadIdx.x;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int e0 = blk * E;

    // ---- gather (restriction G): x -> Xs[el][c][iz][iy][ix]
    for (int w = tid; w < E * XS; w += NT) {
        const int el = w / XS, r = w % XS;
        const int c = r / D3, a = r % D3;
        const int ix = a % D, iy = (a / D) % D, iz = a / (D * D);
        const int e = e0 + el;
        T v = T(0);
        if (e < g.NE) {
            const int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
            const int gx = ex * P + ix, gy = ey * P + iy, gz = ez * P + iz;
            if (!clamped_node(g.clamp, gx, gy, gz, g))
                v = x[(size_t)c * g.Nn + gx + g.Nx * (gy + g.Ny * gz)];
        }
        Xs[w] = v;
    }

    // column owned by this thread in the Z / pointwise stage
    const int cel = tid / QQ, cq = tid % QQ;
    const int cqx = cq % Q, cqy = cq / Q;
    const bool has_col = tid < E * QQ;
    T gq[3][3][Q];   // [component][reference direction][qz]

    __syncthreads();

#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // ---- forward X: lines (el, iz, iy)
        for (int w = tid; w < E * D * D; w += NT) {
            const int el = w / (D * D), r = w % (D * D);
            const T* xin = Xs + el * XS + c * D3 + r * D;
            T xv[D];
#pragma unroll
            for (int i = 0; i < D; ++i) xv[i] = xin[i];
            T* uo = Us + el * US + r * Q;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                T u = T(0), v = T(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    u = fma(xv[i], tab.B[i * Q + k], u);
                    v = fma(xv[i], tab.G[i * Q + k], v);
                }
                uo[k] = u;
                uo[D * D * Q + k] = v;
            }
        }
        __syncthreads();
        // ---- forward Y: lines (el, iz, qx)
        for (int w = tid; w < E * D * Q; w += NT) {
            const int el = w / (D * Q), r = w % (D * Q);
            const int iz = r / Q, qx = r % Q;
            const T* ui = Us + el * US + iz * D * Q + qx;
            T uv[D], vv[D];
#pragma unroll
            for (int i = 0; i < D; ++i) { uv[i] = ui[i * Q]; vv[i] = ui[D * D * Q + i * Q]; }
            T* so = Ss + el * SS + iz * QQ + qx;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    s0 = fma(vv[i], tab.B[i * Q + k], s0);   // d/dxi
                    s1 = fma(uv[i], tab.G[i * Q + k], s1);   // d/deta
                    s2 = fma(uv[i], tab.B[i * Q + k], s2);   // value (for d/dzeta)
                }
                so[k * Q] = s0;
                so[D * QQ + k * Q] = s1;
                so[2 * D * QQ + k * Q] = s2;
            }
        }
        __syncthreads();
        // ---- forward Z: the thread's own (qx,qy) column
        if (has_col) {
            const T* si = Ss + cel * SS + cq;
#pragma unroll
            for (int k = 0; k < Q; ++k) { gq[c][0][k] = T(0); gq[c][1][k] = T(0); gq[c][2][k] = T(0); }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const T s0 = si[i * QQ], s1 = si[D * QQ + i * QQ], s2 = si[2 * D * QQ + i * QQ];
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    gq[c][0][k] = fma(s0, tab.B[i * Q + k], gq[c][0][k]);
                    gq[c][1][k] = fma(s1, tab.B[i * Q + k], gq[c][1][k]);
                    gq[c][2][k] = fma(s2, tab.G[i * Q + k], gq[c][2][k]);
                }
            }
        }
        // the next X pass writes Us only; Ss is rewritten after the next barrier
    }

    // ---- pointwise stage: Voigt stress and Q = sigma J^{-T}, in place
    if (has_col) {
        const int e = e0 + cel;
        T Ji[9], lw = T(0), mw = T(0);
        if (e < g.NE) {
            const T* d = ed + (size_t)e * kEdStride;
#pragma unroll
            for (int k = 0; k < 9; ++k) Ji[k] = d[k];
            lw = d[9];
            mw = d[10];
        } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) Ji[k] = T(0);
        }
        const T wxy = tab.w[cqx] * tab.w[cqy];
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const T W = wxy * tab.w[k];
            const T lam = W * lw, mu = W * mw;
            // physical gradient du[c][i] = d u_c / d x_i = sum_m Jinv[m][i] * ref[c][m]
            T du[3][3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    du[cc][i] = Ji[0 * 3 + i] * gq[cc][0][k] + Ji[1 * 3 + i] * gq[cc][1][k] +
                                Ji[2 * 3 + i] * gq[cc][2][k];
            const T div = du[0][0] + du[1][1] + du[2][2];
            const T ld = lam * div, m2 = mu + mu;
            T s[3][3];
            s[0][0] = ld + m2 * du[0][0];
            s[1][1] = ld + m2 * du[1][1];
            s[2][2] = ld + m2 * du[2][2];
            s[0][1] = s[1][0] = mu * (du[0][1] + du[1][0]);
            s[0][2] = s[2][0] = mu * (du[0][2] + du[2][0]);
            s[1][2] = s[2][1] = mu * (du[1][2] + du[2][1]);
            // Q_{c,m} = sum_i sigma_{c,i} Jinv[m][i]
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    gq[cc][m][k] = s[cc][0] * Ji[m * 3 + 0] + s[cc][1] * Ji[m * 3 + 1] + s[cc][2] * Ji[m * 3 + 2];
        }
    }

    // ---- backward sweeps, one output component at a time
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // backward Z: column -> Ss[el][m][iz][qy][qx]
        if (has_col) {
            T* so = Ss + cel * SS + cq;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                T t0 = T(0), t1 = T(0), t2 = T(0);
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    t0 = fma(gq[c][0][k], tab.B[i * Q + k], t0);
                    t1 = fma(gq[c][1][k], tab.B[i * Q + k], t1);
                    t2 = fma(gq[c][2][k], tab.G[i * Q + k], t2);
                }
                so[i * QQ] = t0;
                so[D * QQ + i * QQ] = t1;
                so[2 * D * QQ + i * QQ] = t2;
            }
        }
        __syncthreads();
        // backward Y: lines (el, iz, qx): R0 = sum_qy T0 B, R12 = sum_qy (T1 G + T2 B)
        for (int w = tid; w < E * D * Q; w += NT) {
            const int el = w / (D * Q), r = w % (D * Q);
            const int iz = r / Q, qx = r % Q;
            const T* ti = Ss + el * SS + iz * QQ + qx;
            T t0[Q], t1[Q], t2[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                t0[k] = ti[k * Q];
                t1[k] = ti[D * QQ + k * Q];
                t2[k] = ti[2 * D * QQ + k * Q];
            }
            T* ro = Us + el * US + iz * D * Q + qx;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                T r0 = T(0), r12 = T(0);
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    r0 = fma(t0[k], tab.B[i * Q + k], r0);
                    r12 = fma(t1[k], tab.G[i * Q + k], r12);
                    r12 = fma(t2[k], tab.B[i * Q + k], r12);
                }
                ro[i * Q] = r0;
                ro[D * D * Q + i * Q] = r12;
            }
        }
        __syncthreads();
        // backward X: lines (el, iz, iy): y(ix) = sum_qx R0 G + R12 B  -> Xs (output tile)
        for (int w = tid; w < E * D * D; w += NT) {
            const int el = w / (D * D), r = w % (D * D);
            const T* ri = Us + el * US + r * Q;
            T r0[Q], r12[Q];
#pragma unroll
            for (int k = 0; k < Q; ++k) { r0[k] = ri[k]; r12[k] = ri[D * D * Q + k]; }
            T* yo = Xs + el * XS + c * D3 + r * D;
#pragma unroll
            for (int i = 0; i < D; ++i) {
                T acc = T(0);
#pragma unroll
                for (int k = 0; k < Q; ++k) {
                    acc = fma(r0[k], tab.G[i * Q + k], acc);
                    acc = fma(r12[k], tab.B[i * Q + k], acc);
                }
                yo[i] = acc;
            }
        }
        // next component's backward Z writes Ss only (last read before the barrier above)
    }
    __syncthreads();

    // ---- scatter-add (G^T)
    for (int w = tid; w < E * XS; w += NT) {
        const int el = w / XS, r = w % XS;
        const int e = e0 + el;
        if (e >= g.NE) continue;
        const int c = r / D3, a = r % D3;
        const int ix = a % D, iy = (a / D) % D, iz = a / (D * D);
        const int ex = e % g.nx, ey = (e / g.nx) % g.ny, ez = e / (g.nx * g.ny);
        const int gx = ex * P + ix, gy = ey * P + iy, gz = ez * P + iz;
        if (clamped_node(g.clamp, gx, gy, gz, g)) continue;
        atomic_add(y + (size_t)c * g.Nn + gx + g.Nx * (gy + g.Ny * gz), Xs[w]);
    }
}

template <int P, int Q, typename T>
int launch_apply_typed(const ApplyLaunch& L) {
    using C = ApplyCfg<P, Q, T>;
    if (L.g.NE == 0) return PA_OK;
    const Tab1D<T, P + 1, Q> tab = make_tab<T, P + 1, Q>(*L.tab);
    const int nb = (L.g.NE + C::E - 1) / C::E;
    hipLaunchKernelGGL((pa_apply_kernel<P, Q, T>), dim3(nb), dim3(C::NT), 0, L.stream,
                       (const T*)L.x, (T*)L.y, (const T*)L.ed, tab, L.g);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

template <int P>
int launch_apply_p(const ApplyLaunch& L, int q_off, int dtype) {
    if (dtype == PA_F64) {
        switch (q_off) {
            case 0: return launch_apply_typed<P, P + 1, double>(L);
            case 1: return launch_apply_typed<P, P + 2, double>(L);
            case 2: return launch_apply_typed<P, P + 3, double>(L);
        }
    } else {
        switch (q_off) {
            case 0: return launch_apply_typed<P, P + 1, float>(L);
            case 1: return launch_apply_typed<P, P + 2, float>(L);
            case 2: return launch_apply_typed<P, P + 3, float>(L);
        }
    }
    return fail(PA_EUNSUPPORTED, "q = p+1+%d not built", q_off);
}

}  // namespace pa
