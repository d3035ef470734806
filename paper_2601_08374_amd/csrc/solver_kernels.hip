// Streaming kernels of the solver: reductions with FP64 accumulation, PCG and
// Chebyshev vector updates, casts, p/h transfers, coarse-matrix assembly and
// inversion, SplitMix64 start vectors.  All of them are HBM-bound except the
// coarse assembly/inversion (setup only).
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kernels.h"
#include "solver.h"

namespace pa {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    return (int)(b < 1 ? 1 : b);
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// ---------------------------------------------------------------- reductions
// Stage 1: every block reduces a fixed grid-stride slice in FP64 (fixed grid ->
// deterministic); stage 2 (one block) sums the partials in a fixed order and
// then runs the scalar logic of the caller (alpha, beta, convergence test).
template <typename TA, typename TB>
__global__ void dot_partial_kernel(const TA* __restrict__ a, const TB* __restrict__ b, const TB* __restrict__ c,
                                   int64_t n, double* __restrict__ part) {
    // part[blk] = sum a*b ; if c: part[gridDim + blk] = sum a*a (second product)
    __shared__ double s0[kBlock], s1[kBlock];
    double acc0 = 0.0, acc1 = 0.0;
    GRID_STRIDE(i, n) {
        const double av = (double)a[i];
        acc0 += av * (double)b[i];
        if (c) acc1 += av * av;
    }
    s0[threadIdx.x] = acc0;
    s1[threadIdx.x] = acc1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] += s0[threadIdx.x + w];
            s1[threadIdx.x] += s1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0[0];
        part[gridDim.x + blockIdx.x] = s1[0];
    }
}

__device__ double block_sum(const double* part, int np, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// PCG scalar logic, run by thread 0 after the sums are known.
//   op = FIN_STORE : s[slot] = sum0
//   op = FIN_ALPHA : s[PAP] = sum0; alpha = rz/pAp unless done; breakdown if pAp <= 0 or NaN
//   op = FIN_BETA  : rz_new = sum0 (r.z), rr = sum1 (r.r); convergence test; beta = rz_new/rz; rz = rz_new
__global__ void dot_final_kernel(const double* __restrict__ part, int np, double* __restrict__ s, int op, int slot) {
    __shared__ double sh[kBlock];
    const double s0 = block_sum(part, np, sh);
    const double s1 = block_sum(part + np, np, sh);
    if (threadIdx.x != 0) return;
    if (op == FIN_STORE) {
        s[slot] = s0;
        s[slot + 1] = s1;
        return;
    }
    if (s[S_DONE] != 0.0) return;
    if (op == FIN_ALPHA) {
        s[S_PAP] = s0;
        if (!(s0 > 0.0) || s0 != s0) {
            s[S_DONE] = 2.0;   // breakdown
            s[S_ALPHA] = 0.0;
            return;
        }
        s[S_ALPHA] = s[S_RZ] / s0;
        return;
    }
    // FIN_BETA
    const double rz_new = s0, rr = s1;
    s[S_ITERS] += 1.0;
    const bool prec = s[S_STOP] == 0.0;
    const double crit = prec ? sqrt(fabs(rz_new) / s[S_RZ0]) : sqrt(rr / s[S_BB]);
    s[S_CRIT] = crit;
    s[S_RRLAST] = rr;
    if (rz_new != rz_new || rr != rr) {
        s[S_DONE] = 2.0;
        return;
    }
    if (crit <= s[S_RTOL]) {
        s[S_DONE] = 1.0;
        s[S_BETA] = 0.0;
        return;
    }
    s[S_BETA] = rz_new / s[S_RZ];
    s[S_RZ] = rz_new;
}

// After the first preconditioner application: rz = rz0 = r.z, rr0 = r.r.
__global__ void pcg_init_scalars_kernel(const double* __restrict__ part, int np, double* __restrict__ s,
                                        double rtol, int stop) {
    __shared__ double sh[kBlock];
    const double s0 = block_sum(part, np, sh);
    const double s1 = block_sum(part + np, np, sh);
    if (threadIdx.x != 0) return;
    s[S_RZ] = s0;
    s[S_RZ0] = s0 > 0.0 ? s0 : 1.0;
    s[S_RTOL] = rtol;
    s[S_STOP] = (double)stop;
    s[S_ITERS] = 0.0;
    s[S_DONE] = 0.0;
    s[S_ALPHA] = 0.0;
    s[S_BETA] = 0.0;
    s[S_RRLAST] = s1;
    const bool prec = stop == 0;
    const double crit = prec ? 1.0 : sqrt(s1 / s[S_BB]);
    s[S_CRIT] = crit;
    if (s0 == 0.0 || (!prec && crit <= rtol) || s1 == 0.0) s[S_DONE] = 1.0;   // already solved
}

// ---------------------------------------------------------------- PCG updates
template <typename T>
__global__ void pcg_xr_kernel(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ Ap,
                              const double* __restrict__ s, int64_t n) {
    if (s[S_DONE] != 0.0) return;
    const T a = (T)s[S_ALPHA];
    GRID_STRIDE(i, n) {
        x[i] += a * p[i];
        r[i] -= a * Ap[i];
    }
}

template <typename T>
__global__ void pcg_p_kernel(T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ s, int64_t n) {
    if (s[S_DONE] != 0.0) return;
    const T b = (T)s[S_BETA];
    GRID_STRIDE(i, n) p[i] = z[i] + b * p[i];
}

// ---------------------------------------------------------------- generic vector ops
template <typename T>
__global__ void residual_kernel(T* __restrict__ r, const T* __restrict__ b, const T* __restrict__ Ax, int64_t n) {
    GRID_STRIDE(i, n) r[i] = b[i] - Ax[i];
}

template <typename T>
__global__ void copy_kernel(T* __restrict__ y, const T* __restrict__ x, int64_t n) {
    GRID_STRIDE(i, n) y[i] = x[i];
}

template <typename TO, typename TI>
__global__ void cast_scale_kernel(TO* __restrict__ y, const TI* __restrict__ x, const double* __restrict__ s, int slot,
                                  int inv_sqrt, int64_t n) {
    // y = x * f, f = 1/sqrt(s[slot]) (inv_sqrt) or sqrt(s[slot]) (!inv_sqrt)
    const double v = s[slot];
    const double f = inv_sqrt ? (v > 0.0 ? 1.0 / sqrt(v) : 0.0) : sqrt(v);
    GRID_STRIDE(i, n) y[i] = (TO)((double)x[i] * f);
}

template <typename TI>
__global__ void ir_update_kernel(double* __restrict__ x, const TI* __restrict__ d, const double* __restrict__ s,
                                 int slot, int64_t n) {
    // x += sqrt(s[slot]) * d   (the correction was solved for the unit-norm residual)
    const double f = sqrt(s[slot]);
    GRID_STRIDE(i, n) x[i] += f * (double)d[i];
}

// Chebyshev step: x += d (x = d when XZERO: the smoother started from x = 0);
// r -= t; d = c1*d + c2*dinv*r.  LAST: the smoother's final update x += d is folded
// in (x = (x + d) + d_new) and r, d are not written back (dead afterwards).
template <typename T, bool XZERO, bool LAST>
__global__ void cheb_step_kernel(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ t, T* __restrict__ d,
                                 const T* __restrict__ dinv, double c1, double c2, int64_t n) {
    const T a = (T)c1, b = (T)c2;
    GRID_STRIDE(i, n) {
        const T dv = d[i];
        const T xv = XZERO ? dv : x[i] + dv;
        const T rv = r[i] - t[i];
        const T dn = a * dv + b * dinv[i] * rv;
        if (LAST) {
            x[i] = xv + dn;
        } else {
            x[i] = xv;
            r[i] = rv;
            d[i] = dn;
        }
    }
}

// Start of the smoother: r = b - t (or r = b when t is null: x = 0); d = c*dinv*r.
template <typename T>
__global__ void cheb_start_kernel(T* __restrict__ r, T* __restrict__ d, const T* __restrict__ dinv,
                                  const T* __restrict__ b, const T* __restrict__ t, double c, int64_t n) {
    const T tc = (T)c;
    GRID_STRIDE(i, n) {
        const T rv = t ? b[i] - t[i] : b[i];
        r[i] = rv;
        d[i] = tc * dinv[i] * rv;
    }
}

template <typename T>
__global__ void add_kernel(T* __restrict__ y, const T* __restrict__ x, int64_t n) {
    GRID_STRIDE(i, n) y[i] += x[i];
}

template <typename T>
__global__ void reciprocal_kernel(T* __restrict__ y, int64_t n) {
    GRID_STRIDE(i, n) y[i] = T(1) / y[i];
}

// v[i] = 2u-1 from the (i+1)-th output of SplitMix64 seeded with `seed` (Steele-Lea-Flood / Vigna).
template <typename T>
__global__ void splitmix_kernel(T* __restrict__ v, uint64_t seed, int64_t n) {
    GRID_STRIDE(i, n) {
        uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        v[i] = (T)(2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0);
    }
}

// One power-iteration pass after w = A v, in one read of v, w and dinv: z = dinv w is
// written out and three stage-1 sums are formed, v.w -> part[blk], v.Dv (v_i^2 / dinv_i)
// -> part[nb + blk], z.z -> part[2 nb + blk] (part[3 nb + blk] = 0).  Each sum is the
// fixed-grid, fixed-order block reduction of the dot kernels, so it is deterministic.
template <typename T>
__global__ void power_pass_kernel(const T* __restrict__ v, const T* __restrict__ w, const T* __restrict__ dinv,
                                  T* __restrict__ z, int64_t n, double* __restrict__ part) {
    __shared__ double s0[kBlock], s1[kBlock], s2[kBlock];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    GRID_STRIDE(i, n) {
        const double vv = (double)v[i];
        const T zt = dinv[i] * w[i];
        z[i] = zt;
        a0 += vv * (double)w[i];
        a1 += vv * vv / (double)dinv[i];
        a2 += (double)zt * (double)zt;
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) {
            s0[threadIdx.x] += s0[threadIdx.x + k];
            s1[threadIdx.x] += s1[threadIdx.x + k];
            s2[threadIdx.x] += s2[threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0[0];
        part[gridDim.x + blockIdx.x] = s1[0];
        part[2 * gridDim.x + blockIdx.x] = s2[0];
        part[3 * gridDim.x + blockIdx.x] = 0.0;
    }
}

// ---------------------------------------------------------------- p-transfer
// Per element, fine nodal values = (I (x) I (x) I) coarse nodal values with
// I[i][j] = l^c_j(xi^f_i) (coarse Lagrange basis at the fine Gauss-Lobatto nodes).
// A fine node is written only by its owner element (local index < pf, or the last
// element of the axis), so prolongation is deterministic and race-free.
// Restriction is the exact transpose: each element contracts the owned entries of
// the fine vector with I^T; coarse nodes inside the element are written directly and
// element-boundary ones go to a per-element buffer that p_restrict_gather_kernel sums
// per coarse node in a fixed order (deterministic, no atomics).
__device__ __forceinline__ bool owns(int e, int i, int n, int p) { return i < p || e == n - 1; }

// Element-boundary local nodes of a D^3 element (some index 0 or D-1), numbered in
// (iz, iy, ix)-lexicographic order: D*D on the full layers iz = 0, D-1 and 4(D-1) on
// each inner layer.
__device__ __forceinline__ int skel_count(int D) { return D * D * D - (D - 2) * (D - 2) * (D - 2); }
__device__ __forceinline__ int skel_slot(int D, int ix, int iy, int iz) {
    const int P = D - 1, layer = 4 * (D - 1);
    if (iz == 0) return iy * D + ix;
    if (iz == P) return D * D + (D - 2) * layer + iy * D + ix;
    const int base = D * D + (iz - 1) * layer;
    if (iy == 0) return base + ix;
    if (iy == P) return base + D + 2 * (D - 2) + ix;
    return base + D + 2 * (iy - 1) + (ix == P ? 1 : 0);
}

// Elements per workgroup of the p-transfer kernels: about 256 lanes, one per fine
// (ix, iy) column of an element.
constexpr int transfer_elems(int Df) { return 256 / (Df * Df) > 0 ? 256 / (Df * Df) : 1; }

// Prolongation xf (+)= P xc between degrees PF and PC = PF / 2 on one mesh.  The
// coarse element values are staged in LDS; one lane per fine (ix, iy) column contracts
// them in x and y for its column, then in z for each fine iz, and writes the nodes of
// its column that the element owns (clamped fine nodes get 0, or keep their value
// when adding).
template <int PF, typename T>
__global__ void __launch_bounds__(256)
p_prolong_kernel(const T* __restrict__ xc, T* __restrict__ xf, const double* __restrict__ I, Geom gc, Geom gf,
                 int add) {
    constexpr int PC = PF / 2, Dc = PC + 1, Df = PF + 1, Dc3 = Dc * Dc * Dc, EB = transfer_elems(Df);
    __shared__ double Is[Df * Dc];          // I[i][j] = l^c_j(xi^f_i)
    __shared__ double X[EB * 3 * Dc3];      // coarse values of the block's elements
    const int tid = threadIdx.x;
    const int e0 = blockIdx.x * EB;
    const int neb = gf.NE - e0 < EB ? gf.NE - e0 : EB;
    for (int w = tid; w < Df * Dc; w += blockDim.x) Is[w] = I[w];
    for (int w = tid; w < neb * 3 * Dc3; w += blockDim.x) {
        const int el = w / (3 * Dc3), r = w % (3 * Dc3), c = r / Dc3, a = r % Dc3;
        const int e = e0 + el;
        const int ex = e % gf.nx, ey = (e / gf.nx) % gf.ny, ez = e / (gf.nx * gf.ny);
        const int jx = a % Dc, jy = (a / Dc) % Dc, jz = a / (Dc * Dc);
        const size_t node = (size_t)(ex * PC + jx) + gc.Nx * ((ey * PC + jy) + (size_t)gc.Ny * (ez * PC + jz));
        X[w] = (double)xc[(size_t)c * gc.Nn + node];
    }
    __syncthreads();
    const int el = tid / (Df * Df), col = tid % (Df * Df);
    if (el >= neb) return;   // no barrier follows
    const int ix = col % Df, iy = col / Df;
    const int e = e0 + el;
    const int ex = e % gf.nx, ey = (e / gf.nx) % gf.ny, ez = e / (gf.nx * gf.ny);
    if (!owns(ex, ix, gf.nx, PF) || !owns(ey, iy, gf.ny, PF)) return;
    const int gx = ex * PF + ix, gy = ey * PF + iy;
    double Ix[Dc], Iy[Dc];
#pragma unroll
    for (int j = 0; j < Dc; ++j) {
        Ix[j] = Is[ix * Dc + j];
        Iy[j] = Is[iy * Dc + j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* Xc = X + (el * 3 + c) * Dc3;
        double Tz[Dc];
#pragma unroll
        for (int jz = 0; jz < Dc; ++jz) {
            double acc = 0.0;
#pragma unroll
            for (int jy = 0; jy < Dc; ++jy) {
                double w = 0.0;
#pragma unroll
                for (int jx = 0; jx < Dc; ++jx) w += Ix[jx] * Xc[(jz * Dc + jy) * Dc + jx];
                acc += Iy[jy] * w;
            }
            Tz[jz] = acc;
        }
#pragma unroll
        for (int iz = 0; iz < Df; ++iz) {
            if (!owns(ez, iz, gf.nz, PF)) continue;
            const int gz = ez * PF + iz;
            double v = 0.0;
#pragma unroll
            for (int jz = 0; jz < Dc; ++jz) v += Is[iz * Dc + jz] * Tz[jz];
            const size_t o = (size_t)c * gf.Nn + gx + gf.Nx * (gy + (size_t)gf.Ny * gz);
            if (clamped_node(gf.clamp, gx, gy, gz, gf)) {
                if (!add) xf[o] = T(0);
            } else {
                xf[o] = add ? xf[o] + (T)v : (T)v;
            }
        }
    }
}

// Restriction rc = P^T (rf - tf) (tf optional), the exact transpose: each element takes
// the fine values it owns.  Stage 1, one lane per fine (ix, iy) column: contract z into
// LDS.  Stage 2, one lane per (element, c, jz, jy): contract y and x; coarse nodes inside
// the element are written directly, element-boundary ones to skr (summed per coarse node
// in a fixed order by p_restrict_gather_kernel).
template <int PF, typename T>
__global__ void __launch_bounds__(256)
p_restrict_kernel(const T* __restrict__ rf, const T* __restrict__ tf, T* __restrict__ rc, T* __restrict__ skr,
                  const double* __restrict__ I, Geom gc, Geom gf) {
    constexpr int PC = PF / 2, Dc = PC + 1, Df = PF + 1, EB = transfer_elems(Df);
    __shared__ double Is[Df * Dc];
    __shared__ double U[EB * 3 * Dc * Df * Df];   // [el][c][jz][iy][ix]
    const int tid = threadIdx.x;
    const int e0 = blockIdx.x * EB;
    const int neb = gf.NE - e0 < EB ? gf.NE - e0 : EB;
    for (int w = tid; w < Df * Dc; w += blockDim.x) Is[w] = I[w];
    __syncthreads();
    {
        const int el = tid / (Df * Df), col = tid % (Df * Df);
        if (el < neb) {
            const int ix = col % Df, iy = col / Df;
            const int e = e0 + el;
            const int ex = e % gf.nx, ey = (e / gf.nx) % gf.ny, ez = e / (gf.nx * gf.ny);
            const bool own_xy = owns(ex, ix, gf.nx, PF) && owns(ey, iy, gf.ny, PF);
            const int gx = ex * PF + ix, gy = ey * PF + iy;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double u[Dc];
#pragma unroll
                for (int jz = 0; jz < Dc; ++jz) u[jz] = 0.0;
#pragma unroll
                for (int iz = 0; iz < Df; ++iz) {
                    if (!own_xy || !owns(ez, iz, gf.nz, PF)) continue;
                    const size_t o = (size_t)c * gf.Nn + gx + gf.Nx * (gy + (size_t)gf.Ny * (ez * PF + iz));
                    const double v = tf ? (double)(rf[o] - tf[o]) : (double)rf[o];
#pragma unroll
                    for (int jz = 0; jz < Dc; ++jz) u[jz] += Is[iz * Dc + jz] * v;
                }
#pragma unroll
                for (int jz = 0; jz < Dc; ++jz) U[((el * 3 + c) * Dc + jz) * Df * Df + col] = u[jz];
            }
        }
    }
    __syncthreads();
    for (int w = tid; w < neb * 3 * Dc * Dc; w += blockDim.x) {
        const int el = w / (3 * Dc * Dc), r = w % (3 * Dc * Dc), c = r / (Dc * Dc), jz = (r / Dc) % Dc, jy = r % Dc;
        const double* Ur = U + ((el * 3 + c) * Dc + jz) * Df * Df;
        double out[Dc];
#pragma unroll
        for (int jx = 0; jx < Dc; ++jx) out[jx] = 0.0;
#pragma unroll 1
        for (int iy = 0; iy < Df; ++iy) {
            const double wy = Is[iy * Dc + jy];
#pragma unroll
            for (int jx = 0; jx < Dc; ++jx) {
                double v = 0.0;
#pragma unroll
                for (int ix = 0; ix < Df; ++ix) v += Is[ix * Dc + jx] * Ur[iy * Df + ix];
                out[jx] += wy * v;
            }
        }
        const int e = e0 + el;
        const int ex = e % gf.nx, ey = (e / gf.nx) % gf.ny, ez = e / (gf.nx * gf.ny);
#pragma unroll
        for (int jx = 0; jx < Dc; ++jx) {
            const bool inner = jx > 0 && jx < PC && jy > 0 && jy < PC && jz > 0 && jz < PC;
            if (inner) {
                const int gx = ex * PC + jx, gy = ey * PC + jy, gz = ez * PC + jz;
                rc[(size_t)c * gc.Nn + gx + gc.Nx * (gy + (size_t)gc.Ny * gz)] = (T)out[jx];
            } else {
                skr[((size_t)e * 3 + c) * skel_count(Dc) + skel_slot(Dc, jx, jy, jz)] = (T)out[jx];
            }
        }
    }
}

// Every coarse node on an element boundary: the sum of its elements' entries in a fixed
// (z, y, x) order; clamped nodes get 0.  Element-interior nodes were written already.
template <typename T>
__global__ void p_restrict_gather_kernel(T* __restrict__ rc, const T* __restrict__ skr, int pc, Geom gc) {
    const int Dc = pc + 1, S = skel_count(Dc);
    GRID_STRIDE(node, (int64_t)gc.Nn) {
        const int gx = (int)(node % gc.Nx), gy = (int)((node / gc.Nx) % gc.Ny), gz = (int)(node / ((int64_t)gc.Nx * gc.Ny));
        if (gx % pc != 0 && gy % pc != 0 && gz % pc != 0) continue;   // written by its element
        const bool cl = clamped_node(gc.clamp, gx, gy, gz, gc);
        double acc[3] = {0.0, 0.0, 0.0};
        if (!cl) {
            const NodeCands nc = node_candidates(gc, pc, gx, gy, gz);
            for (int kz = 0; kz < 2; ++kz)
                for (int ky = 0; ky < 2; ++ky)
                    for (int kx = 0; kx < 2; ++kx) {
                        if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                        const int e = nc.e[0][kx] + gc.nx * (nc.e[1][ky] + gc.ny * nc.e[2][kz]);
                        const int sl = skel_slot(Dc, nc.l[0][kx], nc.l[1][ky], nc.l[2][kz]);
                        for (int c = 0; c < 3; ++c) acc[c] += (double)skr[((size_t)e * 3 + c) * S + sl];
                    }
        }
        for (int c = 0; c < 3; ++c) rc[(size_t)c * gc.Nn + node] = (T)acc[c];
    }
}

// I[i][j] = l^c_j(xi^f_i) from the two sets of Gauss-Lobatto nodes
__global__ void p_interp_matrix_kernel(const double* __restrict__ gll_c, const double* __restrict__ gll_f, int pc,
                                       int pf, double* __restrict__ I) {
    const int Dc = pc + 1, Df = pf + 1;
    const int w = threadIdx.x;
    if (w >= Df * Dc) return;
    const int i = w / Dc, j = w % Dc;
    const double x = gll_f[i];
    double v = 1.0;
    for (int m = 0; m < Dc; ++m)
        if (m != j) v *= (x - gll_c[m]) / (gll_c[j] - gll_c[m]);
    I[w] = v;
}

// ---------------------------------------------------------------- h-transfer (p = 1)
// Per axis: fine vertex g takes coarse vertices i0[g], i1[g] with weights 1-t[g], t[g];
// the transpose lists, for coarse vertex j, up to 3 fine vertices fi[j][k] with fw[j][k].
template <typename T>
__global__ void h_prolong_kernel(const T* __restrict__ xc, T* __restrict__ xf, HAxis ax, HAxis ay, HAxis az, Geom gc,
                                 Geom gf, int add) {
    GRID_STRIDE(node, (int64_t)gf.Nn) {
        const int gx = (int)(node % gf.Nx), gy = (int)((node / gf.Nx) % gf.Ny), gz = (int)(node / ((int64_t)gf.Nx * gf.Ny));
        const bool cl = clamped_node(gf.clamp, gx, gy, gz, gf);
        const int xs[2] = {ax.i0[gx], ax.i1[gx]}, ys[2] = {ay.i0[gy], ay.i1[gy]}, zs[2] = {az.i0[gz], az.i1[gz]};
        const double wx[2] = {1.0 - ax.t[gx], ax.t[gx]}, wy[2] = {1.0 - ay.t[gy], ay.t[gy]},
                     wz[2] = {1.0 - az.t[gz], az.t[gz]};
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int d = 0; d < 2; ++d) {
                        const double w = wx[d] * wy[b] * wz[a];
                        if (w != 0.0)
                            acc += w * (double)xc[(size_t)c * gc.Nn + xs[d] + gc.Nx * (ys[b] + gc.Ny * zs[a])];
                    }
            const size_t o = (size_t)c * gf.Nn + node;
            if (cl) {
                if (!add) xf[o] = T(0);
            } else {
                xf[o] = add ? xf[o] + (T)acc : (T)acc;
            }
        }
    }
}

template <typename T>
__global__ void h_restrict_kernel(const T* __restrict__ rf, const T* __restrict__ tf, T* __restrict__ rc, HAxis ax,
                                  HAxis ay, HAxis az, Geom gc, Geom gf) {
    // one lane per (component, coarse node): the coarse levels are small
    GRID_STRIDE(w, 3 * (int64_t)gc.Nn) {
        const int c = (int)(w / gc.Nn);
        const int64_t node = w % gc.Nn;
        const int jx = (int)(node % gc.Nx), jy = (int)((node / gc.Nx) % gc.Ny), jz = (int)(node / ((int64_t)gc.Nx * gc.Ny));
        double acc = 0.0;
        if (!clamped_node(gc.clamp, jx, jy, jz, gc)) {
            for (int a = 0; a < 3; ++a) {
                const double wz = az.fw[jz * 3 + a];
                if (wz == 0.0) continue;
                for (int b = 0; b < 3; ++b) {
                    const double wy = ay.fw[jy * 3 + b];
                    if (wy == 0.0) continue;
                    for (int d = 0; d < 3; ++d) {
                        const double wx = ax.fw[jx * 3 + d];
                        if (wx == 0.0) continue;
                        const size_t o = (size_t)c * gf.Nn + ax.fi[jx * 3 + d] +
                                         gf.Nx * (ay.fi[jy * 3 + b] + gf.Ny * az.fi[jz * 3 + a]);
                        acc += wx * wy * wz * (tf ? (double)(rf[o] - tf[o]) : (double)rf[o]);
                    }
                }
            }
        }
        rc[(size_t)c * gc.Nn + node] = (T)acc;
    }
}

// ---------------------------------------------------------------- coarse matrix
// Dense assembly of the constrained operator of a (small) level:
// K[(c,a),(d,b)] = detJ lambda P_cd + detJ mu (delta_cd tr P + P_dc), P = J^{-T} M(a,b) J^{-1},
// M_mn(a,b) = prod over directions of 1D integrals sum_k w_k F(i_a,k) F'(i_b,k), F = G in
// direction m (resp. n) and B otherwise.  One thread per (element, a, b).
// Block K_e[(c, a), (d, b)] (c, d = 0..2) of element e for its local nodes a, b.
template <typename T>
__device__ void coarse_block(const T* __restrict__ ed, const double* __restrict__ tab, int p, int q, int e,
                             const int (&ia)[3], const int (&ib)[3], double (&K)[3][3]) {
    const int D = p + 1;
    const double* w = tab + D + q;
    const double* Bt = w + q;
    const double* Gt = Bt + D * q;
    double M[3][3];
    for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
            double f = 1.0;
            for (int d = 0; d < 3; ++d) {
                const double* Fa = (m == d) ? Gt : Bt;
                const double* Fb = (n == d) ? Gt : Bt;
                double s = 0.0;
                for (int k = 0; k < q; ++k) s += w[k] * Fa[ia[d] * q + k] * Fb[ib[d] * q + k];
                f *= s;
            }
            M[m][n] = f;
        }
    const T* o = ed + (size_t)e * kEdStride;
    double Ji[9];
    for (int k = 0; k < 9; ++k) Ji[k] = (double)o[k];
    double P[3][3];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m)
                for (int n = 0; n < 3; ++n) s += Ji[m * 3 + c] * M[m][n] * Ji[n * 3 + d];
            P[c][d] = s;
        }
    const double tr = P[0][0] + P[1][1] + P[2][2];
    const double lw = (double)o[9], mw = (double)o[10];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) K[c][d] = lw * P[c][d] + mw * ((c == d ? tr : 0.0) + P[d][c]);
}

// One thread per node pair (na, nb): the blocks of the elements containing both, summed
// in a fixed order (deterministic, no atomics); pairs sharing no element get 0.
template <typename T>
__global__ void coarse_assemble_kernel(double* __restrict__ A, int N, const T* __restrict__ ed,
                                       const double* __restrict__ tab, int p, int q, Geom g) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)g.Nn * g.Nn) return;
    const int na = (int)(t / g.Nn), nb = (int)(t % g.Nn);
    const int ax = na % g.Nx, ay = (na / g.Nx) % g.Ny, az = na / (g.Nx * g.Ny);
    const int bx = nb % g.Nx, by = (nb / g.Nx) % g.Ny, bz = nb / (g.Nx * g.Ny);
    double acc[3][3] = {};
    if (abs(ax - bx) <= p && abs(ay - by) <= p && abs(az - bz) <= p) {
        const NodeCands nc = node_candidates(g, p, ax, ay, az);
        for (int kz = 0; kz < 2; ++kz)
            for (int ky = 0; ky < 2; ++ky)
                for (int kx = 0; kx < 2; ++kx) {
                    if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                    const int ex = nc.e[0][kx], ey = nc.e[1][ky], ez = nc.e[2][kz];
                    const int ib[3] = {bx - ex * p, by - ey * p, bz - ez * p};
                    if (ib[0] < 0 || ib[0] > p || ib[1] < 0 || ib[1] > p || ib[2] < 0 || ib[2] > p) continue;
                    const int ia[3] = {nc.l[0][kx], nc.l[1][ky], nc.l[2][kz]};
                    double K[3][3];
                    coarse_block(ed, tab, p, q, ex + g.nx * (ey + g.ny * ez), ia, ib, K);
                    for (int c = 0; c < 3; ++c)
                        for (int d = 0; d < 3; ++d) acc[c][d] += K[c][d];
                }
    }
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) A[(size_t)(c * g.Nn + na) * N + (d * g.Nn + nb)] = acc[c][d];
}

__global__ void coarse_constrain_kernel(double* __restrict__ A, int N, Geom g) {
    GRID_STRIDE(t, (int64_t)N * N) {
        const int i = (int)(t / N), j = (int)(t % N);
        const int ni = i % g.Nn, nj = j % g.Nn;
        const bool ci = clamped_node(g.clamp, ni % g.Nx, (ni / g.Nx) % g.Ny, ni / (g.Nx * g.Ny), g);
        const bool cj = clamped_node(g.clamp, nj % g.Nx, (nj / g.Nx) % g.Ny, nj / (g.Nx * g.Ny), g);
        if (ci || cj) A[t] = (i == j) ? 1.0 : 0.0;
    }
}

// Blocked Gauss-Jordan inversion of the coarse matrix, in place (A becomes A^{-1}),
// kGjNB pivots per block; the constrained coarse matrix is SPD, so no pivoting.  With K
// the indices of a block, P = A[K,K] and Pi = P^{-1}, one block step is the scalar
// elimination step applied to the block of pivots:
//   A[i,j] <- A[i,j] - A[i,K] Pi A[K,j]   (i, j not in K)
//   A[i,K] <- -A[i,K] Pi,   A[K,j] <- Pi A[K,j],   A[K,K] <- Pi.
// Four kernels per block: save the column and row blocks, invert P in one workgroup,
// form the new row block W = Pi A[K,:] (W[:,K] = Pi), then one rank-nb update of A.

// C = A[:, K] (N x nb, row-major), R = A[K, :] (nb x N)
__global__ void gjb_save_kernel(const double* __restrict__ A, double* __restrict__ C, double* __restrict__ R,
                                int N, int k0, int nb) {
    GRID_STRIDE(t, (int64_t)N * nb) {
        const int i = (int)(t / nb), m = (int)(t % nb);
        C[t] = A[(size_t)i * N + k0 + m];
        R[(size_t)m * N + i] = A[(size_t)(k0 + m) * N + i];
    }
}

// Pi = P^{-1} for the nb x nb pivot block P = C[K rows], by scalar Gauss-Jordan in LDS
// (one thread per entry).
__global__ void __launch_bounds__(kGjNB * kGjNB)
gjb_pivot_inverse_kernel(const double* __restrict__ C, double* __restrict__ Pi, int k0, int nb) {
    __shared__ double P[kGjNB][kGjNB + 1];
    __shared__ double colk[kGjNB];
    const int i = threadIdx.y, j = threadIdx.x;
    const bool in = i < nb && j < nb;
    if (in) P[i][j] = C[(size_t)(k0 + i) * nb + j];
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (in && j == 0) colk[i] = P[i][k];
        __syncthreads();
        double v = 0.0;
        if (in) {
            const double piv = colk[k];
            const double akj = (j == k) ? 1.0 / piv : P[k][j] / piv;
            v = (i == k) ? akj : ((j == k) ? 0.0 : P[i][j]) - colk[i] * akj;
        }
        __syncthreads();
        if (in) P[i][j] = v;
        __syncthreads();
    }
    if (in) Pi[i * nb + j] = P[i][j];
}

// W = Pi R (nb x N) with W[:, K] = Pi
__global__ void gjb_rows_kernel(const double* __restrict__ Pi, const double* __restrict__ R, double* __restrict__ W,
                                int N, int k0, int nb) {
    GRID_STRIDE(t, (int64_t)nb * N) {
        const int m = (int)(t / N), j = (int)(t % N);
        double v = 0.0;
        if (j >= k0 && j < k0 + nb) {
            v = Pi[m * nb + (j - k0)];
        } else {
            for (int l = 0; l < nb; ++l) v = fma(Pi[m * nb + l], R[(size_t)l * N + j], v);
        }
        W[t] = v;
    }
}

// Rank-nb update on 64 x 64 tiles (256 threads, 4 x 4 entries each):
//   rows in K:      A[i,j] = W[i - k0, j]
//   other rows:     A[i,j] = (j in K ? 0 : A[i,j]) - sum_m C[i,m] W[m,j]
__global__ void __launch_bounds__(256)
gjb_update_kernel(double* __restrict__ A, const double* __restrict__ C, const double* __restrict__ W, int N, int k0,
                  int nb) {
    __shared__ double Cs[64][kGjNB + 1];
    __shared__ double Ws[kGjNB][64 + 1];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int tid = threadIdx.x;
    for (int t = tid; t < 64 * kGjNB; t += 256) {
        const int r = t / kGjNB, m = t % kGjNB;
        Cs[r][m] = (i0 + r < N && m < nb) ? C[(size_t)(i0 + r) * nb + m] : 0.0;
    }
    for (int t = tid; t < kGjNB * 64; t += 256) {
        const int m = t / 64, c = t % 64;
        Ws[m][c] = (j0 + c < N && m < nb) ? W[(size_t)m * N + j0 + c] : 0.0;
    }
    __syncthreads();
    const int tr = tid / 16, tc = tid % 16;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    // (a partial unroll: the full one hoists every LDS read and spills)
#pragma unroll 4
    for (int m = 0; m < kGjNB; ++m) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Cs[tr + 16 * u][m];
            b[u] = Ws[m][tc + 16 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = i0 + tr + 16 * u;
        if (i >= N) continue;
        const bool iK = i >= k0 && i < k0 + nb;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + tc + 16 * v;
            if (j >= N) continue;
            const size_t o = (size_t)i * N + j;
            if (iK) {
                A[o] = W[(size_t)(i - k0) * N + j];
            } else {
                const bool jK = j >= k0 && j < k0 + nb;
                A[o] = (jK ? 0.0 : A[o]) - acc[u][v];
            }
        }
    }
}

template <typename T>
__global__ void dense_cast_kernel(T* __restrict__ out, const double* __restrict__ in, int64_t n) {
    GRID_STRIDE(i, n) out[i] = (T)in[i];
}

// y = Ainv x (dense, one wavefront per row, FP64 accumulation)
template <typename T>
__global__ void dense_matvec_kernel(const T* __restrict__ Ai, const T* __restrict__ x, T* __restrict__ y, int N) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (row >= N) return;
    double acc = 0.0;
    for (int j = lane; j < N; j += 64) acc += (double)Ai[(size_t)row * N + j] * (double)x[j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) y[row] = (T)acc;
}

}  // namespace

// ============================================================ host launchers

template <typename T> static inline const T* cp(const void* p) { return (const T*)p; }
template <typename T> static inline T* mp(void* p) { return (T*)p; }

#define PA_CHECK_LAUNCH() PA_HIP(hipGetLastError())

int launch_dot(const void* a, const void* b, const void* c, int dtype, int64_t n, double* part, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL((dot_partial_kernel<double, double>), dim3(kReduceBlocks), dim3(kBlock), 0, s,
                           cp<double>(a), cp<double>(b), cp<double>(c), n, part);
    else
        hipLaunchKernelGGL((dot_partial_kernel<float, float>), dim3(kReduceBlocks), dim3(kBlock), 0, s,
                           cp<float>(a), cp<float>(b), cp<float>(c), n, part);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_dot_final(const double* part, double* scal, int op, int slot, hipStream_t s) {
    hipLaunchKernelGGL(dot_final_kernel, dim3(1), dim3(kBlock), 0, s, part, kReduceBlocks, scal, op, slot);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_pcg_init(const double* part, double* scal, double rtol, int stop, hipStream_t s) {
    hipLaunchKernelGGL(pcg_init_scalars_kernel, dim3(1), dim3(kBlock), 0, s, part, kReduceBlocks, scal, rtol, stop);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_power_pass(const void* v, const void* w, const void* dinv, void* z, int dtype, int64_t n, double* part,
                      hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(power_pass_kernel<double>, dim3(kReduceBlocks), dim3(kBlock), 0, s, cp<double>(v),
                           cp<double>(w), cp<double>(dinv), mp<double>(z), n, part);
    else
        hipLaunchKernelGGL(power_pass_kernel<float>, dim3(kReduceBlocks), dim3(kBlock), 0, s, cp<float>(v),
                           cp<float>(w), cp<float>(dinv), mp<float>(z), n, part);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_pcg_xr(void* x, void* r, const void* p, const void* Ap, const double* sc, int dtype, int64_t n,
                  hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(pcg_xr_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(x), mp<double>(r),
                           cp<double>(p), cp<double>(Ap), sc, n);
    else
        hipLaunchKernelGGL(pcg_xr_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(x), mp<float>(r),
                           cp<float>(p), cp<float>(Ap), sc, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_pcg_p(void* p, const void* z, const double* sc, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(pcg_p_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(p), cp<double>(z),
                           sc, n);
    else
        hipLaunchKernelGGL(pcg_p_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(p), cp<float>(z), sc,
                           n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_residual(void* r, const void* b, const void* Ax, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(residual_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(r),
                           cp<double>(b), cp<double>(Ax), n);
    else
        hipLaunchKernelGGL(residual_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(r), cp<float>(b),
                           cp<float>(Ax), n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_copy(void* y, const void* x, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(copy_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(y), cp<double>(x), n);
    else
        hipLaunchKernelGGL(copy_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(y), cp<float>(x), n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_cast_scale(void* y, int dty, const void* x, int dtx, const double* sc, int slot, int inv_sqrt, int64_t n,
                      hipStream_t s) {
    const dim3 g(grid_for(n)), b(kBlock);
    if (dty == PA_F32 && dtx == PA_F64)
        hipLaunchKernelGGL((cast_scale_kernel<float, double>), g, b, 0, s, mp<float>(y), cp<double>(x), sc, slot, inv_sqrt, n);
    else if (dty == PA_F64 && dtx == PA_F64)
        hipLaunchKernelGGL((cast_scale_kernel<double, double>), g, b, 0, s, mp<double>(y), cp<double>(x), sc, slot, inv_sqrt, n);
    else if (dty == PA_F64 && dtx == PA_F32)
        hipLaunchKernelGGL((cast_scale_kernel<double, float>), g, b, 0, s, mp<double>(y), cp<float>(x), sc, slot, inv_sqrt, n);
    else
        hipLaunchKernelGGL((cast_scale_kernel<float, float>), g, b, 0, s, mp<float>(y), cp<float>(x), sc, slot, inv_sqrt, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_ir_update(double* x, const void* d, int dtd, const double* sc, int slot, int64_t n, hipStream_t s) {
    if (dtd == PA_F64)
        hipLaunchKernelGGL(ir_update_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, x, cp<double>(d), sc, slot, n);
    else
        hipLaunchKernelGGL(ir_update_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, x, cp<float>(d), sc, slot, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

template <typename T>
void cheb_step_dispatch(void* x, void* r, const void* t, void* d, const void* dinv, double c1, double c2, bool x_zero,
                        bool last, int64_t n, hipStream_t s) {
    const dim3 g(grid_for(n)), b(kBlock);
    if (x_zero && last)
        hipLaunchKernelGGL((cheb_step_kernel<T, true, true>), g, b, 0, s, mp<T>(x), mp<T>(r), cp<T>(t), mp<T>(d),
                           cp<T>(dinv), c1, c2, n);
    else if (x_zero)
        hipLaunchKernelGGL((cheb_step_kernel<T, true, false>), g, b, 0, s, mp<T>(x), mp<T>(r), cp<T>(t), mp<T>(d),
                           cp<T>(dinv), c1, c2, n);
    else if (last)
        hipLaunchKernelGGL((cheb_step_kernel<T, false, true>), g, b, 0, s, mp<T>(x), mp<T>(r), cp<T>(t), mp<T>(d),
                           cp<T>(dinv), c1, c2, n);
    else
        hipLaunchKernelGGL((cheb_step_kernel<T, false, false>), g, b, 0, s, mp<T>(x), mp<T>(r), cp<T>(t), mp<T>(d),
                           cp<T>(dinv), c1, c2, n);
}

int launch_cheb_step(void* x, void* r, const void* t, void* d, const void* dinv, double c1, double c2, bool x_zero,
                     bool last, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        cheb_step_dispatch<double>(x, r, t, d, dinv, c1, c2, x_zero, last, n, s);
    else
        cheb_step_dispatch<float>(x, r, t, d, dinv, c1, c2, x_zero, last, n, s);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_cheb_start(void* r, void* d, const void* dinv, const void* b, const void* t, double c, int dtype,
                      int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(cheb_start_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(r),
                           mp<double>(d), cp<double>(dinv), cp<double>(b), cp<double>(t), c, n);
    else
        hipLaunchKernelGGL(cheb_start_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(r),
                           mp<float>(d), cp<float>(dinv), cp<float>(b), cp<float>(t), c, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_add(void* y, const void* x, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(add_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(y), cp<double>(x), n);
    else
        hipLaunchKernelGGL(add_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(y), cp<float>(x), n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_reciprocal(void* y, int dtype, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(reciprocal_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(y), n);
    else
        hipLaunchKernelGGL(reciprocal_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(y), n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_splitmix(void* v, int dtype, uint64_t seed, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(splitmix_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(v), seed, n);
    else
        hipLaunchKernelGGL(splitmix_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(v), seed, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_p_interp_matrix(const double* gll_c, const double* gll_f, int pc, int pf, double* I, hipStream_t s) {
    hipLaunchKernelGGL(p_interp_matrix_kernel, dim3(1), dim3(128), 0, s, gll_c, gll_f, pc, pf, I);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

template <int PF, typename T>
void p_prolong_launch(const void* xc, void* xf, const double* I, const Geom& gc, const Geom& gf, int add,
                      hipStream_t s) {
    constexpr int EB = transfer_elems(PF + 1);
    const int nb = (gf.NE + EB - 1) / EB;
    hipLaunchKernelGGL((p_prolong_kernel<PF, T>), dim3(nb), dim3(256), 0, s, cp<T>(xc), mp<T>(xf), I, gc, gf, add);
}

template <int PF, typename T>
void p_restrict_launch(const void* rf, const void* tf, void* rc, void* skr, const double* I, const Geom& gc,
                       const Geom& gf, hipStream_t s) {
    constexpr int EB = transfer_elems(PF + 1);
    const int nb = (gf.NE + EB - 1) / EB;
    hipLaunchKernelGGL((p_restrict_kernel<PF, T>), dim3(nb), dim3(256), 0, s, cp<T>(rf), cp<T>(tf), mp<T>(rc),
                       mp<T>(skr), I, gc, gf);
    hipLaunchKernelGGL((p_restrict_gather_kernel<T>), dim3(grid_for(gc.Nn)), dim3(kBlock), 0, s, mp<T>(rc),
                       cp<T>(skr), PF / 2, gc);
}

#define PA_PF_SWITCH(pf, CALL)                                                                \
    switch (pf) {                                                                             \
        case 2: CALL(2); break;                                                               \
        case 3: CALL(3); break;                                                               \
        case 4: CALL(4); break;                                                               \
        case 5: CALL(5); break;                                                               \
        case 6: CALL(6); break;                                                               \
        case 7: CALL(7); break;                                                               \
        case 8: CALL(8); break;                                                               \
        default: return fail(PA_EUNSUPPORTED, "p-transfer from degree %d is not built", pf); \
    }

int launch_p_prolong(const void* xc, void* xf, const double* I, int pc, int pf, const Geom& gc, const Geom& gf,
                     int add, int dtype, hipStream_t s) {
    if (pc != pf / 2) return fail(PA_EUNSUPPORTED, "p-transfer %d -> %d: the coarse degree must be %d", pf, pc, pf / 2);
#define PA_PROLONG(PF)                                                   \
    if (dtype == PA_F64) p_prolong_launch<PF, double>(xc, xf, I, gc, gf, add, s); \
    else p_prolong_launch<PF, float>(xc, xf, I, gc, gf, add, s)
    PA_PF_SWITCH(pf, PA_PROLONG)
#undef PA_PROLONG
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_p_restrict(const void* rf, const void* tf, void* rc, void* skr, const double* I, int pc, int pf,
                      const Geom& gc, const Geom& gf, int dtype, hipStream_t s) {
    if (pc != pf / 2) return fail(PA_EUNSUPPORTED, "p-transfer %d -> %d: the coarse degree must be %d", pf, pc, pf / 2);
#define PA_RESTRICT(PF)                                                              \
    if (dtype == PA_F64) p_restrict_launch<PF, double>(rf, tf, rc, skr, I, gc, gf, s); \
    else p_restrict_launch<PF, float>(rf, tf, rc, skr, I, gc, gf, s)
    PA_PF_SWITCH(pf, PA_RESTRICT)
#undef PA_RESTRICT
    PA_CHECK_LAUNCH();
    return PA_OK;
}
#undef PA_PF_SWITCH

int launch_h_prolong(const void* xc, void* xf, const HAxis ax[3], const Geom& gc, const Geom& gf, int add, int dtype,
                     hipStream_t s) {
    const int g = grid_for(gf.Nn);
    if (dtype == PA_F64)
        hipLaunchKernelGGL(h_prolong_kernel<double>, dim3(g), dim3(kBlock), 0, s, cp<double>(xc), mp<double>(xf), ax[0],
                           ax[1], ax[2], gc, gf, add);
    else
        hipLaunchKernelGGL(h_prolong_kernel<float>, dim3(g), dim3(kBlock), 0, s, cp<float>(xc), mp<float>(xf), ax[0],
                           ax[1], ax[2], gc, gf, add);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_h_restrict(const void* rf, const void* tf, void* rc, const HAxis ax[3], const Geom& gc, const Geom& gf, int dtype,
                      hipStream_t s) {
    // 64-lane groups: the coarse levels are small, spread them over more CUs
    const int g = (int)((3 * (int64_t)gc.Nn + 63) / 64);
    if (dtype == PA_F64)
        hipLaunchKernelGGL(h_restrict_kernel<double>, dim3(g), dim3(64), 0, s, cp<double>(rf), cp<double>(tf), mp<double>(rc),
                           ax[0], ax[1], ax[2], gc, gf);
    else
        hipLaunchKernelGGL(h_restrict_kernel<float>, dim3(g), dim3(64), 0, s, cp<float>(rf), cp<float>(tf), mp<float>(rc), ax[0],
                           ax[1], ax[2], gc, gf);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_coarse_assemble(double* A, int N, const pa_op* op, hipStream_t s) {
    const Geom g = make_geom(op->mesh, op->p, true);
    const long long work = (long long)g.Nn * g.Nn;
    const int nb = (int)((work + 255) / 256);
    if (op->dtype == PA_F64)
        hipLaunchKernelGGL(coarse_assemble_kernel<double>, dim3(nb), dim3(256), 0, s, A, N, cp<double>(op->ed),
                           op->d_tab, op->p, op->q, g);
    else
        hipLaunchKernelGGL(coarse_assemble_kernel<float>, dim3(nb), dim3(256), 0, s, A, N, cp<float>(op->ed),
                           op->d_tab, op->p, op->q, g);
    PA_CHECK_LAUNCH();
    hipLaunchKernelGGL(coarse_constrain_kernel, dim3(grid_for((int64_t)N * N)), dim3(kBlock), 0, s, A, N, g);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int64_t coarse_invert_words(int N) { return 3 * (int64_t)N * kGjNB + (int64_t)kGjNB * kGjNB; }

int coarse_invert(double* A, double* work, int N, hipStream_t s) {
    double* C = work;
    double* R = C + (size_t)N * kGjNB;
    double* W = R + (size_t)N * kGjNB;
    double* Pi = W + (size_t)N * kGjNB;
    const dim3 gu((N + 63) / 64, (N + 63) / 64);
    for (int k0 = 0; k0 < N; k0 += kGjNB) {
        const int nb = N - k0 < kGjNB ? N - k0 : kGjNB;
        hipLaunchKernelGGL(gjb_save_kernel, dim3(grid_for((int64_t)N * nb)), dim3(kBlock), 0, s, A, C, R, N, k0, nb);
        hipLaunchKernelGGL(gjb_pivot_inverse_kernel, dim3(1), dim3(kGjNB, kGjNB), 0, s, C, Pi, k0, nb);
        hipLaunchKernelGGL(gjb_rows_kernel, dim3(grid_for((int64_t)nb * N)), dim3(kBlock), 0, s, Pi, R, W, N, k0, nb);
        hipLaunchKernelGGL(gjb_update_kernel, gu, dim3(256), 0, s, A, C, W, N, k0, nb);
    }
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_dense_cast(void* out, int dtype, const double* in, int64_t n, hipStream_t s) {
    if (dtype == PA_F64)
        hipLaunchKernelGGL(dense_cast_kernel<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<double>(out), in, n);
    else
        hipLaunchKernelGGL(dense_cast_kernel<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, mp<float>(out), in, n);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

int launch_dense_matvec(const void* Ai, const void* x, void* y, int N, int dtype, hipStream_t s) {
    const int rows_per_block = 4;
    const int nb = (N + rows_per_block - 1) / rows_per_block;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(dense_matvec_kernel<double>, dim3(nb), dim3(64 * rows_per_block), 0, s, cp<double>(Ai),
                           cp<double>(x), mp<double>(y), N);
    else
        hipLaunchKernelGGL(dense_matvec_kernel<float>, dim3(nb), dim3(64 * rows_per_block), 0, s, cp<float>(Ai),
                           cp<float>(x), mp<float>(y), N);
    PA_CHECK_LAUNCH();
    return PA_OK;
}

}  // namespace pa
