// Device-side setup of the partial assembly: 1D tables, per-element PA data,
// the operator diagonal and the load vector.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "internal.h"
#include "kernels.h"

namespace pa {

// ---------------------------------------------------------------------------
// 1D tables (Sec. 4.4: B(D1D,Q1D), G(D1D,Q1D) on (p+1) Gauss-Lobatto nodes and
// (p+2) Gauss-Legendre points; any q >= p+1 is accepted).
// Layout of the FP64 device buffer:
//   gll[D] | xq[Q] | w[Q] | B[D*Q] | G[D*Q] | bb[D] | bg[D] | gg[D] | sB[D]
// with bb[i] = sum_k w_k B_ik^2, bg[i] = sum_k w_k B_ik G_ik, gg[i] = sum_k w_k G_ik^2,
// sB[i] = sum_k w_k B_ik (1D integrals used by the diagonal and the load vector).
// ---------------------------------------------------------------------------

// P_n(x) and P_{n-1}(x) by the three-term recurrence.
__device__ static void legendre_pair(int n, double x, double& pn, double& pn1) {
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2.0 * k - 1.0) * x * b - (k - 1.0) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pn1 = a;
}

__global__ void tables_kernel(int p, int q, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int D = p + 1, Q = q;
    double* gll = out;
    double* xq = gll + D;
    double* w = xq + Q;
    double* B = w + Q;
    double* G = B + D * Q;
    double* bb = G + D * Q;
    double* bg = bb + D;
    double* gg = bg + D;
    double* sB = gg + D;
    const double pi = 3.14159265358979323846;
    // Gauss-Legendre: Newton on P_q from x = -cos(pi (k+3/4)/(q+1/2)); w = 2/((1-x^2) P_q'^2)
    for (int k = 0; k < Q; ++k) {
        double x = -cos(pi * (k + 0.75) / (Q + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            legendre_pair(Q, x, pn, pn1);
            dp = Q * (x * pn - pn1) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double pn, pn1;
        legendre_pair(Q, x, pn, pn1);
        dp = Q * (x * pn - pn1) / (x * x - 1.0);
        xq[k] = 0.5 * (x + 1.0);
        w[k] = 1.0 / ((1.0 - x * x) * dp * dp);   // (2/((1-x^2)P'^2)) / 2
    }
    // Gauss-Lobatto: end points and the roots of P_p', Newton from -cos(pi j/p)
    gll[0] = 0.0;
    gll[p] = 1.0;
    for (int j = 1; j < p; ++j) {
        double x = -cos(pi * j / p);
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            legendre_pair(p, x, pn, pn1);
            double d1 = p * (x * pn - pn1) / (x * x - 1.0);               // P_p'
            double d2 = (2.0 * x * d1 - p * (p + 1.0) * pn) / (1.0 - x * x); // P_p''
            double dx = d1 / d2;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        gll[j] = 0.5 * (x + 1.0);
    }
    // Lagrange values and derivatives at the quadrature points (product rule)
    for (int i = 0; i < D; ++i) {
        double s_bb = 0, s_bg = 0, s_gg = 0, s_b = 0;
        for (int k = 0; k < Q; ++k) {
            const double x = xq[k];
            double v = 1.0, dv = 0.0;
            for (int j = 0; j < D; ++j)
                if (j != i) v *= (x - gll[j]) / (gll[i] - gll[j]);
            for (int m = 0; m < D; ++m) {
                if (m == i) continue;
                double t = 1.0 / (gll[i] - gll[m]);
                for (int j = 0; j < D; ++j)
                    if (j != i && j != m) t *= (x - gll[j]) / (gll[i] - gll[j]);
                dv += t;
            }
            B[i * Q + k] = v;
            G[i * Q + k] = dv;
            s_bb += w[k] * v * v;
            s_bg += w[k] * v * dv;
            s_gg += w[k] * dv * dv;
            s_b += w[k] * v;
        }
        bb[i] = s_bb;
        bg[i] = s_bg;
        gg[i] = s_gg;
        sB[i] = s_b;
    }
}

int tables_words(int p, int q) { return 2 * (p + 1) * q + 2 * q + 5 * (p + 1); }

// The tables depend on (p, q) only: the first operator of a (p, q) computes them on the
// device, later ones (solver levels, served requests) copy the kept words.
struct TableWords {
    Tables host;
    std::vector<double> words;
};
static std::mutex g_tables_mu;
static std::map<std::pair<int, int>, TableWords> g_tables;

int compute_tables(int p, int q, hipStream_t s, double** d_tab, Tables* host) {
    const int n = tables_words(p, q);
    double* d = nullptr;
    PA_HIP(hipMalloc(&d, n * sizeof(double)));
    {
        std::lock_guard<std::mutex> lk(g_tables_mu);
        const auto it = g_tables.find({p, q});
        if (it != g_tables.end()) {
            const hipError_t e = hipMemcpyAsync(d, it->second.words.data(), n * sizeof(double),
                                                hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                (void)hipFree(d);
                return fail(PA_EHIP, "1D table upload failed: %s", hipGetErrorString(e));
            }
            *host = it->second.host;
            *d_tab = d;
            return PA_OK;
        }
    }
    hipLaunchKernelGGL(tables_kernel, dim3(1), dim3(64), 0, s, p, q, d);
    hipError_t e = hipGetLastError();
    std::vector<double> h(n);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(PA_EHIP, "1D table kernel failed: %s", hipGetErrorString(e));
    }
    const int D = p + 1, Q = q;
    host->p = p;
    host->q = q;
    for (int i = 0; i < D; ++i) host->gll[i] = h[i];
    for (int k = 0; k < Q; ++k) { host->xq[k] = h[D + k]; host->w[k] = h[D + Q + k]; }
    for (int i = 0; i < D * Q; ++i) {
        host->B[i] = h[D + 2 * Q + i];
        host->G[i] = h[D + 2 * Q + D * Q + i];
    }
    *d_tab = d;
    {
        std::lock_guard<std::mutex> lk(g_tables_mu);
        g_tables.emplace(std::make_pair(p, q), TableWords{*host, std::move(h)});
    }
    return PA_OK;
}

// ---------------------------------------------------------------------------
// Per-element PA data (Sec. 4.4: J^{-1} and det J constant per affine element):
//   ed[e][m*3+i] = (J^{-1})_{m,i},  ed[e][9] = det J * lambda_e,  ed[e][10] = det J * mu_e
// with J_e = A diag(h_x, h_y, h_z), so J^{-1} = diag(1/h) A^{-1}.
// ---------------------------------------------------------------------------
struct Mat3 { double a[9]; };

template <typename T>
__global__ void element_data_kernel(T* __restrict__ ed, const double* __restrict__ vert,
                                    const double* __restrict__ lam, const double* __restrict__ mu,
                                    Mat3 A, int nx, int ny, int nz) {
    const int NE = nx * ny * nz;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NE) return;
    const int ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
    const double* vx = vert;
    const double* vy = vx + nx + 1;
    const double* vz = vy + ny + 1;
    const double h[3] = {vx[ex + 1] - vx[ex], vy[ey + 1] - vy[ey], vz[ez + 1] - vz[ez]};
    const double* a = A.a;
    // adjugate / determinant of A (row-major)
    double c[9];
    c[0] = a[4] * a[8] - a[5] * a[7];
    c[1] = a[2] * a[7] - a[1] * a[8];
    c[2] = a[1] * a[5] - a[2] * a[4];
    c[3] = a[5] * a[6] - a[3] * a[8];
    c[4] = a[0] * a[8] - a[2] * a[6];
    c[5] = a[2] * a[3] - a[0] * a[5];
    c[6] = a[3] * a[7] - a[4] * a[6];
    c[7] = a[1] * a[6] - a[0] * a[7];
    c[8] = a[0] * a[4] - a[1] * a[3];
    const double det = a[0] * c[0] + a[1] * c[3] + a[2] * c[6];
    T* o = ed + (size_t)e * kEdStride;
    for (int m = 0; m < 3; ++m)
        for (int i = 0; i < 3; ++i) o[m * 3 + i] = (T)(c[m * 3 + i] / (det * h[m]));
    const double detJ = det * h[0] * h[1] * h[2];
    o[9] = (T)(detJ * lam[e]);
    o[10] = (T)(detJ * mu[e]);
    o[11] = (T)0;
}

int compute_element_data(const MeshDesc& m, const double* d_vert, const double* d_lam, const double* d_mu,
                         int dtype, void* ed, hipStream_t s) {
    Mat3 A;
    for (int i = 0; i < 9; ++i) A.a[i] = m.A[i];
    const int NE = m.n[0] * m.n[1] * m.n[2];
    const int nb = (NE + 255) / 256;
    if (dtype == PA_F64)
        hipLaunchKernelGGL(element_data_kernel<double>, dim3(nb), dim3(256), 0, s, (double*)ed, d_vert, d_lam,
                           d_mu, A, m.n[0], m.n[1], m.n[2]);
    else
        hipLaunchKernelGGL(element_data_kernel<float>, dim3(nb), dim3(256), 0, s, (float*)ed, d_vert, d_lam,
                           d_mu, A, m.n[0], m.n[1], m.n[2]);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

// ---------------------------------------------------------------------------
// Diagonal of A (Sec. 3.1 Jacobi diagonal).  For local node a = (ix,iy,iz):
//   M_mn(a) = sum_alpha w_alpha dref_m phi_a dref_n phi_a = prod_d f_d,
//   f_d = gg[i_d] if m==n==d, bg[i_d] if exactly one of m,n is d, else bb[i_d];
//   P = J^{-T} M J^{-1} (P_cd = int d_c phi_a d_d phi_a / det J);
//   diag(c,a) += detJ*lambda P_cc + detJ*mu (tr P + P_cc).
// ---------------------------------------------------------------------------
// Contribution of element e to the diagonal at its local node (ix, iy, iz), component c.
template <typename T>
__device__ __forceinline__ void diagonal_part(const T* __restrict__ ed, const double* __restrict__ tab, int D, int q,
                                              int e, int ix, int iy, int iz, double (&out)[3]) {
    const double* bb = tab + D + 2 * q + 2 * D * q;
    const double* bg = bb + D;
    const double* gg = bg + D;
    const int idx[3] = {ix, iy, iz};
    double M[3][3];
    for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
            double f = 1.0;
            for (int d = 0; d < 3; ++d) {
                const int i = idx[d];
                f *= (m == d && n == d) ? gg[i] : ((m == d || n == d) ? bg[i] : bb[i]);
            }
            M[m][n] = f;
        }
    const T* o = ed + (size_t)e * kEdStride;
    double Ji[9];
    for (int k = 0; k < 9; ++k) Ji[k] = (double)o[k];
    double P[3];
    double tr = 0.0;
    for (int c = 0; c < 3; ++c) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m)
            for (int n = 0; n < 3; ++n) s += Ji[m * 3 + c] * M[m][n] * Ji[n * 3 + c];
        P[c] = s;
        tr += s;
    }
    const double lw = (double)o[9], mw = (double)o[10];
    for (int c = 0; c < 3; ++c) out[c] = lw * P[c] + mw * (tr + P[c]);
}

// One thread per node: the contributions of its elements summed in a fixed order.
template <typename T>
__global__ void diagonal_kernel(T* __restrict__ dg, const T* __restrict__ ed, const double* __restrict__ tab,
                                int p, int q, Geom g) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.Nn) return;
    const int gx = node % g.Nx, gy = (node / g.Nx) % g.Ny, gz = node / (g.Nx * g.Ny);
    const NodeCands nc = node_candidates(g, p, gx, gy, gz);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int kz = 0; kz < 2; ++kz)
        for (int ky = 0; ky < 2; ++ky)
            for (int kx = 0; kx < 2; ++kx) {
                if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                const int e = nc.e[0][kx] + g.nx * (nc.e[1][ky] + g.ny * nc.e[2][kz]);
                double part[3];
                diagonal_part(ed, tab, p + 1, q, e, nc.l[0][kx], nc.l[1][ky], nc.l[2][kz], part);
                for (int c = 0; c < 3; ++c) acc[c] += part[c];
            }
    for (int c = 0; c < 3; ++c) dg[(size_t)c * g.Nn + node] = (T)acc[c];
}

// Per-point Lame parameters: the quadrature sum of the diagonal entry written out,
//   diag(c, a) += sum_alpha w_alpha detJ [lambda_alpha g_c^2 + mu_alpha (|g|^2 + g_c^2)],
//   g = J^{-T} grad_ref phi_a(alpha), grad_ref phi_a = (G_x B_y B_z, B_x G_y B_z, B_x B_y G_z),
// with md word k of point alpha of element e at md_word(e, alpha, k) (element-major
// [NE][q^3][2], or point-major [2 q^3][NE] for the linear-element kernel's layout).
template <typename T>
__device__ __forceinline__ void diagonal_part_qp(const T* __restrict__ ed, const T* __restrict__ md, bool pm,
                                                 int NE, const double* __restrict__ tab, int D, int q, int e, int ix,
                                                 int iy, int iz, double (&out)[3]) {
    const double* w = tab + D + q;
    const double* B = w + q;
    const double* G = B + D * q;
    const T* o = ed + (size_t)e * kEdStride;
    double Ji[9];
    for (int k = 0; k < 9; ++k) Ji[k] = (double)o[k];
    const double detJ = (double)o[9];   // unit Lame parameters in the element data
    const int Q3 = q * q * q;
    out[0] = out[1] = out[2] = 0.0;
    for (int qz = 0; qz < q; ++qz) {
        const double bz = B[iz * q + qz], gz = G[iz * q + qz];
        for (int qy = 0; qy < q; ++qy) {
            const double by = B[iy * q + qy], gy = G[iy * q + qy];
            for (int qx = 0; qx < q; ++qx) {
                const double bx = B[ix * q + qx], gx = G[ix * q + qx];
                const double r[3] = {gx * by * bz, bx * gy * bz, bx * by * gz};
                double gr[3];
                for (int c = 0; c < 3; ++c) gr[c] = Ji[c] * r[0] + Ji[3 + c] * r[1] + Ji[6 + c] * r[2];
                const int al = qx + q * (qy + q * qz);
                const size_t i0 = pm ? (size_t)(2 * al) * NE + e : ((size_t)e * Q3 + al) * 2;
                const size_t i1 = pm ? i0 + (size_t)NE : i0 + 1;
                const double W = w[qx] * w[qy] * w[qz] * detJ;
                const double lam = (double)md[i0], mu = (double)md[i1];
                const double n2 = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
                for (int c = 0; c < 3; ++c) out[c] += W * (lam * gr[c] * gr[c] + mu * (n2 + gr[c] * gr[c]));
            }
        }
    }
}

// Per-element anisotropic Voigt stiffness C (md = [NE][21], upper triangle row by row):
// a unit displacement in direction c at node a has the engineering strain S_c g with
// g = grad phi_a, so diag(c, a) = sum_ij C[v_c(i)][v_c(j)] int d_i phi_a d_j phi_a, where
// v_c(i) is the Voigt row of strain component d_i u_c: v_0 = (0, 5, 4), v_1 = (5, 1, 3),
// v_2 = (4, 3, 2); the integrals come from the 1D-factorized M as in diagonal_part.
template <typename T>
__device__ __forceinline__ void diagonal_part_aniso(const T* __restrict__ ed, const T* __restrict__ md,
                                                    const double* __restrict__ tab, int D, int q, int e, int ix,
                                                    int iy, int iz, double (&out)[3]) {
    const double* bb = tab + D + 2 * q + 2 * D * q;
    const double* bg = bb + D;
    const double* gg = bg + D;
    const int idx[3] = {ix, iy, iz};
    double M[3][3];
    for (int m = 0; m < 3; ++m)
        for (int n = 0; n < 3; ++n) {
            double f = 1.0;
            for (int d = 0; d < 3; ++d) {
                const int i = idx[d];
                f *= (m == d && n == d) ? gg[i] : ((m == d || n == d) ? bg[i] : bb[i]);
            }
            M[m][n] = f;
        }
    const T* o = ed + (size_t)e * kEdStride;
    double Ji[9];
    for (int k = 0; k < 9; ++k) Ji[k] = (double)o[k];
    double P[3][3];   // int d_i phi_a d_j phi_a / det J
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m)
                for (int n = 0; n < 3; ++n) s += Ji[m * 3 + i] * M[m][n] * Ji[n * 3 + j];
            P[i][j] = s;
        }
    const T* c = md + (size_t)e * 21;
    auto C = [&](int a, int b) -> double {
        const int lo = a < b ? a : b, hi = a < b ? b : a;
        return (double)c[lo * 6 - lo * (lo - 1) / 2 + (hi - lo)];
    };
    constexpr int v[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
    const double detJ = (double)o[9];   // unit Lame parameters in the element data
    for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) s += C(v[k][i], v[k][j]) * P[i][j];
        out[k] = detJ * s;
    }
}

template <typename T>
__global__ void diagonal_aniso_kernel(T* __restrict__ dg, const T* __restrict__ ed, const T* __restrict__ md,
                                      const double* __restrict__ tab, int p, int q, Geom g) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.Nn) return;
    const int gx = node % g.Nx, gy = (node / g.Nx) % g.Ny, gz = node / (g.Nx * g.Ny);
    const NodeCands nc = node_candidates(g, p, gx, gy, gz);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int kz = 0; kz < 2; ++kz)
        for (int ky = 0; ky < 2; ++ky)
            for (int kx = 0; kx < 2; ++kx) {
                if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                const int e = nc.e[0][kx] + g.nx * (nc.e[1][ky] + g.ny * nc.e[2][kz]);
                double part[3];
                diagonal_part_aniso(ed, md, tab, p + 1, q, e, nc.l[0][kx], nc.l[1][ky], nc.l[2][kz], part);
                for (int c = 0; c < 3; ++c) acc[c] += part[c];
            }
    for (int c = 0; c < 3; ++c) dg[(size_t)c * g.Nn + node] = (T)acc[c];
}

template <typename T>
__global__ void diagonal_qp_kernel(T* __restrict__ dg, const T* __restrict__ ed, const T* __restrict__ md, int pm,
                                   const double* __restrict__ tab, int p, int q, Geom g) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.Nn) return;
    const int gx = node % g.Nx, gy = (node / g.Nx) % g.Ny, gz = node / (g.Nx * g.Ny);
    const NodeCands nc = node_candidates(g, p, gx, gy, gz);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int kz = 0; kz < 2; ++kz)
        for (int ky = 0; ky < 2; ++ky)
            for (int kx = 0; kx < 2; ++kx) {
                if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                const int e = nc.e[0][kx] + g.nx * (nc.e[1][ky] + g.ny * nc.e[2][kz]);
                double part[3];
                diagonal_part_qp(ed, md, pm != 0, g.NE, tab, p + 1, q, e, nc.l[0][kx], nc.l[1][ky], nc.l[2][kz],
                                 part);
                for (int c = 0; c < 3; ++c) acc[c] += part[c];
            }
    for (int c = 0; c < 3; ++c) dg[(size_t)c * g.Nn + node] = (T)acc[c];
}

int launch_diagonal(const pa_op* op, void* d, int constrained) {
    if (op->geo != PA_GEOM_AFFINE) return fail(PA_EUNSUPPORTED, "diagonal of non-affine geometry is not built");
    const Geom g = make_geom(op->mesh, op->p, constrained != 0);
    const int nb = (g.Nn + 255) / 256;
    if (op->mat == PA_MAT_ANISO) {
        if (op->dtype == PA_F64)
            hipLaunchKernelGGL(diagonal_aniso_kernel<double>, dim3(nb), dim3(256), 0, op->stream, (double*)d,
                               (const double*)op->ed, (const double*)op->md, op->d_tab, op->p, op->q, g);
        else
            hipLaunchKernelGGL(diagonal_aniso_kernel<float>, dim3(nb), dim3(256), 0, op->stream, (float*)d,
                               (const float*)op->ed, (const float*)op->md, op->d_tab, op->p, op->q, g);
    } else if (op->mat == PA_MAT_QP_ISO) {
        const int pm = op->md_point_major ? 1 : 0;
        if (op->dtype == PA_F64)
            hipLaunchKernelGGL(diagonal_qp_kernel<double>, dim3(nb), dim3(256), 0, op->stream, (double*)d,
                               (const double*)op->ed, (const double*)op->md, pm, op->d_tab, op->p, op->q, g);
        else
            hipLaunchKernelGGL(diagonal_qp_kernel<float>, dim3(nb), dim3(256), 0, op->stream, (float*)d,
                               (const float*)op->ed, (const float*)op->md, pm, op->d_tab, op->p, op->q, g);
    } else if (op->dtype == PA_F64)
        hipLaunchKernelGGL(diagonal_kernel<double>, dim3(nb), dim3(256), 0, op->stream, (double*)d,
                           (const double*)op->ed, op->d_tab, op->p, op->q, g);
    else
        hipLaunchKernelGGL(diagonal_kernel<float>, dim3(nb), dim3(256), 0, op->stream, (float*)d,
                           (const float*)op->ed, op->d_tab, op->p, op->q, g);
    PA_HIP(hipGetLastError());
    if (constrained && g.clamp) return launch_set_clamped(d, op->dtype, g, 1.0, op->stream);
    return PA_OK;
}

// ---------------------------------------------------------------------------
// Load vector of eq. 4 for a constant body force f and a constant traction t on
// one box face.  Volume: int phi_a = detJ sB[ix] sB[iy] sB[iz].  Face x=const
// (similarly y, z): int phi_a dGamma = |J e_t1 x J e_t2| sB[i_t1] sB[i_t2] for
// nodes on the face (l_i at the end point is 1 for the end node, 0 otherwise).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rhs_part(const double* __restrict__ vert, const double* __restrict__ tab,
                                         const Mat3& A, int p, int q, const Geom& g, int ex, int ey, int ez,
                                         const int (&idx)[3], const double (&f)[3], int face, const double (&t)[3],
                                         double (&out)[3]) {
    const int D = p + 1;
    const int epos[3] = {ex, ey, ez};
    const int nel[3] = {g.nx, g.ny, g.nz};
    const double* vx = vert;
    const double* vy = vx + g.nx + 1;
    const double* vz = vy + g.ny + 1;
    const double h[3] = {vx[ex + 1] - vx[ex], vy[ey + 1] - vy[ey], vz[ez + 1] - vz[ez]};
    const double* sB = tab + D + 2 * q + 2 * D * q + 3 * D;
    const double* a9 = A.a;
    const double detA = a9[0] * (a9[4] * a9[8] - a9[5] * a9[7]) - a9[1] * (a9[3] * a9[8] - a9[5] * a9[6]) +
                        a9[2] * (a9[3] * a9[7] - a9[4] * a9[6]);
    const double vol = detA * h[0] * h[1] * h[2] * sB[idx[0]] * sB[idx[1]] * sB[idx[2]];
    for (int c = 0; c < 3; ++c) out[c] = f[c] * vol;
    if (face >= 0) {
        const int ax = face / 2, side = face % 2;
        const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
        const bool on = (side == 0) ? (epos[ax] == 0 && idx[ax] == 0) : (epos[ax] == nel[ax] - 1 && idx[ax] == p);
        if (on) {
            // |A e_t1 x A e_t2| h_t1 h_t2
            const double u0 = a9[0 * 3 + t1], u1 = a9[1 * 3 + t1], u2 = a9[2 * 3 + t1];
            const double v0 = a9[0 * 3 + t2], v1 = a9[1 * 3 + t2], v2 = a9[2 * 3 + t2];
            const double cx = u1 * v2 - u2 * v1, cy = u2 * v0 - u0 * v2, cz = u0 * v1 - u1 * v0;
            const double area = sqrt(cx * cx + cy * cy + cz * cz) * h[t1] * h[t2] * sB[idx[t1]] * sB[idx[t2]];
            for (int c = 0; c < 3; ++c) out[c] += t[c] * area;
        }
    }
}

// One thread per node: the contributions of its elements summed in a fixed order;
// clamped nodes get 0.
__global__ void rhs_kernel(double* __restrict__ b, const double* __restrict__ vert, const double* __restrict__ tab,
                           Mat3 A, int p, int q, Geom g, double fx, double fy, double fz, int face, double tx,
                           double ty, double tz) {
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= g.Nn) return;
    const int gx = node % g.Nx, gy = (node / g.Nx) % g.Ny, gz = node / (g.Nx * g.Ny);
    double acc[3] = {0.0, 0.0, 0.0};
    if (!clamped_node(g.clamp, gx, gy, gz, g)) {
        const NodeCands nc = node_candidates(g, p, gx, gy, gz);
        const double f[3] = {fx, fy, fz}, t[3] = {tx, ty, tz};
        for (int kz = 0; kz < 2; ++kz)
            for (int ky = 0; ky < 2; ++ky)
                for (int kx = 0; kx < 2; ++kx) {
                    if (!(nc.v[0][kx] && nc.v[1][ky] && nc.v[2][kz])) continue;
                    const int idx[3] = {nc.l[0][kx], nc.l[1][ky], nc.l[2][kz]};
                    double part[3];
                    rhs_part(vert, tab, A, p, q, g, nc.e[0][kx], nc.e[1][ky], nc.e[2][kz], idx, f, face, t, part);
                    for (int c = 0; c < 3; ++c) acc[c] += part[c];
                }
    }
    for (int c = 0; c < 3; ++c) b[(size_t)c * g.Nn + node] = acc[c];
}

int launch_rhs(const pa_op* op, const double f[3], int face, const double t[3], double* b, const double* d_vert) {
    const Geom g = make_geom(op->mesh, op->p, true);
    Mat3 A;
    for (int i = 0; i < 9; ++i) A.a[i] = op->mesh.A[i];
    const int nb = (g.Nn + 255) / 256;
    const double tt[3] = {t ? t[0] : 0.0, t ? t[1] : 0.0, t ? t[2] : 0.0};
    hipLaunchKernelGGL(rhs_kernel, dim3(nb), dim3(256), 0, op->stream, b, d_vert, op->d_tab, A, op->p, op->q, g,
                       f ? f[0] : 0.0, f ? f[1] : 0.0, f ? f[2] : 0.0, face, tt[0], tt[1], tt[2]);
    PA_HIP(hipGetLastError());
    return PA_OK;
}

}  // namespace pa
