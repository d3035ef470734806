// Non-affine (trilinear) element geometry: the per-element map coefficients, the
// per-quadrature-point data of the stored form, the positivity check of det J and
// the C entry point pa_elast_setup_geometry.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace pa {
namespace {

struct QRule {
    double x[kMaxQ];
    double w[kMaxQ];
};

// One thread per element.  The trilinear map through the vertices X_abc is
//   x(xi, eta, zeta) = x0 + a xi + b eta + c zeta + d xi eta + e xi zeta + f eta zeta + g xi eta zeta,
// coef[e] = (a, b, c, d, e, f, g), 3 words each.  At every Gauss-Legendre point the
// thread forms J = dx/dxi, records the smallest det J of the element and, for the
// stored form (gd != nullptr), writes gd[e][w][alpha]: w = m*3+i -> (J^{-1})_{m,i},
// w = 9 -> w_alpha det J, alpha = qx + Q (qy + Q qz).
template <typename T>
__global__ void geometry_qp_kernel(const double* __restrict__ coef, const QRule r, const int Q, const int NE,
                                   T* __restrict__ gd, double* __restrict__ min_det) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NE) return;
    const double* c = coef + (size_t)e * 21;
    const int Q3 = Q * Q * Q;
    double mn = HUGE_VAL;
    for (int kz = 0; kz < Q; ++kz)
        for (int ky = 0; ky < Q; ++ky)
            for (int kx = 0; kx < Q; ++kx) {
                const double xi = r.x[kx], eta = r.x[ky], zeta = r.x[kz];
                double J[3][3];
                for (int i = 0; i < 3; ++i) {
                    J[i][0] = c[i] + c[9 + i] * eta + c[12 + i] * zeta + c[18 + i] * eta * zeta;
                    J[i][1] = c[3 + i] + c[9 + i] * xi + c[15 + i] * zeta + c[18 + i] * xi * zeta;
                    J[i][2] = c[6 + i] + c[12 + i] * xi + c[15 + i] * eta + c[18 + i] * xi * eta;
                }
                double adj[9];   // adj[m][i] = cofactor of J[i][m]
                adj[0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
                adj[1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
                adj[2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
                adj[3] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
                adj[4] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
                adj[5] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
                adj[6] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
                adj[7] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
                adj[8] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
                const double det = J[0][0] * adj[0] + J[0][1] * adj[3] + J[0][2] * adj[6];
                mn = det < mn ? det : mn;
                if (gd) {
                    T* o = gd + (size_t)e * 10 * Q3 + kx + Q * (ky + Q * kz);
                    for (int w = 0; w < 9; ++w) o[w * Q3] = (T)(adj[w] / det);
                    o[9 * Q3] = (T)(r.w[kx] * r.w[ky] * r.w[kz] * det);
                }
            }
    min_det[e] = mn;
}

}  // namespace

// The 21 map coefficients of one element from its corner positions X[a + 2(b + 2c)].
void element_map_coefficients(const double* const X[8], double* o) {
    for (int d = 0; d < 3; ++d) {
        const double x000 = X[0][d], x100 = X[1][d], x010 = X[2][d], x110 = X[3][d];
        const double x001 = X[4][d], x101 = X[5][d], x011 = X[6][d], x111 = X[7][d];
        o[d] = x100 - x000;                                                  // a
        o[3 + d] = x010 - x000;                                              // b
        o[6 + d] = x001 - x000;                                              // c
        o[9 + d] = x110 - x100 - x010 + x000;                                // d
        o[12 + d] = x101 - x100 - x001 + x000;                               // e
        o[15 + d] = x011 - x010 - x001 + x000;                               // f
        o[18 + d] = x111 - x110 - x101 - x011 + x100 + x010 + x001 - x000;   // g
    }
}

namespace {

// Map coefficients of every element of the box from the vertex array (host, FP64).
void map_coefficients(const int n[3], const double* v, std::vector<double>& coef) {
    const int64_t NE = (int64_t)n[0] * n[1] * n[2];
    coef.resize((size_t)NE * 21);
    const int64_t sx = 1, sy = n[0] + 1, sz = (int64_t)(n[0] + 1) * (n[1] + 1);
    for (int64_t e = 0; e < NE; ++e) {
        const int64_t ex = e % n[0], ey = (e / n[0]) % n[1], ez = e / ((int64_t)n[0] * n[1]);
        const int64_t b = ex * sx + ey * sy + ez * sz;
        const double* X[8];   // X[a + 2(b + 2c)] = vertex (ex+a, ey+b, ez+c)
        for (int k = 0; k < 2; ++k)
            for (int j = 0; j < 2; ++j)
                for (int i = 0; i < 2; ++i) X[i + 2 * (j + 2 * k)] = v + 3 * (b + i * sx + j * sy + k * sz);
        element_map_coefficients(X, coef.data() + (size_t)e * 21);
    }
}

template <typename T>
int upload_as(const std::vector<double>& h, void** dst) {
    std::vector<T> t(h.begin(), h.end());
    if (hipMalloc(dst, t.size() * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(PA_ENOMEM, "device allocation of %zu words failed", t.size());
    }
    PA_HIP(hipMemcpy(*dst, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
    return PA_OK;
}

}  // namespace

// Device geometry of a non-affine operator from its map coefficients coef [NE][21]:
// the det J > 0 check at every quadrature point, gd of op->geo's form, and element
// data holding lambda, mu without det J.
int finish_geometry(pa_op* op, const std::vector<double>& coef, const double* lam, const double* mu) {
    const int64_t NE = op->NE;
    const int Q = op->q, Q3 = Q * Q * Q;
    const size_t esz = op->dtype == PA_F64 ? sizeof(double) : sizeof(float);
    double* d_coef = nullptr;
    double* d_min = nullptr;
    int rc = PA_OK;
    do {
        if (hipMalloc(&d_coef, coef.size() * sizeof(double)) != hipSuccess ||
            hipMalloc(&d_min, (size_t)NE * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(PA_ENOMEM, "device allocation of the geometry setup failed");
            break;
        }
        hipError_t e = hipMemcpy(d_coef, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e != hipSuccess) { rc = fail(PA_EHIP, "upload failed: %s", hipGetErrorString(e)); break; }
        if (op->geo == PA_GEOM_QP_DATA &&
            hipMalloc(&op->gd, (size_t)NE * 10 * Q3 * esz) != hipSuccess) {
            (void)hipGetLastError();
            op->gd = nullptr;
            rc = fail(PA_ENOMEM, "device allocation of the quadrature-point geometry (%lld elements) failed",
                      (long long)NE);
            break;
        }
        QRule r;
        for (int k = 0; k < Q; ++k) {
            r.x[k] = op->tab.xq[k];
            r.w[k] = op->tab.w[k];
        }
        const int nb = (int)((NE + 255) / 256);
        if (op->dtype == PA_F64)
            hipLaunchKernelGGL(geometry_qp_kernel<double>, dim3(nb), dim3(256), 0, op->stream, d_coef, r, Q, (int)NE,
                               (double*)op->gd, d_min);
        else
            hipLaunchKernelGGL(geometry_qp_kernel<float>, dim3(nb), dim3(256), 0, op->stream, d_coef, r, Q, (int)NE,
                               (float*)op->gd, d_min);
        e = hipGetLastError();
        std::vector<double> mn((size_t)NE);
        if (e == hipSuccess) e = hipMemcpyAsync(mn.data(), d_min, NE * sizeof(double), hipMemcpyDeviceToHost, op->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(op->stream);
        if (e != hipSuccess) { rc = fail(PA_EHIP, "geometry setup failed: %s", hipGetErrorString(e)); break; }
        for (int64_t i = 0; i < NE; ++i)
            if (!(mn[i] > 0.0)) {
                rc = fail(PA_EINVAL, "element %lld: det J = %g <= 0 at a quadrature point", (long long)i, mn[i]);
                break;
            }
        if (rc) break;
        if (op->geo == PA_GEOM_TRILINEAR) {
            rc = op->dtype == PA_F64 ? upload_as<double>(coef, &op->gd) : upload_as<float>(coef, &op->gd);
            if (rc) break;
        }
        // element data of the non-affine forms: lambda, mu without det J
        std::vector<double> ed((size_t)NE * kEdStride, 0.0);
        for (int64_t i = 0; i < NE; ++i) {
            ed[(size_t)i * kEdStride + 9] = lam[i];
            ed[(size_t)i * kEdStride + 10] = mu[i];
        }
        void* d_ed = nullptr;
        rc = op->dtype == PA_F64 ? upload_as<double>(ed, &d_ed) : upload_as<float>(ed, &d_ed);
        if (rc) break;
        (void)hipFree(op->ed);
        op->ed = d_ed;
    } while (0);
    if (d_coef) (void)hipFree(d_coef);
    if (d_min) (void)hipFree(d_min);
    return rc;
}

}  // namespace pa

using namespace pa;

extern "C" int pa_elast_setup_geometry(const pa_mesh_t* m, const double* vertices, int kind, int p, int q,
                                       const double* lambda, const double* mu, int dtype, void* hip_stream,
                                       pa_op_t** out) {
    if (!out) return fail(PA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!vertices || !lambda || !mu) return fail(PA_EINVAL, "vertices/lambda/mu is NULL");
    if (kind != PA_GEOM_QP_DATA && kind != PA_GEOM_TRILINEAR) return fail(PA_EINVAL, "geometry kind %d", kind);
    MeshDesc md;
    int rc = validate_mesh(m, &md);
    if (rc) return rc;
    if (p < 1) return fail(PA_EINVAL, "p = %d must be >= 1", p);
    if (p > kMaxP) return fail(PA_EUNSUPPORTED, "p = %d > %d is not built", p, kMaxP);
    if (q != p + 2) return fail(PA_EUNSUPPORTED, "non-affine geometry is built for q = p + 2 only");
    const int64_t NV = (int64_t)(md.n[0] + 1) * (md.n[1] + 1) * (md.n[2] + 1);
    for (int64_t i = 0; i < 3 * NV; ++i)
        if (!std::isfinite(vertices[i])) return fail(PA_EINVAL, "vertex coordinate %lld is not finite", (long long)i);
    pa_op* op = nullptr;
    rc = create_op(md, p, q, lambda, mu, dtype, (hipStream_t)hip_stream, &op, kLinNever);
    if (rc) return rc;
    op->geo = kind;
    std::vector<double> coef;
    map_coefficients(md.n, vertices, coef);
    rc = finish_geometry(op, coef, lambda, mu);
    if (rc) {
        pa_elast_destroy(op);
        return rc;
    }
    *out = op;
    return PA_OK;
}
