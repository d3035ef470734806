// C ABI: operator setup, apply, diagonal, load vector, errors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "internal.h"
#include "kernels.h"

namespace pa {

static thread_local char g_err[1024] = "";

// ---- scratch of pa_elast_apply_noalloc: the element-boundary partial sums of one apply
// live in this array instead of the operator's own buffer.  Each device holds its own
// copy until the process ends; host code never passes the array's name to a kernel, only
// the device address looked up once per device.
constexpr size_t kScratchBytes = (size_t)PA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(PA_EUNSUPPORTED, "device %d is beyond the %d devices the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return fail(PA_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess)
            return fail(PA_EHIP, "hipSetDevice(%d): %s", dev, hipGetErrorString(e));
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !a)
            return fail(PA_EHIP, "address of the scratch array on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_addr[dev] = a;
    }
    *out = g_scratch_addr[dev];
    return PA_OK;
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int validate_mesh(const pa_mesh_t* m, MeshDesc* out) {
    if (!m) return fail(PA_EINVAL, "mesh is NULL");
    for (int a = 0; a < 3; ++a)
        if (m->n[a] < 1) return fail(PA_EINVAL, "mesh n[%d] = %d must be >= 1", a, m->n[a]);
    const double* A = m->A;
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0) || !std::isfinite(det)) return fail(PA_EINVAL, "det(A) = %g must be > 0", det);
    if (m->clamped_faces >> 6) return fail(PA_EINVAL, "clamped_faces has bits beyond the 6 faces");
    for (int a = 0; a < 3; ++a) {
        out->vert[a].resize(m->n[a] + 1);
        if (m->grade[a]) {
            for (int i = 0; i <= m->n[a]; ++i) {
                const double v = m->grade[a][i];
                if (!std::isfinite(v)) return fail(PA_EINVAL, "grade[%d][%d] is not finite", a, i);
                if (i > 0 && !(v > m->grade[a][i - 1]))
                    return fail(PA_EINVAL, "grade[%d] must be strictly increasing", a);
                out->vert[a][i] = v;
            }
        } else {
            if (!(m->L[a] > 0.0) || !std::isfinite(m->L[a])) return fail(PA_EINVAL, "L[%d] must be > 0", a);
            for (int i = 0; i <= m->n[a]; ++i) out->vert[a][i] = m->L[a] * (double)i / (double)m->n[a];
            out->vert[a][m->n[a]] = m->L[a];
        }
        out->n[a] = m->n[a];
        out->x0[a] = m->x0[a];
    }
    for (int i = 0; i < 9; ++i) out->A[i] = A[i];
    out->clamp = m->clamped_faces;
    return PA_OK;
}

// Build an operator from a validated mesh description (also used for solver levels).
int create_op(const MeshDesc& md, int p, int q, const double* lam, const double* mu, int dtype, hipStream_t s,
              pa_op** out, int lin_mode) {
    if (p < 1) return fail(PA_EINVAL, "p = %d must be >= 1", p);
    if (p > kMaxP) return fail(PA_EUNSUPPORTED, "p = %d > %d is not built", p, kMaxP);
    if (q < p + 1 || q > p + 3) return fail(PA_EINVAL, "q = %d must be in [p+1, p+3] = [%d, %d]", q, p + 1, p + 3);
    if (dtype != PA_F64 && dtype != PA_F32) return fail(PA_EINVAL, "dtype %d is not PA_F64/PA_F32", dtype);
    const int64_t NE = (int64_t)md.n[0] * md.n[1] * md.n[2];
    const int64_t Nn = (int64_t)(md.n[0] * (int64_t)p + 1) * (md.n[1] * (int64_t)p + 1) * (md.n[2] * (int64_t)p + 1);
    if (3 * Nn >= (int64_t(1) << 31) || NE >= (int64_t(1) << 31))
        return fail(PA_EUNSUPPORTED, "problem too large (%lld dofs): 32-bit indexing", (long long)(3 * Nn));
    for (int64_t e = 0; e < NE; ++e) {
        const double l = lam[e], m = mu[e];
        if (!std::isfinite(l) || !std::isfinite(m) || !(m > 0.0) || !(l + 2.0 * m / 3.0 > 0.0))
            return fail(PA_EINVAL, "element %lld: need mu > 0 and lambda + 2 mu / 3 > 0 (lambda=%g, mu=%g)",
                        (long long)e, l, m);
    }
    pa_op* op = new (std::nothrow) pa_op();
    if (!op) return fail(PA_ENOMEM, "host allocation failed");
    op->mesh = md;
    op->p = p;
    op->q = q;
    op->dtype = dtype;
    op->NE = NE;
    op->Nn = Nn;
    op->N = 3 * Nn;
    op->stream = s;
    op->lin = p == 1 && p1_runs_lin(md.n, lin_mode);
    op->sk_bytes = (size_t)skeleton_words(p, md.n, lin_mode, dtype) * (dtype == PA_F64 ? sizeof(double) : sizeof(float));
    op->lam.assign(lam, lam + NE);
    op->mu.assign(mu, mu + NE);
    pa_solve_opts_default(&op->cached_opts);
    int rc = PA_OK;
    double* d_lm = nullptr;
    const size_t nvert = md.vert[0].size() + md.vert[1].size() + md.vert[2].size();
    const size_t esz = dtype == PA_F64 ? sizeof(double) : sizeof(float);
    do {
        if (hipGetDevice(&op->device) != hipSuccess) {
            rc = fail(PA_EHIP, "hipGetDevice failed");
            break;
        }
        rc = compute_tables(p, q, s, &op->d_tab, &op->tab);
        if (rc) break;
        if (hipMalloc(&op->d_vert, nvert * sizeof(double)) != hipSuccess ||
            hipMalloc(&op->ed, (size_t)NE * kEdStride * esz) != hipSuccess ||
            hipMalloc(&op->sk, op->sk_bytes) != hipSuccess ||
            hipMalloc(&d_lm, 2 * (size_t)NE * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(PA_ENOMEM, "device allocation failed (%lld elements)", (long long)NE);
            break;
        }
        std::vector<double> hv;
        hv.reserve(nvert);
        for (int a = 0; a < 3; ++a) hv.insert(hv.end(), md.vert[a].begin(), md.vert[a].end());
        hipError_t e = hipMemcpyAsync(op->d_vert, hv.data(), nvert * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_lm, lam, NE * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_lm + NE, mu, NE * sizeof(double), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) { rc = fail(PA_EHIP, "upload failed: %s", hipGetErrorString(e)); break; }
        rc = compute_element_data(md, op->d_vert, d_lm, d_lm + NE, dtype, op->ed, s);
        if (rc) break;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) { rc = fail(PA_EHIP, "setup failed: %s", hipGetErrorString(e)); break; }
    } while (0);
    if (d_lm) (void)hipFree(d_lm);
    if (rc) {
        pa_elast_destroy(op);
        return rc;
    }
    // set-up of the no-allocation apply on this device (a failure is reported by that entry point)
    void* sa = nullptr;
    (void)scratch_address(op->device, &sa);
    *out = op;
    return PA_OK;
}

// Validate general material data: positive shear modulus and bulk modulus per
// point (isotropic), positive definite Voigt stiffness per element (anisotropic,
// by Cholesky factorisation of the unpacked upper triangle).
int check_material(int kind, const double* data, int64_t NE, int64_t per) {
    for (int64_t i = 0; i < NE * per; ++i)
        if (!std::isfinite(data[i])) return fail(PA_EINVAL, "material data entry %lld is not finite", (long long)i);
    if (kind == PA_MAT_QP_ISO) {
        for (int64_t i = 0; i < NE * per / 2; ++i) {
            const double l = data[2 * i], m = data[2 * i + 1];
            if (!(m > 0.0) || !(l + 2.0 * m / 3.0 > 0.0))
                return fail(PA_EINVAL, "element %lld point %lld: need mu > 0 and lambda + 2 mu / 3 > 0",
                            (long long)(i / (per / 2)), (long long)(i % (per / 2)));
        }
        return PA_OK;
    }
    for (int64_t e = 0; e < NE; ++e) {
        const double* c = data + e * 21;
        double A[6][6];
        for (int a = 0, k = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b, ++k) A[a][b] = A[b][a] = c[k];
        for (int j = 0; j < 6; ++j) {
            double d = A[j][j];
            for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
            if (!(d > 0.0))
                return fail(PA_EINVAL, "element %lld: the Voigt stiffness is not positive definite", (long long)e);
            A[j][j] = std::sqrt(d);
            for (int i = j + 1; i < 6; ++i) {
                double s = A[i][j];
                for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
                A[i][j] = s / A[j][j];
            }
        }
    }
    return PA_OK;
}

int apply_op(const pa_op* op, const void* x, void* y, int flags, void* sk) {
    const bool constrained = !(flags & PA_UNCONSTRAINED);
    const int add = (flags & PA_ADD) ? 1 : 0;
    ApplyLaunch L;
    if (op->kmap) {
        // unstructured mesh: only NE, Nn and the constrained flag are read
        Geom g{};
        g.nx = (int)op->NE; g.ny = g.nz = 1;
        g.Nx = (int)op->Nn; g.Ny = g.Nz = 1;
        g.Nn = (int)op->Nn;
        g.NE = (int)op->NE;
        g.clamp = constrained ? 1u : 0u;
        L.g = g;
        L.kmap = op->kmap;
        L.sk_ptr = op->sk_ptr;
        L.kpos = op->kpos;
        L.sk_node = op->sk_node;
        L.n_sk = op->n_sk;
    } else {
        L.g = make_geom(op->mesh, op->p, constrained);
    }
    L.x = x;
    L.y = y;
    L.sk = sk ? sk : op->sk;
    L.ed = op->ed;
    L.mat = op->mat;
    L.md = op->md;
    L.geo = op->geo;
    L.gd = op->gd;
    L.tab = &op->tab;
    L.add = add;
    L.lin = op->lin;
    L.stream = op->stream;
    const int qo = op->q - op->p - 1;
    switch (op->p) {
        case 1: return launch_apply_p1(L, qo, op->dtype);
        case 2: return launch_apply_p2(L, qo, op->dtype);
        case 3: return launch_apply_p3(L, qo, op->dtype);
        case 4: return launch_apply_p4(L, qo, op->dtype);
        case 5: return launch_apply_p5(L, qo, op->dtype);
        case 6: return launch_apply_p6(L, qo, op->dtype);
        case 7: return launch_apply_p7(L, qo, op->dtype);
        case 8: return launch_apply_p8(L, qo, op->dtype);
    }
    return fail(PA_EUNSUPPORTED, "p = %d not built", op->p);
}

int create_material_op(const MeshDesc& md, int p, int q, int kind, const double* data, int dtype, hipStream_t s,
                       pa_op** out) {
    const int64_t NE = (int64_t)md.n[0] * md.n[1] * md.n[2];
    const int64_t Q3 = (int64_t)q * q * q;
    const int64_t per = kind == PA_MAT_QP_ISO ? 2 * Q3 : 21;
    // unit Lame parameters: the element data then carries detJ where the kernel needs it
    std::vector<double> one((size_t)NE, 1.0);
    pa_op* op = nullptr;
    // p = 1 with per-point Lame data runs in the linear-element kernel (one lane per element),
    // which reads the data point-major: word k of point alpha of element e at (2 alpha + k) NE + e
    const bool lin = p == 1 && kind == PA_MAT_QP_ISO;
    int rc = create_op(md, p, q, one.data(), one.data(), dtype, s, &op, lin ? kLinAlways : kLinNever);
    if (rc) return rc;
    op->mat = kind;
    op->md_point_major = lin;
    // kept for solver hierarchies: the data itself (level operators in another precision)
    // and per-element isotropic parameters for the coarse levels
    op->mdata.assign(data, data + NE * per);
    if (kind == PA_MAT_ANISO) {
        // the isotropic stiffness with the same traces of the normal block (9 lambda + 6 mu)
        // and of the shear block (3 mu): positive for a positive definite C
        for (int64_t e = 0; e < NE; ++e) {
            // upper triangle row by row: (0,0) 0, (0,1) 1, (0,2) 2, (1,1) 6, (1,2) 7, (2,2) 11,
            // (3,3) 15, (4,4) 18, (5,5) 20
            const double* c = data + e * 21;
            const double m = (c[15] + c[18] + c[20]) / 3.0;
            const double n = c[0] + c[6] + c[11] + 2.0 * (c[1] + c[2] + c[7]);
            op->lam[e] = (n - 6.0 * m) / 9.0;
            op->mu[e] = m;
        }
    }
    if (kind == PA_MAT_QP_ISO) {
        for (int64_t e = 0; e < NE; ++e) {
            double sl = 0.0, sm = 0.0, sw = 0.0;
            for (int kz = 0; kz < q; ++kz)
                for (int ky = 0; ky < q; ++ky)
                    for (int kx = 0; kx < q; ++kx) {
                        const double w = op->tab.w[kx] * op->tab.w[ky] * op->tab.w[kz];
                        const int64_t al = kx + q * (ky + (int64_t)q * kz);
                        sl += w * data[(e * Q3 + al) * 2];
                        sm += w * data[(e * Q3 + al) * 2 + 1];
                        sw += w;
                    }
            op->lam[e] = sl / sw;
            op->mu[e] = sm / sw;
        }
    }
    const size_t words = (size_t)(NE * per);
    const size_t esz = dtype == PA_F64 ? sizeof(double) : sizeof(float);
    std::vector<double> tr;
    if (lin) {
        tr.resize(words);
        for (int64_t e = 0; e < NE; ++e)
            for (int64_t w = 0; w < per; ++w) tr[(size_t)(w * NE + e)] = data[e * per + w];
        data = tr.data();
    }
    if (hipMalloc(&op->md, words * esz) != hipSuccess) {
        (void)hipGetLastError();
        op->md = nullptr;
        pa_elast_destroy(op);
        return fail(PA_ENOMEM, "device allocation of the material data failed");
    }
    hipError_t e;
    if (dtype == PA_F64) {
        e = hipMemcpy(op->md, data, words * esz, hipMemcpyHostToDevice);
    } else {
        std::vector<float> f(words);
        for (size_t i = 0; i < words; ++i) f[i] = (float)data[i];
        e = hipMemcpy(op->md, f.data(), words * esz, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        pa_elast_destroy(op);
        return fail(PA_EHIP, "material upload failed: %s", hipGetErrorString(e));
    }
    *out = op;
    return PA_OK;
}

}  // namespace pa

using namespace pa;

extern "C" {

const char* pa_last_error(void) { return g_err; }

void pa_solve_opts_default(pa_solve_opts_t* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mode = PA_SOLVE_F64;
    o->stop = PA_STOP_PREC;
    o->p_levels = -1;
    o->h_levels = -1;
    o->cheb_degree = 2;
    o->power_iters = 10;
    // [0.1, 1] x 1.2 lambda_hat: measured 23-29% faster GMG-PCG solves at p >= 4 than [0.3, 1]
    // (fewer iterations); narrower safety margins diverged on some boxes
    o->cheb_lo_frac = 0.1;
    o->cheb_safety = 1.2;
    o->max_iter = 5000;
    // each refinement step gains only 2-3 digits (the FP32 operator's own error bounds the
    // contraction), so a tighter inner solve spends iterations the next step discards
    o->inner_rtol = 3e-3;
    o->inner_max_iter = 50;
    o->max_outer = 20;
    o->seed = 7;
    o->coarse_max_dofs = 3000;
    o->lambda_max = nullptr;
}

int pa_elast_setup(const pa_mesh_t* m, int p, int q, const double* lambda, const double* mu, int dtype,
                   void* hip_stream, pa_op_t** out) {
    if (!out) return fail(PA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!lambda || !mu) return fail(PA_EINVAL, "lambda/mu is NULL");
    MeshDesc md;
    int rc = validate_mesh(m, &md);
    if (rc) return rc;
    return create_op(md, p, q, lambda, mu, dtype, (hipStream_t)hip_stream, out);
}

int pa_elast_setup_material(const pa_mesh_t* m, int p, int q, int kind, const double* data, int dtype,
                            void* hip_stream, pa_op_t** out) {
    if (!out) return fail(PA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!data) return fail(PA_EINVAL, "data is NULL");
    if (kind != PA_MAT_QP_ISO && kind != PA_MAT_ANISO) return fail(PA_EINVAL, "material kind %d", kind);
    MeshDesc md;
    int rc = validate_mesh(m, &md);
    if (rc) return rc;
    if (p < 1) return fail(PA_EINVAL, "p = %d must be >= 1", p);
    if (p > kMaxP) return fail(PA_EUNSUPPORTED, "p = %d > %d is not built", p, kMaxP);
    if (q != p + 2) return fail(PA_EUNSUPPORTED, "general material data is built for q = p + 2 only");
    if (dtype != PA_F64 && dtype != PA_F32) return fail(PA_EINVAL, "dtype %d is not PA_F64/PA_F32", dtype);
    const int64_t NE = (int64_t)md.n[0] * md.n[1] * md.n[2];
    const int64_t per = kind == PA_MAT_QP_ISO ? 2 * (int64_t)q * q * q : 21;
    rc = check_material(kind, data, NE, per);
    if (rc) return rc;
    return create_material_op(md, p, q, kind, data, dtype, (hipStream_t)hip_stream, out);
}

void pa_elast_destroy(pa_op_t* op) {
    if (!op) return;
    if (op->cached) gmg_destroy(op->cached);
    if (op->abl) free_ablation(op->abl);
    if (op->ed) (void)hipFree(op->ed);
    if (op->md) (void)hipFree(op->md);
    if (op->gd) (void)hipFree(op->gd);
    for (int* a : {op->kmap, op->sk_ptr, op->kpos, op->sk_node})
        if (a) (void)hipFree(a);
    if (op->sk) (void)hipFree(op->sk);
    if (op->d_tab) (void)hipFree(op->d_tab);
    if (op->d_vert) (void)hipFree(op->d_vert);
    delete op;
}

int pa_elast_set_stream(pa_op_t* op, void* hip_stream) {
    if (!op) return fail(PA_EINVAL, "op is NULL");
    op->stream = (hipStream_t)hip_stream;
    return PA_OK;
}

int pa_elast_ndofs(const pa_op_t* op, int64_t* n) {
    if (!op || !n) return fail(PA_EINVAL, "NULL argument");
    *n = op->N;
    return PA_OK;
}

int pa_elast_apply_ex(pa_op_t* op, const void* x, void* y, int flags) {
    if (!op || !x || !y) return fail(PA_EINVAL, "NULL argument");
    if (x == y) return fail(PA_EINVAL, "x and y must not alias");
    if (flags & ~(PA_UNCONSTRAINED | PA_ADD)) return fail(PA_EINVAL, "unknown flags 0x%x", flags);
    return apply_op(op, x, y, flags);
}

int pa_elast_apply(pa_op_t* op, const void* x, void* y) { return pa_elast_apply_ex(op, x, y, 0); }

int pa_elast_apply_noalloc(pa_op_t* op, const void* x, void* y, int flags) {
    if (!op || !x || !y) return fail(PA_EINVAL, "NULL argument");
    if (x == y) return fail(PA_EINVAL, "x and y must not alias");
    if (flags & ~(PA_UNCONSTRAINED | PA_ADD)) return fail(PA_EINVAL, "unknown flags 0x%x", flags);
    if (op->sk_bytes > kScratchBytes)
        return fail(PA_EINVAL, "the operator's element-boundary sums need %zu bytes, above the %zu-byte scratch of "
                               "pa_elast_apply_noalloc (use pa_elast_apply_ex)", op->sk_bytes, kScratchBytes);
    void* s = nullptr;
    const int rc = scratch_address(op->device, &s);
    if (rc) return rc;
    return apply_op(op, x, y, flags, s);
}

int pa_elast_diagonal(pa_op_t* op, void* d, int flags) {
    if (!op || !d) return fail(PA_EINVAL, "NULL argument");
    if (flags & ~PA_UNCONSTRAINED) return fail(PA_EINVAL, "unknown flags 0x%x", flags);
    return launch_diagonal(op, d, (flags & PA_UNCONSTRAINED) ? 0 : 1);
}

int pa_elast_rhs(pa_op_t* op, const double f[3], int traction_face, const double t[3], double* b) {
    if (!op || !b) return fail(PA_EINVAL, "NULL argument");
    if (traction_face < -1 || traction_face > 5) return fail(PA_EINVAL, "traction_face %d", traction_face);
    if (traction_face >= 0 && !t) return fail(PA_EINVAL, "traction vector is NULL");
    if (op->geo != PA_GEOM_AFFINE) return fail(PA_EUNSUPPORTED, "load vectors of non-affine geometry are not built");
    return launch_rhs(op, f, traction_face, t, b, op->d_vert);
}

}  // extern "C"
