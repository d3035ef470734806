// Geometric multigrid preconditioned CG (paper Sec. 3): level hierarchy,
// Chebyshev-Jacobi smoothing, p/h transfers, exact coarse solve, V(1,1)-cycle,
// PCG and FP64 iterative refinement around an FP32 PCG, and the step API used
// to interleave many solves on one device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "solver.h"

namespace pa {


namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct LevelPlan {
    MeshDesc mesh;
    int p;
    int kind;   // transfer from this level to the next coarser one: 0 = p, 1 = h, -1 = none
    std::vector<int> elem_map[3];   // h-coarsening: coarse element index of every fine element per axis
};

// Merge element pairs along every axis with more than one element: coarse element k
// covers fine elements 2k and 2k+1 (the last one alone when n is odd).  The fine
// mesh is a refinement of the coarse one, so the p = 1 spaces are nested.
MeshDesc coarsen_h(const MeshDesc& f) {
    MeshDesc c = f;
    for (int a = 0; a < 3; ++a) {
        if (f.n[a] <= 1) continue;
        const int nc = (f.n[a] + 1) / 2;
        c.n[a] = nc;
        c.vert[a].resize(nc + 1);
        for (int k = 0; k < nc; ++k) c.vert[a][k] = f.vert[a][2 * k];
        c.vert[a][nc] = f.vert[a][f.n[a]];
    }
    return c;
}

int64_t dofs_of(const MeshDesc& m, int p) {
    return 3 * (int64_t)(m.n[0] * p + 1) * (m.n[1] * p + 1) * (m.n[2] * p + 1);
}

std::vector<LevelPlan> plan_levels(const MeshDesc& fine, int p, const pa_solve_opts_t& o) {
    std::vector<LevelPlan> L;
    L.push_back({fine, p, -1, {}});
    int np = 0;
    while (L.back().p > 1 && (o.p_levels < 0 || np < o.p_levels)) {
        L.back().kind = 0;
        L.push_back({fine, L.back().p / 2, -1, {}});
        ++np;
    }
    if (L.back().p == 1) {
        int nh = 0;
        while (true) {
            const MeshDesc& m = L.back().mesh;
            const bool can = m.n[0] > 1 || m.n[1] > 1 || m.n[2] > 1;
            if (!can) break;
            if (o.h_levels >= 0 ? nh >= o.h_levels : dofs_of(m, 1) <= o.coarse_max_dofs) break;
            L.back().kind = 1;
            L.push_back({coarsen_h(m), 1, -1, {}});
            ++nh;
        }
    }
    return L;
}

// Host tables of the h-transfer along one axis between fine vertices xf (nf+1)
// and coarse vertices xc (nc+1), nested by pair merging.
void h_axis_tables(const std::vector<double>& xf, const std::vector<double>& xc, std::vector<int>& i0,
                   std::vector<int>& i1, std::vector<double>& t, std::vector<int>& fi, std::vector<double>& fw) {
    const int nf = (int)xf.size() - 1, nc = (int)xc.size() - 1;
    i0.assign(nf + 1, 0);
    i1.assign(nf + 1, 0);
    t.assign(nf + 1, 0.0);
    fi.assign(3 * (nc + 1), 0);
    fw.assign(3 * (nc + 1), 0.0);
    std::vector<int> cnt(nc + 1, 0);
    auto push = [&](int j, int g, double w) {
        if (w == 0.0) return;
        fi[3 * j + cnt[j]] = g;
        fw[3 * j + cnt[j]] = w;
        ++cnt[j];
    };
    for (int g = 0; g <= nf; ++g) {
        if (nf == nc) {   // axis not coarsened
            i0[g] = i1[g] = g;
            push(g, g, 1.0);
            continue;
        }
        int j;
        bool on_vertex;
        if (g == nf) { j = nc; on_vertex = true; }
        else if (g % 2 == 0) { j = g / 2; on_vertex = true; }
        else { j = g / 2; on_vertex = false; }
        if (on_vertex) {
            i0[g] = i1[g] = j;
            t[g] = 0.0;
            push(j, g, 1.0);
        } else {
            const double tt = (xf[g] - xc[j]) / (xc[j + 1] - xc[j]);
            i0[g] = j;
            i1[g] = j + 1;
            t[g] = tt;
            push(j, g, 1.0 - tt);
            push(j + 1, g, tt);
        }
    }
}

}  // namespace

struct Level {
    pa_op* op = nullptr;
    int dtype = PA_F64;
    int64_t N = 0;
    Geom g;
    void* dinv = nullptr;
    void* b = nullptr;
    void* x = nullptr;
    void* r = nullptr;
    void* d = nullptr;
    void* t = nullptr;
    double lam_hat = 0.0, lmax = 0.0, lmin = 0.0;
    int tkind = -1;
    double* Ip = nullptr;
    void* skr = nullptr;   // p-restriction: element-boundary coarse entries [NE][3][slots of the coarse element]
    HAxis hax[3];
    void* hbuf = nullptr;
};

}  // namespace pa

struct pa_gmg {
    pa_op* user = nullptr;
    pa_op* fine64 = nullptr;
    bool own_fine64 = false;
    pa_solve_opts_t opts;
    int vdtype = PA_F64;     // precision of the levels (V-cycle)
    int mode = PA_SOLVE_F64;
    std::vector<pa::Level> L;
    int Nc = 0;
    void* cinv = nullptr;
    hipStream_t stream = nullptr;
    double* part = nullptr;
    double* scal = nullptr;
    double* hscal = nullptr;
    void *pr = nullptr, *pz = nullptr, *pp = nullptr, *pAp = nullptr, *pd = nullptr;
    void* pz32 = nullptr;    // PA_SOLVE_F32_PREC: FP32 V-cycle output
    double* r64 = nullptr;
    double* t64 = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;   // a step-API solve holds the work vectors
};

struct pa_solve {
    pa_gmg* G = nullptr;
    const double* b = nullptr;
    double* x = nullptr;
    double rtol = 0.0;
    int phase = 0;       // 0 inner PCG running, 1 outer residual pending (IR), 2 finished
    int status = PA_OK;
    int inner_iters = 0; // iterations enqueued in the current inner solve
    int total_iters = 0;
    int outer = 0;
    double last_outer = 0.0;
    int stall = 0;
    bool pending = false;
    double t0 = 0.0;
    double crit_prec = 0.0;
};

namespace pa {
namespace {

void free_level(Level& v) {
    for (void* p : {v.dinv, v.b, v.x, v.r, v.d, v.t, (void*)v.Ip, v.skr, v.hbuf})
        if (p) (void)hipFree(p);
    if (v.op) pa_elast_destroy(v.op);
    v = Level();
}

size_t wsize(int dtype) { return dtype == PA_F64 ? sizeof(double) : sizeof(float); }

int alloc_vec(void** p, int64_t n, int dtype) {
    if (hipMalloc(p, (size_t)(n > 0 ? n : 1) * wsize(dtype)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PA_ENOMEM, "device allocation of %lld words failed", (long long)n);
    }
    return PA_OK;
}

// ---------------------------------------------------------------- smoothing / V-cycle

int level_apply(Level& v, const void* x, void* y) { return apply_op(v.op, x, y, 0); }

// k steps of Chebyshev acceleration on [lmin, lmax] for D^{-1}A x = D^{-1}b
// (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1).
int smooth(pa_gmg* G, int l, const void* b, void* x, bool zero) {
    Level& v = G->L[l];
    hipStream_t s = G->stream;
    const int k = G->opts.cheb_degree;
    const double theta = 0.5 * (v.lmax + v.lmin), delta = 0.5 * (v.lmax - v.lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    int rc;
    // r = b - A x (r = b from x = 0) and the first direction d = dinv r / theta, in one pass
    if (!zero && (rc = level_apply(v, x, v.t))) return rc;
    if ((rc = launch_cheb_start(v.r, v.d, v.dinv, b, zero ? nullptr : v.t, 1.0 / theta, v.dtype, v.N, s))) return rc;
    if (k == 1) return zero ? launch_copy(x, v.d, v.dtype, v.N, s) : launch_add(x, v.d, v.dtype, v.N, s);
    for (int j = 0; j + 1 < k; ++j) {
        if ((rc = level_apply(v, v.d, v.t))) return rc;
        const double rho_n = 1.0 / (2.0 * sigma - rho);
        // the first step sets x = d when x started at 0; the last one also adds the final d
        if ((rc = launch_cheb_step(x, v.r, v.t, v.d, v.dinv, rho_n * rho, 2.0 * rho_n / delta, zero && j == 0,
                                   j + 2 == k, v.dtype, v.N, s)))
            return rc;
        rho = rho_n;
    }
    return PA_OK;
}

// rc = R (rf - tf), tf optional: the residual b - A x restricted without storing it.
int restrict_to(pa_gmg* G, int l, const void* rf, void* rc, const void* tf = nullptr) {
    Level& f = G->L[l];
    Level& c = G->L[l + 1];
    if (f.tkind == 0) return launch_p_restrict(rf, tf, rc, f.skr, f.Ip, c.op->p, f.op->p, c.g, f.g, f.dtype, G->stream);
    return launch_h_restrict(rf, tf, rc, f.hax, c.g, f.g, f.dtype, G->stream);
}

int prolong_to(pa_gmg* G, int l, const void* xc, void* xf, int add) {
    Level& f = G->L[l];
    Level& c = G->L[l + 1];
    if (f.tkind == 0) return launch_p_prolong(xc, xf, f.Ip, c.op->p, f.op->p, c.g, f.g, add, f.dtype, G->stream);
    return launch_h_prolong(xc, xf, f.hax, c.g, f.g, add, f.dtype, G->stream);
}

int coarse_solve(pa_gmg* G, const void* b, void* x) {
    return launch_dense_matvec(G->cinv, b, x, G->Nc, G->vdtype, G->stream);
}

int vcycle(pa_gmg* G, int l, const void* b, void* x) {
    const int last = (int)G->L.size() - 1;
    if (l == last) return coarse_solve(G, b, x);
    Level& v = G->L[l];
    Level& c = G->L[l + 1];
    int rc;
    if ((rc = smooth(G, l, b, x, true))) return rc;
    if ((rc = level_apply(v, x, v.t))) return rc;
    if ((rc = restrict_to(G, l, b, c.b, v.t))) return rc;   // c.b = R (b - A x)
    if ((rc = vcycle(G, l + 1, c.b, c.x))) return rc;
    if ((rc = prolong_to(G, l, c.x, x, 1))) return rc;
    return smooth(G, l, b, x, false);
}

// ---------------------------------------------------------------- setup

int sync_scalars(pa_gmg* G) {
    PA_HIP(hipMemcpyAsync(G->hscal, G->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, G->stream));
    PA_HIP(hipStreamSynchronize(G->stream));
    return PA_OK;
}

// lambda_max(D^{-1}A) by power iteration from a SplitMix64 vector (clamped entries
// zeroed): w = A v, lambda = v.w / v.Dv, v <- D^{-1}w / |D^{-1}w|.  The normalisations
// read their norms from the device scalars, so the host waits once, for the last lambda.
int power_iteration(pa_gmg* G, int l, double* out) {
    Level& v = G->L[l];
    hipStream_t s = G->stream;
    int rc;
    void* vv = v.r;
    void* w = v.t;
    void* z = v.d;
    if ((rc = launch_splitmix(z, v.dtype, G->opts.seed + (uint64_t)l, v.N, s))) return rc;
    if ((rc = launch_set_clamped(z, v.dtype, v.g, 0.0, s))) return rc;
    if ((rc = launch_dot(z, z, nullptr, v.dtype, v.N, G->part, s))) return rc;
    if ((rc = launch_dot_final(G->part, G->scal, FIN_STORE, S_NB, s))) return rc;
    if ((rc = launch_cast_scale(vv, v.dtype, z, v.dtype, G->scal, S_NB, 1, v.N, s))) return rc;
    for (int it = 0; it < G->opts.power_iters; ++it) {
        if ((rc = level_apply(v, vv, w))) return rc;
        // z = D^{-1} w with v.w -> S_T0, v.Dv -> S_T1 and z.z -> S_NB, in one pass
        if ((rc = launch_power_pass(vv, w, v.dinv, z, v.dtype, v.N, G->part, s))) return rc;
        if ((rc = launch_dot_final(G->part, G->scal, FIN_STORE, S_T0, s))) return rc;
        if ((rc = launch_dot_final(G->part + 2 * kReduceBlocks, G->scal, FIN_STORE, S_NB, s))) return rc;
        if ((rc = launch_cast_scale(vv, v.dtype, z, v.dtype, G->scal, S_NB, 1, v.N, s))) return rc;
    }
    if ((rc = sync_scalars(G))) return rc;
    if (!(G->hscal[S_T1] > 0.0)) return fail(PA_EINVAL, "level %d has no free dofs", l);
    const double lam = G->hscal[S_T0] / G->hscal[S_T1];
    if (!(G->hscal[S_NB] > 0.0) || !std::isfinite(lam))
        return fail(PA_EBREAKDOWN, "power iteration broke down on level %d", l);
    *out = lam;
    return PA_OK;
}

int build_transfer(pa_gmg* G, int l, const LevelPlan& pf, const LevelPlan& pc) {
    Level& f = G->L[l];
    Level& c = G->L[l + 1];
    f.tkind = pf.kind;
    hipStream_t s = G->stream;
    if (pf.kind == 0) {
        const int Df = f.op->p + 1, Dc = c.op->p + 1;
        if (hipMalloc(&f.Ip, Df * Dc * sizeof(double)) != hipSuccess) return fail(PA_ENOMEM, "transfer alloc");
        const size_t slots = (size_t)Dc * Dc * Dc - (size_t)(Dc - 2) * (Dc - 2) * (Dc - 2);
        const size_t esz = f.dtype == PA_F64 ? sizeof(double) : sizeof(float);
        if (hipMalloc(&f.skr, (size_t)f.g.NE * 3 * slots * esz) != hipSuccess) {
            (void)hipGetLastError();
            f.skr = nullptr;
            return fail(PA_ENOMEM, "transfer alloc");
        }
        return launch_p_interp_matrix(c.op->d_tab, f.op->d_tab, c.op->p, f.op->p, f.Ip, s);
    }
    // h-transfer tables
    std::vector<int> i0[3], i1[3], fi[3];
    std::vector<double> t[3], fw[3];
    size_t ints = 0, dbls = 0;
    for (int a = 0; a < 3; ++a) {
        h_axis_tables(pf.mesh.vert[a], pc.mesh.vert[a], i0[a], i1[a], t[a], fi[a], fw[a]);
        ints += i0[a].size() + i1[a].size() + fi[a].size();
        dbls += t[a].size() + fw[a].size();
    }
    const size_t bytes = dbls * sizeof(double) + ints * sizeof(int) + 64;
    if (hipMalloc(&f.hbuf, bytes) != hipSuccess) return fail(PA_ENOMEM, "transfer alloc");
    std::vector<unsigned char> host(bytes, 0);
    size_t off = 0;
    auto put = [&](const void* src, size_t n) {
        const size_t o = off;
        std::memcpy(host.data() + off, src, n);
        off += n;
        return (unsigned char*)f.hbuf + o;
    };
    for (int a = 0; a < 3; ++a) {   // doubles first (8-byte aligned)
        f.hax[a].t = (const double*)put(t[a].data(), t[a].size() * sizeof(double));
        f.hax[a].fw = (const double*)put(fw[a].data(), fw[a].size() * sizeof(double));
    }
    for (int a = 0; a < 3; ++a) {
        f.hax[a].i0 = (const int*)put(i0[a].data(), i0[a].size() * sizeof(int));
        f.hax[a].i1 = (const int*)put(i1[a].data(), i1[a].size() * sizeof(int));
        f.hax[a].fi = (const int*)put(fi[a].data(), fi[a].size() * sizeof(int));
    }
    PA_HIP(hipMemcpyAsync(f.hbuf, host.data(), bytes, hipMemcpyHostToDevice, s));
    PA_HIP(hipStreamSynchronize(s));   // host staging buffer goes out of scope
    return PA_OK;
}

void destroy_gmg(pa_gmg* G) {
    if (!G) return;
    if (G->stream) (void)hipStreamSynchronize(G->stream);
    for (auto& v : G->L) free_level(v);
    if (G->own_fine64 && G->fine64) pa_elast_destroy(G->fine64);
    for (void* p : {G->cinv, (void*)G->part, (void*)G->scal, G->pr, G->pz, G->pp, G->pAp, G->pd, G->pz32,
                    (void*)G->r64, (void*)G->t64})
        if (p) (void)hipFree(p);
    if (G->hscal) (void)hipHostFree(G->hscal);
    if (G->ev) (void)hipEventDestroy(G->ev);
    delete G;
}

int setup_gmg(pa_op* op, const pa_solve_opts_t* o, pa_gmg** out) {
    if (op->geo != PA_GEOM_AFFINE || op->kmap) return fail(PA_EUNSUPPORTED, "the multigrid hierarchy needs the affine box");
    // general material data: the finest level keeps it, coarser levels take per-element
    // isotropic parameters derived from it (op->lam, op->mu)
    const bool gen = op->mat != PA_MAT_ELEM_ISO;
    pa_solve_opts_t opts;
    if (o) opts = *o; else pa_solve_opts_default(&opts);
    if (opts.mode != PA_SOLVE_F64 && opts.mode != PA_SOLVE_F32_IR && opts.mode != PA_SOLVE_F32_PREC)
        return fail(PA_EINVAL, "mode %d", opts.mode);
    if (opts.stop != PA_STOP_PREC && opts.stop != PA_STOP_TRUE) return fail(PA_EINVAL, "stop %d", opts.stop);
    if (opts.cheb_degree < 1 || opts.cheb_degree > 64) return fail(PA_EINVAL, "cheb_degree %d", opts.cheb_degree);
    if (opts.power_iters < 1) return fail(PA_EINVAL, "power_iters %d", opts.power_iters);
    if (!(opts.cheb_lo_frac > 0.0 && opts.cheb_lo_frac < 1.0)) return fail(PA_EINVAL, "cheb_lo_frac");
    if (!(opts.cheb_safety >= 1.0)) return fail(PA_EINVAL, "cheb_safety must be >= 1");
    if (opts.max_iter < 1 || opts.inner_max_iter < 1 || opts.max_outer < 1) return fail(PA_EINVAL, "iteration caps");
    const double t0 = now_s();
    pa_gmg* G = new (std::nothrow) pa_gmg();
    if (!G) return fail(PA_ENOMEM, "host allocation failed");
    G->user = op;
    G->opts = opts;
    G->stream = op->stream;
    G->mode = opts.mode;
    G->vdtype = opts.mode == PA_SOLVE_F64 ? PA_F64 : PA_F32;
    int rc = PA_OK;
    do {
        const std::vector<LevelPlan> plan = plan_levels(op->mesh, op->p, opts);
        const int64_t Nc = dofs_of(plan.back().mesh, plan.back().p);
        if (Nc > 20000) {
            rc = fail(PA_EUNSUPPORTED, "coarsest level has %lld dofs (> 20000): allow more h-levels",
                      (long long)Nc);
            break;
        }
        if (gen && plan.size() < 2) {
            // the coarse matrix is assembled from per-element Lame parameters
            rc = fail(PA_EUNSUPPORTED, "general material data needs at least one coarser level (p > 1 or h-levels)");
            break;
        }
        G->L.resize(plan.size());
        // level operators: per-element Lame parameters follow the element map of the coarsening;
        // with general material data the finest level keeps it, and the coarser levels take
        // op->lam, op->mu (quadrature-weighted element means of per-point data; the
        // trace-matched isotropic stiffness of an anisotropic C)
        std::vector<double> lam = op->lam, mu = op->mu;
        for (size_t l = 0; l < plan.size() && !rc; ++l) {
            Level& v = G->L[l];
            const LevelPlan& P = plan[l];
            if (l > 0 && plan[l - 1].kind == 1) {
                // coarse element properties: volume-weighted average of the merged fine elements
                const MeshDesc& mf = plan[l - 1].mesh;
                const MeshDesc& mc = P.mesh;
                const int ncE = mc.n[0] * mc.n[1] * mc.n[2];
                std::vector<double> cl(ncE, 0.0), cm(ncE, 0.0), cv(ncE, 0.0);
                for (int ez = 0; ez < mf.n[2]; ++ez)
                    for (int ey = 0; ey < mf.n[1]; ++ey)
                        for (int ex = 0; ex < mf.n[0]; ++ex) {
                            const int e = ex + mf.n[0] * (ey + mf.n[1] * ez);
                            const int cx = mf.n[0] > 1 ? ex / 2 : ex, cy = mf.n[1] > 1 ? ey / 2 : ey,
                                      cz = mf.n[2] > 1 ? ez / 2 : ez;
                            const int ce = cx + mc.n[0] * (cy + mc.n[1] * cz);
                            const double vol = (mf.vert[0][ex + 1] - mf.vert[0][ex]) *
                                               (mf.vert[1][ey + 1] - mf.vert[1][ey]) *
                                               (mf.vert[2][ez + 1] - mf.vert[2][ez]);
                            cl[ce] += vol * lam[e];
                            cm[ce] += vol * mu[e];
                            cv[ce] += vol;
                        }
                for (int e = 0; e < ncE; ++e) { cl[e] /= cv[e]; cm[e] /= cv[e]; }
                lam.swap(cl);
                mu.swap(cm);
            }
            if (l == 0 && gen)
                rc = create_material_op(P.mesh, P.p, op->q, op->mat, op->mdata.data(), G->vdtype, G->stream, &v.op);
            else
                rc = create_op(P.mesh, P.p, P.p + (op->q - op->p), lam.data(), mu.data(), G->vdtype, G->stream,
                               &v.op);
            if (rc) break;
            v.dtype = G->vdtype;
            v.N = v.op->N;
            v.g = make_geom(P.mesh, P.p, true);
            if ((rc = alloc_vec(&v.b, v.N, v.dtype)) || (rc = alloc_vec(&v.x, v.N, v.dtype))) break;
            if (l + 1 < plan.size()) {
                if ((rc = alloc_vec(&v.dinv, v.N, v.dtype)) || (rc = alloc_vec(&v.r, v.N, v.dtype)) ||
                    (rc = alloc_vec(&v.d, v.N, v.dtype)) || (rc = alloc_vec(&v.t, v.N, v.dtype)))
                    break;
            }
        }
        if (rc) break;
        if (hipMalloc(&G->part, 4 * kReduceBlocks * sizeof(double)) != hipSuccess ||
            hipMalloc(&G->scal, S_COUNT * sizeof(double)) != hipSuccess ||
            hipHostMalloc(&G->hscal, S_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&G->ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            rc = fail(PA_ENOMEM, "solver scalar allocation failed");
            break;
        }
        PA_HIP(hipMemsetAsync(G->scal, 0, S_COUNT * sizeof(double), G->stream));
        if ((rc = launch_fill(G->scal + S_ONE, PA_F64, 1, 1.0, G->stream))) break;
        for (size_t l = 0; l + 1 < plan.size() && !rc; ++l) rc = build_transfer(G, (int)l, plan[l], plan[l + 1]);
        if (rc) break;
        // smoothers: diagonal, lambda_max
        for (size_t l = 0; l + 1 < plan.size() && !rc; ++l) {
            Level& v = G->L[l];
            if ((rc = launch_diagonal(v.op, v.dinv, 1))) break;
            if ((rc = launch_reciprocal(v.dinv, v.dtype, v.N, G->stream))) break;
            double lh = 0.0;
            if (opts.lambda_max && opts.lambda_max[l] > 0.0) lh = opts.lambda_max[l];
            else if ((rc = power_iteration(G, (int)l, &lh))) break;
            v.lam_hat = lh;
            v.lmax = opts.cheb_safety * lh;
            v.lmin = opts.cheb_lo_frac * v.lmax;
        }
        if (rc) break;
        // exact coarse solve: dense inverse of the assembled constrained coarsest matrix
        {
            Level& c = G->L.back();
            G->Nc = (int)c.N;
            double* A = nullptr;
            double* work = nullptr;
            if (hipMalloc(&A, (size_t)G->Nc * G->Nc * sizeof(double)) != hipSuccess ||
                hipMalloc(&work, (size_t)coarse_invert_words(G->Nc) * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                if (A) (void)hipFree(A);
                rc = fail(PA_ENOMEM, "coarse matrix allocation failed (%d dofs)", G->Nc);
                break;
            }
            rc = launch_coarse_assemble(A, G->Nc, c.op, G->stream);
            if (!rc) rc = coarse_invert(A, work, G->Nc, G->stream);
            if (!rc && G->vdtype == PA_F32) {
                void* a32 = nullptr;
                rc = alloc_vec(&a32, (int64_t)G->Nc * G->Nc, PA_F32);
                if (!rc) rc = launch_dense_cast(a32, PA_F32, A, (int64_t)G->Nc * G->Nc, G->stream);
                if (!rc) {
                    PA_HIP(hipStreamSynchronize(G->stream));
                    (void)hipFree(A);
                    A = (double*)a32;
                }
            }
            PA_HIP(hipStreamSynchronize(G->stream));
            (void)hipFree(work);
            G->cinv = A;
            if (rc) break;
        }
        // PCG work vectors (PCG precision) and the FP64 outer operator
        const int64_t N0 = G->L[0].N;
        const int pdt = G->mode == PA_SOLVE_F32_IR ? PA_F32 : PA_F64;
        if ((rc = alloc_vec(&G->pr, N0, pdt)) || (rc = alloc_vec(&G->pz, N0, pdt)) ||
            (rc = alloc_vec(&G->pp, N0, pdt)) || (rc = alloc_vec(&G->pAp, N0, pdt)))
            break;
        if (G->mode == PA_SOLVE_F32_PREC) {
            if ((rc = alloc_vec(&G->pd, N0, PA_F32)) || (rc = alloc_vec(&G->pz32, N0, PA_F32))) break;
        }
        if (G->mode == PA_SOLVE_F32_IR) {
            if ((rc = alloc_vec(&G->pd, N0, PA_F32)) || (rc = alloc_vec((void**)&G->r64, N0, PA_F64)) ||
                (rc = alloc_vec((void**)&G->t64, N0, PA_F64)))
                break;
        }
        if (op->dtype == PA_F64) {
            G->fine64 = op;
        } else {
            rc = gen ? create_material_op(op->mesh, op->p, op->q, op->mat, op->mdata.data(), PA_F64, G->stream,
                                         &G->fine64)
                    : create_op(op->mesh, op->p, op->q, op->lam.data(), op->mu.data(), PA_F64, G->stream, &G->fine64);
            if (rc) break;
            G->own_fine64 = true;
        }
        hipError_t e = hipStreamSynchronize(G->stream);
        if (e != hipSuccess) rc = fail(PA_EHIP, "gmg setup failed: %s", hipGetErrorString(e));
    } while (0);
    if (rc) {
        destroy_gmg(G);
        return rc;
    }
    (void)t0;
    *out = G;
    return PA_OK;
}

// ---------------------------------------------------------------- PCG state machine

int enqueue_copy_event(pa_solve* S) {
    pa_gmg* G = S->G;
    PA_HIP(hipMemcpyAsync(G->hscal, G->scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, G->stream));
    PA_HIP(hipEventRecord(G->ev, G->stream));
    S->pending = true;
    return PA_OK;
}

// Inner PCG vectors: x = xin (the unknown), r, z, p, Ap in dtype dt; operator Aop.
struct InnerCtx {
    pa_op* Aop;
    void* x;
    int dt;
    int64_t N;
};

InnerCtx inner_ctx(pa_solve* S) {
    pa_gmg* G = S->G;
    if (G->mode == PA_SOLVE_F32_IR) return {G->L[0].op, G->pd, PA_F32, G->L[0].N};
    return {G->fine64, S->x, PA_F64, G->L[0].N};
}

// Preconditioner z = B r of the PCG: the V-cycle in the levels' precision; in
// PA_SOLVE_F32_PREC mode r and z are FP64 and the V-cycle runs in FP32 between two casts.
int precondition(pa_gmg* G, const void* r, void* z) {
    if (G->mode != PA_SOLVE_F32_PREC) return vcycle(G, 0, r, z);
    const int64_t N = G->L[0].N;
    int rc;
    if ((rc = launch_cast_scale(G->pd, PA_F32, r, PA_F64, G->scal, S_ONE, 0, N, G->stream))) return rc;
    if ((rc = vcycle(G, 0, G->pd, G->pz32))) return rc;
    return launch_cast_scale(z, PA_F64, G->pz32, PA_F32, G->scal, S_ONE, 0, N, G->stream);
}

// Start the inner PCG on A x = b_in where r already holds b_in - A x: z = B r, p = z, rz0.
int inner_begin(pa_solve* S, double rtol, int stop) {
    pa_gmg* G = S->G;
    InnerCtx c = inner_ctx(S);
    int rc;
    if ((rc = precondition(G, G->pr, G->pz))) return rc;
    if ((rc = launch_copy(G->pp, G->pz, c.dt, c.N, G->stream))) return rc;
    if ((rc = launch_dot(G->pr, G->pz, G->pr, c.dt, c.N, G->part, G->stream))) return rc;
    S->inner_iters = 0;
    return launch_pcg_init(G->part, G->scal, rtol, stop, G->stream);
}

int inner_iteration(pa_solve* S) {
    pa_gmg* G = S->G;
    InnerCtx c = inner_ctx(S);
    hipStream_t s = G->stream;
    int rc;
    if ((rc = apply_op(c.Aop, G->pp, G->pAp, 0))) return rc;
    if ((rc = launch_dot(G->pp, G->pAp, nullptr, c.dt, c.N, G->part, s))) return rc;
    if ((rc = launch_dot_final(G->part, G->scal, FIN_ALPHA, 0, s))) return rc;
    if ((rc = launch_pcg_xr(c.x, G->pr, G->pp, G->pAp, G->scal, c.dt, c.N, s))) return rc;
    if ((rc = precondition(G, G->pr, G->pz))) return rc;
    if ((rc = launch_dot(G->pr, G->pz, G->pr, c.dt, c.N, G->part, s))) return rc;
    if ((rc = launch_dot_final(G->part, G->scal, FIN_BETA, 0, s))) return rc;
    if ((rc = launch_pcg_p(G->pp, G->pz, G->scal, c.dt, c.N, s))) return rc;
    S->inner_iters++;
    S->total_iters++;
    return PA_OK;
}

// FP64 outer residual r64 = b - A64 x and its squared norm into S_NR.
int outer_residual(pa_solve* S, double* r, double* tmp) {
    pa_gmg* G = S->G;
    int rc;
    if ((rc = apply_op(G->fine64, S->x, tmp, 0))) return rc;
    if ((rc = launch_residual(r, S->b, tmp, PA_F64, G->fine64->N, G->stream))) return rc;
    if ((rc = launch_dot(r, r, nullptr, PA_F64, G->fine64->N, G->part, G->stream))) return rc;
    return launch_dot_final(G->part, G->scal, FIN_STORE, S_NR, G->stream);
}

int enqueue_inner_batch(pa_solve* S, int n) {
    const pa_solve_opts_t& o = S->G->opts;
    const bool ir = S->G->mode == PA_SOLVE_F32_IR;
    int rc;
    for (int i = 0; i < n; ++i) {
        if (ir ? S->inner_iters >= o.inner_max_iter : S->total_iters >= o.max_iter) break;
        if ((rc = inner_iteration(S))) return rc;
    }
    return enqueue_copy_event(S);
}

int solve_begin(pa_gmg* G, const double* b, double* x, double rtol, pa_solve* S) {
    S->G = G;
    S->b = b;
    S->x = x;
    S->rtol = rtol;
    S->t0 = now_s();
    int rc;
    hipStream_t s = G->stream;
    // |b|^2 -> S_BB (true-residual stop) and S_NB
    if ((rc = launch_dot(b, b, nullptr, PA_F64, G->fine64->N, G->part, s))) return rc;
    if ((rc = launch_dot_final(G->part, G->scal, FIN_STORE, S_NB, s))) return rc;
    if ((rc = launch_dot_final(G->part, G->scal, FIN_STORE, S_BB, s))) return rc;
    if (G->mode != PA_SOLVE_F32_IR) {
        // r = b - A x
        if ((rc = apply_op(G->fine64, x, G->pAp, 0))) return rc;
        if ((rc = launch_residual(G->pr, b, G->pAp, PA_F64, G->fine64->N, s))) return rc;
        if ((rc = inner_begin(S, rtol, G->opts.stop))) return rc;
        S->phase = 0;
    } else {
        if ((rc = outer_residual(S, G->r64, G->t64))) return rc;
        S->phase = 1;
    }
    return enqueue_copy_event(S);
}

// Decide from the host copy of the scalars; enqueue the next batch unless finished.
int solve_advance(pa_solve* S, int batch, bool may_enqueue) {
    pa_gmg* G = S->G;
    const double* h = G->hscal;
    const pa_solve_opts_t& o = G->opts;
    int rc;
    if (S->phase == 2) return PA_OK;
    if (G->mode != PA_SOLVE_F32_IR) {
        if (S->phase == 1) {
            // true-residual check after the recursive residual met the test: the recursion
            // drifts from b - A x, so restart from the current x when the true one is too big
            const double nr = std::sqrt(h[S_NR]), nb = std::sqrt(h[S_NB]);
            if ((nb > 0.0 ? nr / nb : 0.0) <= S->rtol || nr == 0.0) { S->phase = 2; S->status = PA_OK; return PA_OK; }
            if (S->total_iters >= o.max_iter || S->outer >= 8) { S->phase = 2; S->status = PA_ENOCONV; return PA_OK; }
            if (!may_enqueue) return PA_OK;
            S->outer++;
            if ((rc = inner_begin(S, S->rtol, o.stop))) return rc;   // pr already holds b - A x
            S->phase = 0;
            return enqueue_inner_batch(S, batch);
        }
        S->crit_prec = h[S_CRIT];
        if (h[S_DONE] == 2.0) { S->phase = 2; S->status = PA_EBREAKDOWN; return PA_OK; }
        if (h[S_DONE] == 1.0) {
            if (o.stop != PA_STOP_TRUE) { S->phase = 2; S->status = PA_OK; return PA_OK; }
            if (!may_enqueue) return PA_OK;
            if ((rc = outer_residual(S, (double*)G->pr, (double*)G->pAp))) return rc;
            S->phase = 1;
            return enqueue_copy_event(S);
        }
        if (S->total_iters >= o.max_iter) { S->phase = 2; S->status = PA_ENOCONV; return PA_OK; }
        if (!may_enqueue) return PA_OK;
        return enqueue_inner_batch(S, batch);
    }
    if (S->phase == 1) {
        // outer test on the FP64 residual
        const double nr = std::sqrt(h[S_NR]), nb = std::sqrt(h[S_NB]);
        const double crit = nb > 0.0 ? nr / nb : 0.0;
        if (crit <= S->rtol || nr == 0.0) { S->phase = 2; S->status = PA_OK; return PA_OK; }
        if (S->outer >= o.max_outer) { S->phase = 2; S->status = PA_ENOCONV; return PA_OK; }
        const bool stalled = S->outer > 0 && crit >= 0.5 * S->last_outer;
        if (stalled && S->stall + 1 >= 3) { S->phase = 2; S->status = PA_ENOCONV; return PA_OK; }
        if (!may_enqueue) return PA_OK;
        S->stall = stalled ? S->stall + 1 : 0;
        S->last_outer = crit;
        // inner solve of A d = r / |r| in FP32 from d = 0
        if ((rc = launch_cast_scale(G->pr, PA_F32, G->r64, PA_F64, G->scal, S_NR, 1, G->fine64->N, G->stream)))
            return rc;
        if ((rc = launch_fill(G->pd, PA_F32, G->L[0].N, 0.0, G->stream))) return rc;
        if ((rc = inner_begin(S, o.inner_rtol, PA_STOP_PREC))) return rc;
        S->phase = 0;
        return enqueue_inner_batch(S, batch);
    }
    // phase 0 in IR mode: inner PCG running
    S->crit_prec = h[S_CRIT];
    const bool inner_done = h[S_DONE] != 0.0 || S->inner_iters >= o.inner_max_iter;
    if (!inner_done) {
        if (!may_enqueue) return PA_OK;
        return enqueue_inner_batch(S, batch);
    }
    if (!may_enqueue) return PA_OK;
    // refinement: x += |r| d (FP64), then the new FP64 residual
    if ((rc = launch_ir_update(S->x, G->pd, PA_F32, G->scal, S_NR, G->fine64->N, G->stream))) return rc;
    if ((rc = outer_residual(S, G->r64, G->t64))) return rc;
    S->outer++;
    S->phase = 1;
    return enqueue_copy_event(S);
}

int solve_end(pa_solve* S, pa_solve_info_t* info) {
    pa_gmg* G = S->G;
    PA_HIP(hipStreamSynchronize(G->stream));
    const double t_solve = now_s() - S->t0;
    if (info) {
        // true FP64 residual of the returned x
        const bool ir = G->mode == PA_SOLVE_F32_IR;
        double* r = ir ? G->r64 : (double*)G->pr;
        double* tmp = ir ? G->t64 : (double*)G->pAp;
        int rc = outer_residual(S, r, tmp);
        if (rc) return rc;
        if ((rc = sync_scalars(G))) return rc;
        info->iters = S->total_iters;
        info->outer_iters = S->outer;
        const double nb = std::sqrt(G->hscal[S_NB]);
        info->rel_res_true = nb > 0.0 ? std::sqrt(G->hscal[S_NR]) / nb : 0.0;
        info->rel_res_prec = S->crit_prec;
        info->t_solve = t_solve;
        info->num_levels = (int)G->L.size();
    }
    return PA_OK;
}

int run_blocking(pa_gmg* G, const double* b, double* x, double rtol, pa_solve_info_t* info) {
    if (G->busy) return fail(PA_EINVAL, "hierarchy is in use by a step-API solve");
    if (!(rtol > 0.0)) return fail(PA_EINVAL, "rtol must be > 0");
    pa_solve S;
    int rc = solve_begin(G, b, x, rtol, &S);
    while (!rc && S.phase != 2) {
        PA_HIP(hipEventSynchronize(G->ev));
        S.pending = false;
        rc = solve_advance(&S, 1, true);
    }
    if (rc) {
        (void)hipStreamSynchronize(G->stream);
        return rc;
    }
    rc = solve_end(&S, info);
    if (rc) return rc;
    return S.status;
}

}  // namespace

int64_t bytes_required(const MeshDesc& md, int p, int dtype, int with_solver) {
    const size_t w = wsize(dtype);
    const int64_t NE = (int64_t)md.n[0] * md.n[1] * md.n[2];
    int64_t bytes = NE * kEdStride * (int64_t)w + skeleton_words(p, md.n, kLinBySize, dtype) * (int64_t)w + 4096;
    if (!with_solver) return bytes;
    pa_solve_opts_t o;
    pa_solve_opts_default(&o);
    if (dtype == PA_F32) o.mode = PA_SOLVE_F32_IR;
    const int vt = dtype == PA_F32 ? PA_F32 : PA_F64;
    const size_t vw = wsize(vt);
    const std::vector<LevelPlan> plan = plan_levels(md, p, o);
    for (size_t l = 0; l < plan.size(); ++l) {
        const MeshDesc& m = plan[l].mesh;
        const int64_t n = dofs_of(m, plan[l].p);
        const int64_t ne = (int64_t)m.n[0] * m.n[1] * m.n[2];
        bytes += (ne * kEdStride + skeleton_words(plan[l].p, m.n, kLinBySize, vt)) * (int64_t)vw +
                 (l + 1 < plan.size() ? 6 : 2) * n * (int64_t)vw + 65536;
    }
    const int64_t nc = dofs_of(plan.back().mesh, plan.back().p);
    bytes += nc * nc * (int64_t)(sizeof(double) + vw) + coarse_invert_words((int)nc) * (int64_t)sizeof(double);
    const int64_t n0 = dofs_of(md, p);
    bytes += 4 * n0 * (int64_t)vw;
    if (vt == PA_F32) bytes += n0 * 4 + 2 * n0 * 8 + (NE * kEdStride + skeleton_words(p, md.n, kLinBySize, PA_F64)) * 8;
    return bytes;
}

}  // namespace pa

using namespace pa;

extern "C" {

int gmg_setup(pa_op_t* op, const pa_solve_opts_t* o, pa_gmg_t** out) {
    if (!op || !out) return fail(PA_EINVAL, "NULL argument");
    *out = nullptr;
    return setup_gmg(op, o, out);
}

void gmg_destroy(pa_gmg_t* g) { destroy_gmg(g); }

int gmg_num_levels(const pa_gmg_t* g) { return g ? (int)g->L.size() : 0; }

int gmg_level_info(const pa_gmg_t* g, int level, int32_t n[3], int* p, int64_t* ndofs, int* dtype,
                   double* lambda_max) {
    if (!g || level < 0 || level >= (int)g->L.size()) return fail(PA_EINVAL, "bad level %d", level);
    const Level& v = g->L[level];
    if (n)
        for (int a = 0; a < 3; ++a) n[a] = v.op->mesh.n[a];
    if (p) *p = v.op->p;
    if (ndofs) *ndofs = v.N;
    if (dtype) *dtype = v.dtype;
    if (lambda_max) *lambda_max = v.lmax;
    return PA_OK;
}

int gmg_level_op(pa_gmg_t* g, int level, pa_op_t** op) {
    if (!g || !op || level < 0 || level >= (int)g->L.size()) return fail(PA_EINVAL, "bad level %d", level);
    *op = g->L[level].op;
    return PA_OK;
}

int gmg_prolong(pa_gmg_t* g, int level, const void* xc, void* xf) {
    if (!g || !xc || !xf || level < 0 || level + 1 >= (int)g->L.size()) return fail(PA_EINVAL, "bad level %d", level);
    return prolong_to(g, level, xc, xf, 0);
}

int gmg_restrict(pa_gmg_t* g, int level, const void* rf, void* rc) {
    if (!g || !rf || !rc || level < 0 || level + 1 >= (int)g->L.size()) return fail(PA_EINVAL, "bad level %d", level);
    return restrict_to(g, level, rf, rc);
}

int gmg_smooth(pa_gmg_t* g, int level, const void* b, void* x, int x_is_zero) {
    if (!g || !b || !x || level < 0 || level + 1 >= (int)g->L.size()) return fail(PA_EINVAL, "bad level %d", level);
    return smooth(g, level, b, x, x_is_zero != 0);
}

int gmg_coarse_solve(pa_gmg_t* g, const void* b, void* x) {
    if (!g || !b || !x) return fail(PA_EINVAL, "NULL argument");
    return coarse_solve(g, b, x);
}

int gmg_vcycle(pa_gmg_t* g, const void* r, void* z) {
    if (!g || !r || !z) return fail(PA_EINVAL, "NULL argument");
    if (r == z) return fail(PA_EINVAL, "r and z must not alias");
    if (g->busy) return fail(PA_EINVAL, "hierarchy is in use by a step-API solve");
    return vcycle(g, 0, r, z);
}

int gmg_pcg_run(pa_gmg_t* g, const double* b, double* x, double rtol, pa_solve_info_t* info) {
    if (!g || !b || !x) return fail(PA_EINVAL, "NULL argument");
    if ((const void*)b == (const void*)x) return fail(PA_EINVAL, "b and x must not alias");
    return run_blocking(g, b, x, rtol, info);
}

int gmg_pcg_solve(pa_op_t* op, const double* b, double* x, double rtol, const pa_solve_opts_t* o,
                  pa_solve_info_t* info) {
    if (!op || !b || !x) return fail(PA_EINVAL, "NULL argument");
    pa_solve_opts_t opts;
    if (o) opts = *o; else pa_solve_opts_default(&opts);
    const double t0 = now_s();
    const bool same = op->cached && std::memcmp(&opts, &op->cached_opts, sizeof(opts)) == 0 && !opts.lambda_max;
    if (!same) {
        if (op->cached) destroy_gmg(op->cached);
        op->cached = nullptr;
        int rc = setup_gmg(op, &opts, &op->cached);
        if (rc) return rc;
        op->cached_opts = opts;
    }
    const double t_setup = now_s() - t0;
    const int rc = run_blocking(op->cached, b, x, rtol, info);
    if (info) info->t_setup = t_setup;
    return rc;
}

int gmg_pcg_begin(pa_gmg_t* g, const double* b, double* x, double rtol, pa_solve_t** out) {
    if (!g || !b || !x || !out) return fail(PA_EINVAL, "NULL argument");
    if (!(rtol > 0.0)) return fail(PA_EINVAL, "rtol must be > 0");
    if (g->busy) return fail(PA_EINVAL, "hierarchy already has a solve in flight");
    pa_solve* S = new (std::nothrow) pa_solve();
    if (!S) return fail(PA_ENOMEM, "host allocation failed");
    int rc = solve_begin(g, b, x, rtol, S);
    if (rc) {
        (void)hipStreamSynchronize(g->stream);
        delete S;
        return rc;
    }
    g->busy = true;
    *out = S;
    return PA_OK;
}

int gmg_pcg_step(pa_solve_t* S, int n_iters) {
    if (!S || n_iters < 1) return fail(PA_EINVAL, "bad arguments");
    if (S->phase == 2) return PA_OK;
    if (S->pending) {
        const hipError_t e = hipEventQuery(S->G->ev);
        if (e == hipErrorNotReady) return PA_OK;
        if (e != hipSuccess) return fail(PA_EHIP, "event query: %s", hipGetErrorString(e));
        S->pending = false;
    }
    return solve_advance(S, n_iters, true);
}

int gmg_pcg_poll(pa_solve_t* S, int* done, int* status) {
    if (!S || !done) return fail(PA_EINVAL, "NULL argument");
    *done = 0;
    if (S->phase != 2 && S->pending) {
        const hipError_t e = hipEventQuery(S->G->ev);
        if (e == hipErrorNotReady) return PA_OK;
        if (e != hipSuccess) return fail(PA_EHIP, "event query: %s", hipGetErrorString(e));
        S->pending = false;
    }
    if (S->phase != 2 && !S->pending) {
        const int rc = solve_advance(S, 1, false);
        if (rc) return rc;
    }
    if (S->phase == 2) {
        *done = 1;
        if (status) *status = S->status;
    }
    return PA_OK;
}

int gmg_pcg_end(pa_solve_t* S, pa_solve_info_t* info) {
    if (!S) return fail(PA_EINVAL, "NULL argument");
    int rc = solve_end(S, info);
    S->G->busy = false;
    const int st = S->phase == 2 ? S->status : PA_ENOCONV;
    delete S;
    return rc ? rc : st;
}

int64_t pa_bytes_required(const pa_mesh_t* m, int p, int dtype, int with_solver) {
    MeshDesc md;
    int rc = validate_mesh(m, &md);
    if (rc) return rc;
    if (p < 1 || p > kMaxP) return fail(PA_EINVAL, "p = %d", p);
    if (dtype != PA_F64 && dtype != PA_F32) return fail(PA_EINVAL, "dtype %d", dtype);
    return bytes_required(md, p, dtype, with_solver);
}

}  // extern "C"
