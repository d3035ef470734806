// Unstructured hexahedral meshes: the operator on an explicit element-to-node map
// (element order and orientation arbitrary), its validation, and the gather lists
// that assemble element-boundary contributions in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "apply_kernel.h"
#include "internal.h"
#include "kernels.h"

namespace pa {
namespace {

template <int D>
void slot_table(std::vector<int>& slot) {
    using SK = Skel<D>;
    slot.assign(D * D * D, -1);
    for (int iz = 0; iz < D; ++iz)
        for (int iy = 0; iy < D; ++iy)
            for (int ix = 0; ix < D; ++ix)
                if (!SK::interior(ix, iy, iz)) slot[ix + D * (iy + D * iz)] = SK::index(ix, iy, iz);
}

// Skeleton slot of every local node (-1 for element-interior nodes) and the slot count.
int skeleton_slots(int p, std::vector<int>& slot) {
    switch (p + 1) {
        case 2: slot_table<2>(slot); return Skel<2>::S;
        case 3: slot_table<3>(slot); return Skel<3>::S;
        case 4: slot_table<4>(slot); return Skel<4>::S;
        case 5: slot_table<5>(slot); return Skel<5>::S;
        case 6: slot_table<6>(slot); return Skel<6>::S;
        case 7: slot_table<7>(slot); return Skel<7>::S;
        case 8: slot_table<8>(slot); return Skel<8>::S;
        case 9: slot_table<9>(slot); return Skel<9>::S;
    }
    return 0;
}

template <typename V>
int upload(const std::vector<V>& h, V** dst) {
    if (h.empty()) {
        *dst = nullptr;
        return PA_OK;
    }
    if (hipMalloc(dst, h.size() * sizeof(V)) != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return fail(PA_ENOMEM, "device allocation of %zu words failed", h.size());
    }
    PA_HIP(hipMemcpy(*dst, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
    return PA_OK;
}

}  // namespace
}  // namespace pa

using namespace pa;

extern "C" int pa_elast_setup_unstructured(int64_t num_vertices, const double* vertices, int64_t num_elements,
                                           const int32_t* elem_vertices, int64_t num_nodes,
                                           const int32_t* elem_nodes, const uint8_t* clamped, int p, int q,
                                           const double* lambda, const double* mu, int dtype, void* hip_stream,
                                           pa_op_t** out) {
    if (!out) return fail(PA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!vertices || !elem_vertices || !elem_nodes || !lambda || !mu) return fail(PA_EINVAL, "NULL argument");
    if (p < 1) return fail(PA_EINVAL, "p = %d must be >= 1", p);
    if (p > kMaxP) return fail(PA_EUNSUPPORTED, "p = %d > %d is not built", p, kMaxP);
    if (q != p + 2) return fail(PA_EUNSUPPORTED, "unstructured meshes are built for q = p + 2 only");
    if (dtype != PA_F64 && dtype != PA_F32) return fail(PA_EINVAL, "dtype %d is not PA_F64/PA_F32", dtype);
    if (num_vertices < 1 || num_elements < 1 || num_nodes < 1)
        return fail(PA_EINVAL, "need at least one vertex, element and node");
    const int D = p + 1, D3 = D * D * D;
    std::vector<int> slot;
    const int S = skeleton_slots(p, slot);
    const int64_t NE = num_elements, NV = num_vertices, Nn = num_nodes;
    if (3 * Nn >= (int64_t(1) << 31) || NE * 3 * S >= (int64_t(1) << 31) || NE * D3 >= (int64_t(1) << 31))
        return fail(PA_EUNSUPPORTED, "problem too large for 32-bit indexing");
    for (int64_t i = 0; i < 3 * NV; ++i)
        if (!std::isfinite(vertices[i])) return fail(PA_EINVAL, "vertex coordinate %lld is not finite", (long long)i);
    for (int64_t i = 0; i < 8 * NE; ++i)
        if (elem_vertices[i] < 0 || elem_vertices[i] >= NV)
            return fail(PA_EINVAL, "element %lld: vertex index %d out of range", (long long)(i / 8), elem_vertices[i]);
    for (int64_t e = 0; e < NE; ++e) {
        const double l = lambda[e], m = mu[e];
        if (!std::isfinite(l) || !std::isfinite(m) || !(m > 0.0) || !(l + 2.0 * m / 3.0 > 0.0))
            return fail(PA_EINVAL, "element %lld: need mu > 0 and lambda + 2 mu / 3 > 0", (long long)e);
    }
    // node references: in range, distinct within an element, element-interior nodes owned once
    std::vector<int> refs((size_t)Nn, 0);
    std::vector<char> interior((size_t)Nn, 0);
    std::vector<int32_t> tmp(D3);
    for (int64_t e = 0; e < NE; ++e) {
        const int32_t* en = elem_nodes + (size_t)e * D3;
        for (int a = 0; a < D3; ++a) {
            if (en[a] < 0 || en[a] >= Nn)
                return fail(PA_EINVAL, "element %lld: node index %d out of range", (long long)e, en[a]);
            ++refs[en[a]];
            if (slot[a] < 0) interior[en[a]] = 1;
        }
        std::copy(en, en + D3, tmp.begin());
        std::sort(tmp.begin(), tmp.end());
        if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end())
            return fail(PA_EINVAL, "element %lld lists a node twice", (long long)e);
    }
    for (int64_t n = 0; n < Nn; ++n)
        if (interior[n] && refs[n] != 1)
            return fail(PA_EINVAL, "node %lld is interior to an element but referenced %d times", (long long)n,
                        refs[n]);
    // gather lists over the non-interior nodes, entries in (element, slot) order
    std::vector<int> pos((size_t)Nn, -1), sk_node, sk_ptr(1, 0);
    for (int64_t n = 0; n < Nn; ++n)
        if (!interior[n]) {
            pos[n] = (int)sk_node.size();
            sk_node.push_back((int)(n | ((clamped && clamped[n]) ? kClampBit : 0u)));
            sk_ptr.push_back(sk_ptr.back() + refs[n]);
        }
    const int n_sk = (int)sk_node.size();
    // entry of every (element, slot): a node's entries follow its position in the list,
    // in ascending element order
    std::vector<int> kpos((size_t)NE * S), fillp(sk_ptr.begin(), sk_ptr.end() - 1);
    std::vector<int> kmap((size_t)NE * D3);
    for (int64_t e = 0; e < NE; ++e) {
        const int32_t* en = elem_nodes + (size_t)e * D3;
        for (int a = 0; a < D3; ++a) {
            const int n = en[a];
            kmap[(size_t)e * D3 + a] = (int)(n | ((clamped && clamped[n]) ? kClampBit : 0u));
            if (slot[a] >= 0) kpos[(size_t)e * S + slot[a]] = fillp[pos[n]]++;
        }
    }
    // map coefficients from the element corners
    std::vector<double> coef((size_t)NE * 21);
    for (int64_t e = 0; e < NE; ++e) {
        const double* X[8];
        for (int v = 0; v < 8; ++v) X[v] = vertices + 3 * (size_t)elem_vertices[e * 8 + v];
        element_map_coefficients(X, coef.data() + (size_t)e * 21);
    }

    pa_op* op = new (std::nothrow) pa_op();
    if (!op) return fail(PA_ENOMEM, "host allocation failed");
    op->p = p;
    op->q = q;
    op->dtype = dtype;
    op->NE = NE;
    op->Nn = Nn;
    op->N = 3 * Nn;
    op->stream = (hipStream_t)hip_stream;
    op->lam.assign(lambda, lambda + NE);
    op->mu.assign(mu, mu + NE);
    op->geo = PA_GEOM_TRILINEAR;
    op->n_sk = n_sk;
    pa_solve_opts_default(&op->cached_opts);
    const size_t esz = dtype == PA_F64 ? sizeof(double) : sizeof(float);
    op->sk_bytes = (size_t)NE * 3 * S * esz;
    int rc = hipGetDevice(&op->device) == hipSuccess ? PA_OK : fail(PA_EHIP, "hipGetDevice failed");
    if (!rc) rc = compute_tables(p, q, op->stream, &op->d_tab, &op->tab);
    if (!rc && hipMalloc(&op->sk, op->sk_bytes) != hipSuccess) {
        (void)hipGetLastError();
        op->sk = nullptr;
        rc = fail(PA_ENOMEM, "device allocation of the skeleton buffer failed");
    }
    if (!rc) rc = finish_geometry(op, coef, lambda, mu);
    if (!rc) rc = upload(kmap, &op->kmap);
    if (!rc) rc = upload(sk_ptr, &op->sk_ptr);
    if (!rc) rc = upload(kpos, &op->kpos);
    if (!rc) rc = upload(sk_node, &op->sk_node);
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
