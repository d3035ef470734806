// Device helpers and host launchers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace pa {

__device__ __forceinline__ bool clamped_node(uint32_t m, int gx, int gy, int gz, const Geom& g) {
    return ((m & 1u) && gx == 0) || ((m & 2u) && gx == g.Nx - 1) || ((m & 4u) && gy == 0) ||
           ((m & 8u) && gy == g.Ny - 1) || ((m & 16u) && gz == 0) || ((m & 32u) && gz == g.Nz - 1);
}

// The elements of the degree-p box that contain node (gx, gy, gz), and the node's local
// index in each: per axis two candidates, the element before (local index p) and the
// element after (local index 0) when the node lies on an element boundary along that
// axis, a single valid one when it lies strictly inside an element.  Summing over the
// valid (x, y, z) combinations in a fixed order gives deterministic node sums.
struct NodeCands {
    int e[3][2], l[3][2];
    bool v[3][2];
};
__device__ __forceinline__ NodeCands node_candidates(const Geom& g, int p, int gx, int gy, int gz) {
    NodeCands c;
    const int gg[3] = {gx, gy, gz}, nn[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int q = gg[a] / p, r = gg[a] % p;
        if (r != 0) {
            c.e[a][0] = c.e[a][1] = q;
            c.l[a][0] = c.l[a][1] = r;
            c.v[a][0] = true;
            c.v[a][1] = false;
        } else {
            c.e[a][0] = q - 1; c.l[a][0] = p; c.v[a][0] = q > 0;
            c.e[a][1] = q; c.l[a][1] = 0; c.v[a][1] = q < nn[a];
        }
    }
    return c;
}

// setup.hip
int tables_words(int p, int q);
int compute_tables(int p, int q, hipStream_t s, double** d_tab, Tables* host);
// Operator with general material data on the box (kind PA_MAT_QP_ISO or PA_MAT_ANISO,
// data validated by the caller).
int create_material_op(const MeshDesc& md, int p, int q, int kind, const double* data, int dtype, hipStream_t s,
                       pa_op** out);
int compute_element_data(const MeshDesc& m, const double* d_vert, const double* d_lam, const double* d_mu,
                         int dtype, void* ed, hipStream_t s);
int launch_diagonal(const pa_op* op, void* d, int constrained);
int validate_mesh(const pa_mesh_t* m, MeshDesc* out);
// An operator on a validated mesh (also used for solver levels).  lin_mode: which kernel
// p = 1 applies run (kLinNever / kLinBySize / kLinAlways, see p1_runs_lin); the skeleton
// buffer is sized for it.
int create_op(const MeshDesc& md, int p, int q, const double* lam, const double* mu, int dtype, hipStream_t s,
              pa_op** out, int lin_mode = kLinBySize);
// geometry.hip
void element_map_coefficients(const double* const X[8], double* o);
int finish_geometry(pa_op* op, const std::vector<double>& coef, const double* lam, const double* mu);

int launch_rhs(const pa_op* op, const double f[3], int face, const double t[3], double* b, const double* d_vert);

// vec.hip
int launch_fill(void* y, int dtype, int64_t n, double v, hipStream_t s);
int launch_set_clamped(void* y, int dtype, const Geom& g, double v, hipStream_t s);
// Before the element kernel: y = 0 (add == 0) on free dofs; clamped dofs get y = x
// (add == 0) or y += x (add != 0).  With add != 0 and no clamp nothing is launched.
int launch_apply_prep(const void* x, void* y, int dtype, const Geom& g, int add, hipStream_t s);

// apply dispatch (api.hip)
// sk: skeleton buffer for this apply (nullptr: the operator's own)
int apply_op(const pa_op* op, const void* x, void* y, int flags, void* sk = nullptr);
// Look up the per-device address of the no-allocation scratch array (set-up).
int scratch_address(int dev, void** out);

}  // namespace pa
