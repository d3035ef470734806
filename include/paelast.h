/*
 * paelast.h -- C ABI of the MI355X (gfx950) matrix-free high-order
 * linear-elasticity library: the partial-assembly (PA) operator apply on
 * affine tensor-product hexahedra and the geometric-multigrid-preconditioned
 * CG solver built around it.
 *
 * Paper: "Shifting the Sweet Spot: High-Performance Matrix-Free Method for
 * High-Order Elasticity" (arXiv 2601.08374).  Section/equation citations below
 * refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Plain C types only; the library never aborts and never prints.  Every call
 *   returns PA_OK (0) or a negative error code; pa_last_error() gives a
 *   thread-local message for the last failure on the calling thread.
 * - Meshes are structured boxes of n[0] x n[1] x n[2] hexahedra (Sec. 5.1.4
 *   uses an 8x1x1 structured hex block; Sec. 4.4 assumes affine elements, so
 *   J^{-1} and det J are constant per element).  Reference vertex coordinates
 *   along axis a are grade[a] (n[a]+1 strictly increasing values) or uniform on
 *   [0, L[a]]; the physical point is A X + x0 with det A > 0.
 * - Element numbering: e = ex + n0*(ey + n1*ez).
 * - Degrees of freedom (the paper leaves the global order open): nodes lie on
 *   the (n0 p+1) x (n1 p+1) x (n2 p+1) grid of per-element Gauss-Lobatto
 *   points, node = gx + (n0 p+1)*(gy + (n1 p+1)*gz); a vector of N = 3*Nn
 *   entries stores component c of node at c*Nn + node ("by nodes").
 * - Device pointers are HIP device allocations owned by the caller (e.g.
 *   torch tensors); host pointers are read during the call only.  Work is
 *   enqueued on the operator's HIP stream; calls marked "async" return before
 *   the device finishes.
 * - clamped_faces bitmask: bit0 x-, bit1 x+, bit2 y-, bit3 y+, bit4 z-, bit5 z+.
 *   Clamped nodes carry homogeneous Dirichlet data on all three components
 *   (Sec. 5.1.4: u = 0 on the clamped end).
 */
#ifndef PAELAST_H
#define PAELAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define PA_OK 0
#define PA_EINVAL (-1)        /* bad argument (NULL, out of range, aliasing, det <= 0, ...) */
#define PA_ENOMEM (-2)        /* a device or host allocation failed                         */
#define PA_EUNSUPPORTED (-3)  /* valid but not built (e.g. p > 8)                           */
#define PA_EHIP (-4)          /* a HIP runtime call failed                                  */
#define PA_ENOCONV (-5)       /* iteration cap reached; x holds the last iterate            */
#define PA_EBREAKDOWN (-6)    /* CG breakdown (p^T A p <= 0 or NaN)                         */

/* ---- element types -------------------------------------------------------- */
#define PA_F64 0
#define PA_F32 1

/* ---- apply flags ---------------------------------------------------------- */
#define PA_UNCONSTRAINED 1    /* ignore clamped faces: y = A x                               */
#define PA_ADD 2              /* accumulate: y += A x instead of y = A x                      */

/* ---- material data forms (pa_elast_setup_material) ---------------------------- */
#define PA_MAT_ELEM_ISO 0   /* lambda, mu per element (pa_elast_setup)                           */
#define PA_MAT_QP_ISO 1     /* lambda, mu per element and quadrature point                         */
#define PA_MAT_ANISO 2      /* symmetric 6x6 Voigt stiffness per element                          */

/* ---- element geometry forms (pa_elast_setup_geometry) ------------------------ */
#define PA_GEOM_AFFINE 0     /* the box map of pa_mesh_t (pa_elast_setup)                         */
#define PA_GEOM_QP_DATA 1    /* trilinear hexahedra, J^{-1} and w det J stored per quadrature point */
#define PA_GEOM_TRILINEAR 2  /* trilinear hexahedra, Jacobian recomputed per point (21 words/elem)  */

/* ---- apply variants (pa_elast_apply_variant) -------------------------------- */
#define PA_VARIANT_FUSED 0            /* the production apply (pa_elast_apply_ex)                  */
#define PA_VARIANT_UNFUSED_DENSE 1    /* three passes, dense gradient/action, full-tensor stress   */
#define PA_VARIANT_UNFUSED_SF 2       /* three passes, sum-factorized gradient/action              */
#define PA_VARIANT_UNFUSED_SF_VOIGT 3 /* as 2 with the Voigt stress form                           */
#define PA_VARIANT_FUSED_UNSTAGED 4   /* the three passes of 3 fused into one kernel per element,
                                         quadrature-point data staged per element (Alg. 2)     */
#define PA_VARIANT_FUSED_QUADRATURE 5 /* the fused, register/LDS-staged kernel with its pointwise
                                         stage at the q^3 Gauss points (no collocation)         */

/* ---- solver modes / stopping tests ----------------------------------------- */
#define PA_SOLVE_F64 0        /* FP64 PCG with an FP64 V-cycle                                */
#define PA_SOLVE_F32_IR 1     /* FP64 iterative refinement around an FP32 PCG + FP32 V-cycle  */
#define PA_SOLVE_F32_PREC 2   /* FP64 PCG (FP64 apply, residual, dots) preconditioned by the
                                 FP32 V-cycle (FP32 applies, smoothers, transfers)              */
#define PA_STOP_PREC 0        /* sqrt(r.Br / r0.Br0) <= rtol (preconditioned norm)            */
#define PA_STOP_TRUE 1        /* |b - A x|_2 / |b|_2 <= rtol (true residual)                  */

typedef struct pa_mesh_t {
    int32_t n[3];             /* elements per axis, each >= 1                                  */
    double L[3];              /* box lengths when grade[a] == NULL                             */
    double A[9];              /* global affine map, row-major, det > 0                         */
    double x0[3];             /* translation (does not change the operator)                    */
    const double* grade[3];   /* optional host arrays of n[a]+1 increasing vertex coordinates  */
    uint32_t clamped_faces;   /* Dirichlet faces, bitmask as above                             */
} pa_mesh_t;

typedef struct pa_op pa_op_t;
typedef struct pa_gmg pa_gmg_t;
typedef struct pa_solve pa_solve_t;

typedef struct pa_solve_opts_t {
    int mode;                 /* PA_SOLVE_F64, PA_SOLVE_F32_IR or PA_SOLVE_F32_PREC            */
    int stop;                 /* PA_STOP_PREC or PA_STOP_TRUE                                  */
    int p_levels;             /* number of p-coarsenings p -> p/2 -> ... (-1: down to p = 1)   */
    int h_levels;             /* number of h-coarsenings at p = 1 (-1: automatic)              */
    int cheb_degree;          /* Chebyshev degree k (Sec. 3.1 uses 2)                          */
    int power_iters;          /* power iterations for lambda_max (Sec. 3.1 uses 10)            */
    double cheb_lo_frac;      /* smoothing interval [lo_frac*lmax, lmax] (default 0.1)         */
    double cheb_safety;       /* lmax = safety * estimate                                      */
    int max_iter;             /* outer PCG iteration cap (Sec. 3.2: 5000)                      */
    double inner_rtol;        /* PA_SOLVE_F32_IR: inner FP32 PCG tolerance (default 3e-3)      */
    int inner_max_iter;       /* PA_SOLVE_F32_IR: inner iteration cap                          */
    int max_outer;            /* PA_SOLVE_F32_IR: refinement step cap                          */
    uint64_t seed;            /* power-iteration start vector (SplitMix64 stream)              */
    int coarse_max_dofs;      /* automatic h-coarsening stops at or below this size            */
    const double* lambda_max; /* optional host array, one per level (finest first): overrides
                                 the power-iteration estimate when > 0                         */
} pa_solve_opts_t;

typedef struct pa_solve_info_t {
    int iters;                /* total (inner) PCG iterations                                  */
    int outer_iters;          /* refinement steps (PA_SOLVE_F32_IR), else 0                    */
    double rel_res_true;      /* |b - A x|_2 / |b|_2 of the returned x, FP64 apply             */
    double rel_res_prec;      /* last sqrt(r.Br / r0.Br0)                                      */
    double t_setup;           /* seconds spent building the hierarchy in this call             */
    double t_solve;           /* seconds in the iteration                                      */
    int num_levels;
} pa_solve_info_t;

/* Fill *o with the defaults: F64, PA_STOP_PREC, full p-hierarchy, automatic h,
 * k = 2, 10 power iterations, interval [0.1, 1] * 1.2 * estimate, 5000 iterations,
 * inner rtol 3e-3 / 50 iterations, 20 refinement steps, seed 7, coarse <= 3000 dofs. */
void pa_solve_opts_default(pa_solve_opts_t* o);

/* ---- operator --------------------------------------------------------------- */

/* Partial assembly (Sec. 2.2.2, Sec. 4.4): stores per element the constant
 * J^{-1}, det J * lambda_e and det J * mu_e (computed on the device from the
 * mesh description), plus the 1D basis tables B (values) and G (derivatives)
 * of the (p+1) Gauss-Lobatto Lagrange polynomials at the q Gauss-Legendre
 * points and the q weights (also computed on the device).
 * p in [1,8]; q in [p+1, p+3] (Sec. 5.1.4 uses q = p+2; the operator is exact,
 * hence q-independent, for q >= p+1 on affine elements).  lambda, mu: host
 * arrays of n0*n1*n2 per-element Lame parameters (mu > 0, lambda + 2mu/3 > 0).
 * dtype PA_F64 or PA_F32 selects the element type of applies.  hip_stream may
 * be NULL (default stream).  Errors: PA_EINVAL, PA_EUNSUPPORTED, PA_ENOMEM,
 * PA_EHIP. On success *out owns all device memory; free with pa_elast_destroy. */
int pa_elast_setup(const pa_mesh_t* m, int p, int q, const double* lambda, const double* mu,
                   int dtype, void* hip_stream, pa_op_t** out);
/* The operator with general material data (Sec. 2.1 eq. 2; the paper's PA data holds
 * the material at every quadrature point, Sec. 4.5).  kind = PA_MAT_QP_ISO: data is a
 * host array [NE][q^3][2] of (lambda, mu) per element and Gauss-Legendre point, point
 * (qx, qy, qz) at qx + q (qy + q qz), each with mu > 0 and lambda + 2 mu / 3 > 0.
 * kind = PA_MAT_ANISO: data is a host array [NE][21], the upper triangle (row by row)
 * of the symmetric positive definite Voigt stiffness C in sigma_V = C eps_V with
 * eps_V = (e_xx, e_yy, e_zz, 2 e_yz, 2 e_xz, 2 e_xy).  The data is copied.  q must be
 * p + 2 (PA_EUNSUPPORTED otherwise); other arguments and errors as pa_elast_setup
 * (PA_EINVAL for a point or element that violates the conditions above).  apply and
 * rhs work as for pa_elast_setup operators, and so do pa_elast_diagonal, gmg_setup
 * and gmg_pcg_solve: the finest level keeps the material data (the library keeps a
 * host copy of it to build that level in the solver's precision); coarser levels
 * take per-element isotropic parameters, the quadrature-weighted element means of
 * per-point lambda and mu, or for an anisotropic C the isotropic stiffness with the
 * same traces of its normal and shear blocks (mu = (C44 + C55 + C66) / 3, 9 lambda +
 * 6 mu = the sum of the normal block).  A hierarchy with no level below the finest
 * returns PA_EUNSUPPORTED (its coarse matrix is assembled from per-element
 * parameters). */
int pa_elast_setup_material(const pa_mesh_t* m, int p, int q, int kind, const double* data, int dtype,
                            void* hip_stream, pa_op_t** out);
/* The operator on non-affine (trilinear) hexahedra.  The paper's kernels take affine
 * elements with J^{-1} and det J constant per element (Sec. 4.4) and name non-affine
 * geometry, with its trade-off between stored quadrature data and recomputation, as
 * future work (Sec. 6); both sides of that trade-off are built here.  vertices is a host
 * array [(n0+1)(n1+1)(n2+1)][3] of physical vertex positions, vertex (i, j, k) at
 * i + (n0+1)(j + (n1+1)k); element (ex, ey, ez) is the trilinear image of [0,1]^3
 * through its 8 vertices (ex+a, ey+b, ez+c).  m supplies n and clamped_faces (the faces
 * of index-space boundaries); its box fields must be valid but do not enter the operator.
 * kind = PA_GEOM_QP_DATA stores (J^{-1}, w det J) at every Gauss-Legendre point (10 words
 * per point, the partial-assembly form); kind = PA_GEOM_TRILINEAR stores the 21
 * coefficients of each element's map and recomputes J, det J and J^{-1} per point inside
 * the apply.  q must be p + 2 (PA_EUNSUPPORTED otherwise).  lambda, mu as pa_elast_setup.
 * PA_EINVAL if a vertex is not finite or det J <= 0 at a quadrature point of an element.
 * apply works as for pa_elast_setup operators; pa_elast_diagonal, pa_elast_rhs,
 * gmg_setup, gmg_pcg_solve and the unfused apply variants return PA_EUNSUPPORTED. */
int pa_elast_setup_geometry(const pa_mesh_t* m, const double* vertices, int kind, int p, int q,
                            const double* lambda, const double* mu, int dtype, void* hip_stream, pa_op_t** out);
/* The operator on an unstructured hexahedral mesh given by an explicit element-to-node
 * map (the box of pa_elast_setup generalised; elements in any order and orientation).
 * vertices: host [num_vertices][3] positions; elem_vertices: host [num_elements][8]
 * vertex indices, local vertex a + 2(b + 2c) at reference corner (a, b, c) of [0,1]^3
 * (the element is the trilinear image of [0,1]^3; its Jacobian is recomputed at every
 * point as for PA_GEOM_TRILINEAR); elem_nodes: host [num_elements][(p+1)^3] global node
 * of local node ix + (p+1)(iy + (p+1) iz), nodes at the GLL points of the element's
 * reference axes; clamped: host [num_nodes] flags of the essential nodes (all three
 * components), or NULL.  Dofs are component blocks c*num_nodes + node.  The map must be
 * conforming: a local node strictly inside an element belongs to no other element
 * (PA_EINVAL otherwise, as for an index out of range, a node listed twice in one element,
 * a non-finite vertex or det J <= 0 at a quadrature point).  The arrays are copied.
 * q must be p + 2 (PA_EUNSUPPORTED otherwise); lambda, mu per element as pa_elast_setup.
 * Element-boundary contributions are summed per node in a fixed order (deterministic).
 * apply works as for pa_elast_setup operators; pa_elast_diagonal, pa_elast_rhs,
 * gmg_setup, gmg_pcg_solve and the unfused apply variants return PA_EUNSUPPORTED. */
int pa_elast_setup_unstructured(int64_t num_vertices, const double* vertices, int64_t num_elements,
                                const int32_t* elem_vertices, int64_t num_nodes, const int32_t* elem_nodes,
                                const uint8_t* clamped, int p, int q, const double* lambda, const double* mu,
                                int dtype, void* hip_stream, pa_op_t** out);
void pa_elast_destroy(pa_op_t* op);
int pa_elast_set_stream(pa_op_t* op, void* hip_stream);
/* N = 3 * number of nodes. */
int pa_elast_ndofs(const pa_op_t* op, int64_t* n);
/* Device bytes an operator (with_solver = 0) or an operator plus a default GMG
 * solver hierarchy and its work vectors (with_solver = 1) needs; used for
 * admission by HBM budget.  with_solver models PA_SOLVE_F64 for dtype PA_F64
 * (an upper bound for PA_SOLVE_F32_PREC, whose levels are FP32) and
 * PA_SOLVE_F32_IR for dtype PA_F32.  Returns a negative error code on bad input. */
int64_t pa_bytes_required(const pa_mesh_t* m, int p, int dtype, int with_solver);

/* y = A x (async).  The fused kernel gathers each element's dofs (the
 * restriction G), interpolates displacement gradients to the quadrature points
 * by sum factorization (Sec. 4.4: X, Y, Z contractions with B and G, then
 * J^{-T}), forms the Voigt stress with the weighted Lame parameters (eq. 7 and
 * Sec. 4.5), reconstructs Q = sigma J^{-T} (Sec. 4.5, backward
 * reconstruction), contracts back with the transposed sweeps (Sec. 4.5) and
 * scatter-adds (G^T).  On affine elements with per-element Lame parameters the
 * same sums of the q-point rule are evaluated regrouped: at p >= 2 the pointwise
 * stage runs at the (p+1)^3 Gauss-Lobatto nodes, where the gradient, the stress and
 * Q are exactly their polynomial interpolants, and the rule enters through its
 * 1D mass matrices; at p = 1 a closed form from the rule's centred moments.  The
 * results equal the point-by-point sums up to rounding.
 * x, y: device arrays of N elements of the op's dtype;
 * x is not modified; x == y is PA_EINVAL.  With clamped faces this is the
 * constrained operator: clamped entries of x are treated as zero and y equals
 * x on them (identity rows and columns).  No allocation. */
int pa_elast_apply(pa_op_t* op, const void* x, void* y);
/* As pa_elast_apply with flags PA_UNCONSTRAINED and/or PA_ADD (async). */
int pa_elast_apply_ex(pa_op_t* op, const void* x, void* y, int flags);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pa_elast_apply_ex with the
 * same kernels and results, whose element-boundary partial sums go to a static
 * per-device scratch array of PA_NOALLOC_SCRATCH_BYTES bytes inside the library
 * instead of the operator's buffer.  The call itself allocates nothing.  The array
 * is set up when the first operator is created on a device (pa_elast_setup and the
 * other setup calls) and stays allocated on every device the library runs on until
 * the process ends.  Every operator whose element-boundary buffer fits is accepted;
 * larger ones return PA_EINVAL with a message naming both sizes (at FP64, the
 * sheared-box sweep of ~4.2M dofs fits at p = 1 and p >= 4).  Nothing in the array
 * has to start at zero: an apply writes every entry it reads.  All calls on one
 * device share the array and keep the last call's contents, so calls that overlap
 * in time on one device (other streams, other host threads) race: serialise them.
 * Flags, errors and stream as pa_elast_apply_ex (async). */
#define PA_NOALLOC_SCRATCH_BYTES (64u << 20)
int pa_elast_apply_noalloc(pa_op_t* op, const void* x, void* y, int flags);

/* The same operator in the earlier forms of the paper's cumulative ablation
 * (Sec. 4.1-4.4, ablation table; baseline dataflow Alg. 1): a gradient pass, a
 * stress pass and an action pass with operator-wide quadrature-point arrays in
 * device memory between them, then a fixed-order assembly; PA_VARIANT_FUSED_UNSTAGED
 * runs the sum-factorized passes and the Voigt stress in one kernel (macro-kernel
 * fusion, Sec. 4.2, Alg. 2), each workgroup staging its elements' quadrature-point
 * data (9 words per point) in its own part of a work array, then the same
 * assembly -- PA_VARIANT_FUSED_QUADRATURE adds the slice-wise organisation (Sec. 4.5):
 * the production kernel with the pointwise stage at the q^3 Gauss points, and the
 * production apply evaluates the same sums in regrouped form (p = 1: closed form from
 * the rule's centred moments; p >= 2: the pointwise stage at the (p+1)^3 Gauss-Lobatto
 * nodes, exact for affine elements with per-element Lame data).  For measurement;
 * results equal pa_elast_apply_ex up to rounding.  FP64 operators with q = p+2
 * only (PA_EUNSUPPORTED otherwise); flags 0 or PA_UNCONSTRAINED (y is
 * overwritten).  The first call on an operator allocates its work arrays
 * (2 x 72 NE q^3 + 24 NE (p+1)^3 bytes and the dense basis-gradient table; freed
 * by pa_elast_destroy; PA_ENOMEM if they do not fit).  Asynchronous on the
 * operator's stream.  PA_VARIANT_FUSED runs pa_elast_apply_ex. */
int pa_elast_apply_variant(pa_op_t* op, const void* x, void* y, int flags, int variant);
/* d = diag(A) (async), the Jacobi diagonal of Sec. 3.1, from 1D-factorized
 * integrals of products of reference derivatives (per-point Lame data: the
 * quadrature sum over the element's points; anisotropic C: the same 1D-factorized
 * integrals contracted with C).  Constrained unless flags has PA_UNCONSTRAINED (then
 * clamped entries hold the true diagonal; otherwise 1).  d: device array of N
 * elements of the op's dtype.  PA_EUNSUPPORTED for non-affine or unstructured
 * operators. */
int pa_elast_diagonal(pa_op_t* op, void* d, int flags);

/* b = load vector of eq. 4 (async): integral of f.v over the box plus integral
 * of t.v over face traction_face (0..5, or -1 for none), f and t constant host
 * 3-vectors.  Clamped entries of b are set to 0.  b: device FP64 array of N. */
int pa_elast_rhs(pa_op_t* op, const double f[3], int traction_face, const double t[3], double* b);

/* ---- geometric multigrid (Sec. 3) ------------------------------------------ */

/* Build the hierarchy of Sec. 3: p-levels p -> floor(p/2) -> ... (polynomial
 * interpolation transfers), then h-coarsenings at p = 1 (each axis with n > 1
 * merges element pairs, natural injection), clamped faces on every level,
 * diag(A) and lambda_max(D^{-1}A) by power iteration per level, and an exact
 * coarse solve (the inverse of the assembled coarsest constrained matrix,
 * formed on the device).  Level 0 is the finest.  Synchronizes the stream. */
int gmg_setup(pa_op_t* op, const pa_solve_opts_t* o, pa_gmg_t** out);
void gmg_destroy(pa_gmg_t* g);
int gmg_num_levels(const pa_gmg_t* g);
/* n[3], p, N, dtype (PA_F32 in PA_SOLVE_F32_IR mode) and the Chebyshev
 * lambda_max (after the safety factor) of a level. Any output may be NULL. */
int gmg_level_info(const pa_gmg_t* g, int level, int32_t n[3], int* p, int64_t* ndofs, int* dtype,
                   double* lambda_max);
/* Level operator (borrowed; valid until gmg_destroy). */
int gmg_level_op(pa_gmg_t* g, int level, pa_op_t** op);
/* Fine vector of level `level` from the coarse vector of level `level+1` (async):
 * xf = P xc, clamped entries zeroed.  Arrays of the level's dtype. */
int gmg_prolong(pa_gmg_t* g, int level, const void* xc, void* xf);
/* Coarse vector of level `level+1` from level `level` (async): rc = P^T rf,
 * clamped entries zeroed. */
int gmg_restrict(pa_gmg_t* g, int level, const void* rf, void* rc);
/* k steps of Chebyshev-Jacobi smoothing on level `level` for A x = b (async),
 * from x (x_is_zero != 0: x is taken as 0 and overwritten). */
int gmg_smooth(pa_gmg_t* g, int level, const void* b, void* x, int x_is_zero);
/* x = A_c^{-1} b on the coarsest level (async). */
int gmg_coarse_solve(pa_gmg_t* g, const void* b, void* x);
/* z = B r, one V(1,1)-cycle from level 0 (async), in the hierarchy's dtype. */
int gmg_vcycle(pa_gmg_t* g, const void* r, void* z);

/* Solve A x = b by GMG-preconditioned CG (Sec. 3.2) to rtol with the hierarchy
 * g; b, x FP64 device arrays (x is the initial guess).  PA_SOLVE_F32_IR runs
 * FP64 refinement steps r = b - A x, x += |r| d with d from an FP32 PCG +
 * FP32 V-cycle on A d = r/|r| (FP64 dot products).  Synchronous.
 * Returns PA_OK, PA_ENOCONV or PA_EBREAKDOWN; info may be NULL. */
int gmg_pcg_run(pa_gmg_t* g, const double* b, double* x, double rtol, pa_solve_info_t* info);

/* One-call solve on an operator: builds (and caches on op) the hierarchy for opts o
 * (NULL: defaults), then runs gmg_pcg_run. */
int gmg_pcg_solve(pa_op_t* op, const double* b, double* x, double rtol, const pa_solve_opts_t* o,
                  pa_solve_info_t* info);

/* Step API for interleaving many solves on one device (no host threads per
 * solve).  begin: initial residual and first preconditioner application are
 * enqueued; step: enqueue up to n_iters more iterations (async), return at
 * once; poll: *done = 1 once the device reached the stopping test or an error
 * (then *status holds PA_OK / PA_ENOCONV / PA_EBREAKDOWN), 0 while work is in
 * flight or more steps are needed; end: wait, fill info, free the state. */
int gmg_pcg_begin(pa_gmg_t* g, const double* b, double* x, double rtol, pa_solve_t** s);
int gmg_pcg_step(pa_solve_t* s, int n_iters);
int gmg_pcg_poll(pa_solve_t* s, int* done, int* status);
int gmg_pcg_end(pa_solve_t* s, pa_solve_info_t* info);

/* ---- measurement ------------------------------------------------------------ */
/* Attainable vector FMA rate (a measured ceiling beside the published peak, for the
 * roofline of the apply kernels; not part of the method).  Launches blocks x 256
 * lanes on hip_stream, each running 8 independent chains of iters dependent FMAs in
 * dtype (PA_F64 / PA_F32, non-packed), i.e. 4096 * blocks * iters FLOPs, and writes
 * one value per lane to out, a device array of blocks * 256 words of dtype owned by
 * the caller.  Asynchronous; time it with events on the same stream.  PA_EINVAL for
 * out == NULL, another dtype, blocks < 1 or iters < 1. */
int pa_probe_fma(void* out, int dtype, int blocks, int iters, void* hip_stream);

/* ---- errors ----------------------------------------------------------------- */
const char* pa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PAELAST_H */
