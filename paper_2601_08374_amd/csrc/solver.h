// Solver-side declarations shared by gmg.hip and solver_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace pa {

constexpr int kReduceBlocks = 512;   // fixed stage-1 grid of every reduction (deterministic sums)

// Operations of the final reduction stage.
enum { FIN_STORE = 0, FIN_ALPHA = 1, FIN_BETA = 2 };

// Device scalar slots of a solve (FP64).
enum {
    S_RZ = 0, S_RZ0, S_PAP, S_ALPHA, S_BETA, S_DONE, S_ITERS, S_CRIT, S_RTOL, S_STOP, S_BB, S_RRLAST,
    S_T0 = 16, S_T1 = 17,      // scratch pair for FIN_STORE
    S_NR = 20, S_NR1 = 21,     // |r|^2 of the refinement residual
    S_NB = 22, S_NB1 = 23,     // |b|^2
    S_ONE = 24,                // constant 1.0 (plain casts through launch_cast_scale)
    S_COUNT = 32
};

// Per-axis h-transfer tables (device pointers).
struct HAxis {
    const int* i0;      // [nf+1] first coarse vertex of fine vertex g
    const int* i1;      // [nf+1] second coarse vertex (== i0 when coincident)
    const double* t;    // [nf+1] weight of i1 (weight of i0 is 1-t)
    const int* fi;      // [nc+1][3] fine vertices touching coarse vertex j
    const double* fw;   // [nc+1][3] their weights (0 pads)
};

int launch_dot(const void* a, const void* b, const void* c, int dtype, int64_t n, double* part, hipStream_t s);
int launch_dot_final(const double* part, double* scal, int op, int slot, hipStream_t s);
int launch_pcg_init(const double* part, double* scal, double rtol, int stop, hipStream_t s);
// Power-iteration pass: z = dinv w and the stage-1 sums of v.w, v.Dv (part, part + nb) and z.z
// (part + 2 nb, with zeros at part + 3 nb); part holds 4 kReduceBlocks doubles.
int launch_power_pass(const void* v, const void* w, const void* dinv, void* z, int dtype, int64_t n, double* part,
                      hipStream_t s);
int launch_pcg_xr(void* x, void* r, const void* p, const void* Ap, const double* sc, int dtype, int64_t n,
                  hipStream_t s);
int launch_pcg_p(void* p, const void* z, const double* sc, int dtype, int64_t n, hipStream_t s);
int launch_residual(void* r, const void* b, const void* Ax, int dtype, int64_t n, hipStream_t s);
int launch_copy(void* y, const void* x, int dtype, int64_t n, hipStream_t s);
int launch_cast_scale(void* y, int dty, const void* x, int dtx, const double* sc, int slot, int inv_sqrt, int64_t n,
                      hipStream_t s);
int launch_ir_update(double* x, const void* d, int dtd, const double* sc, int slot, int64_t n, hipStream_t s);
int launch_cheb_step(void* x, void* r, const void* t, void* d, const void* dinv, double c1, double c2, bool x_zero,
                     bool last, int dtype, int64_t n, hipStream_t s);
int launch_cheb_start(void* r, void* d, const void* dinv, const void* b, const void* t, double c, int dtype,
                      int64_t n, hipStream_t s);
int launch_add(void* y, const void* x, int dtype, int64_t n, hipStream_t s);
int launch_reciprocal(void* y, int dtype, int64_t n, hipStream_t s);
int launch_splitmix(void* v, int dtype, uint64_t seed, int64_t n, hipStream_t s);
int launch_p_interp_matrix(const double* gll_c, const double* gll_f, int pc, int pf, double* I, hipStream_t s);
int launch_p_prolong(const void* xc, void* xf, const double* I, int pc, int pf, const Geom& gc, const Geom& gf,
                     int add, int dtype, hipStream_t s);
int launch_p_restrict(const void* rf, const void* tf, void* rc, void* skr, const double* I, int pc, int pf,
                      const Geom& gc, const Geom& gf, int dtype, hipStream_t s);
int launch_h_prolong(const void* xc, void* xf, const HAxis ax[3], const Geom& gc, const Geom& gf, int add, int dtype,
                     hipStream_t s);
int launch_h_restrict(const void* rf, const void* tf, void* rc, const HAxis ax[3], const Geom& gc, const Geom& gf, int dtype,
                      hipStream_t s);
int launch_coarse_assemble(double* A, int N, const pa_op* op, hipStream_t s);
// Blocked Gauss-Jordan inverse of the SPD coarse matrix in place; work holds
// coarse_invert_words(N) doubles.
constexpr int kGjNB = 32;
int64_t coarse_invert_words(int N);
int coarse_invert(double* A, double* work, int N, hipStream_t s);
int launch_dense_cast(void* out, int dtype, const double* in, int64_t n, hipStream_t s);
int launch_dense_matvec(const void* Ai, const void* x, void* y, int N, int dtype, hipStream_t s);

}  // namespace pa
