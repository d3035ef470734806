// Geometric multigrid: placeholder entry points until the hierarchy lands.
#include "internal.h"

using namespace pa;
extern "C" {
int gmg_setup(pa_op_t*, const pa_solve_opts_t*, pa_gmg_t**) { return fail(PA_EUNSUPPORTED, "gmg not built"); }
void gmg_destroy(pa_gmg_t*) {}
int gmg_num_levels(const pa_gmg_t*) { return 0; }
int gmg_level_info(const pa_gmg_t*, int, int32_t*, int*, int64_t*, int*, double*) { return PA_EUNSUPPORTED; }
int gmg_level_op(pa_gmg_t*, int, pa_op_t**) { return PA_EUNSUPPORTED; }
int gmg_prolong(pa_gmg_t*, int, const void*, void*) { return PA_EUNSUPPORTED; }
int gmg_restrict(pa_gmg_t*, int, const void*, void*) { return PA_EUNSUPPORTED; }
int gmg_smooth(pa_gmg_t*, int, const void*, void*, int) { return PA_EUNSUPPORTED; }
int gmg_coarse_solve(pa_gmg_t*, const void*, void*) { return PA_EUNSUPPORTED; }
int gmg_vcycle(pa_gmg_t*, const void*, void*) { return PA_EUNSUPPORTED; }
int gmg_pcg_run(pa_gmg_t*, const double*, double*, double, pa_solve_info_t*) { return PA_EUNSUPPORTED; }
int gmg_pcg_solve(pa_op_t*, const double*, double*, double, const pa_solve_opts_t*, pa_solve_info_t*) { return PA_EUNSUPPORTED; }
int gmg_pcg_begin(pa_gmg_t*, const double*, double*, double, pa_solve_t**) { return PA_EUNSUPPORTED; }
int gmg_pcg_step(pa_solve_t*, int) { return PA_EUNSUPPORTED; }
int gmg_pcg_poll(pa_solve_t*, int*, int*) { return PA_EUNSUPPORTED; }
int gmg_pcg_end(pa_solve_t*, pa_solve_info_t*) { return PA_EUNSUPPORTED; }
int64_t pa_bytes_required(const pa_mesh_t*, int, int, int) { return PA_EUNSUPPORTED; }
}
