// Fused apply instantiations for polynomial degree p = 2 (q = p+1, p+2, p+3; FP64 and FP32).
#include "apply_kernel.h"

namespace pa {
int launch_apply_p2(const ApplyLaunch& L, int q_off, int dtype) { return launch_apply_p<2>(L, q_off, dtype); }
}  // namespace pa
