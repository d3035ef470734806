// Fused apply instantiations for polynomial degree p = 3 (q = p+1, p+2, p+3; FP64 and FP32).
#include "apply_kernel.h"

namespace pa {
int launch_apply_p3(const ApplyLaunch& L, int q_off, int dtype) { return launch_apply_p<3>(L, q_off, dtype); }
}  // namespace pa
