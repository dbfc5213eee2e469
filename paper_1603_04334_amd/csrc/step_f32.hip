// Instantiation of the fused step launches for float blocks (see stencil.hip).
#include "step_launch.hpp"

namespace sparc {

int launch_step_f32(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp, void *out,
                    int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream, void *part)
{
    return launch_step_t<float>(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, op->d_veff32, part, op->d_chi32);
}

}  // namespace sparc
