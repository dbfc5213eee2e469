// Instantiation of the FP64 step on FP32 blocks (values widened as they are
// loaded), used by the Rayleigh-Ritz product H Y (see stencil.hip).
#include "step_launch.hpp"

namespace sparc {

int launch_step_mixed(const sparc_op *op, const float *yk, int64_t ldk, double *out, int64_t ldo, int ns,
                      const StepCoef &c, const StepLaunch &L, hipStream_t stream)
{
    return launch_step_t<double, float>(op, yk, ldk, nullptr, 0, out, ldo, ns, c, L, stream, op->d_veff64);
}

}  // namespace sparc
