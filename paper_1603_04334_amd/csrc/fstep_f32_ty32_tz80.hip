// Vector step kernels for float blocks on patches of 32 x 80 nodes (see fstep.hip).
#include "fstep_launch.hpp"

namespace sparc {

int fstep_f32_ty32_tz80(const FStepArgs<float> &a, const GatherArgs<float, float> &g, int natoms, int ncb, int nitems, int ngb,
                        bool prev, bool strm, int cblk, hipStream_t s)
{
    return fstep_dispatch<float, 32, 80>(a, g, natoms, ncb, nitems, ngb, prev, strm, cblk, s);
}

}  // namespace sparc
