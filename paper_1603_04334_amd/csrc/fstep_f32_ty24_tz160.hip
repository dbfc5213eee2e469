// Vector step kernels for float blocks on patches of 24 x 160 nodes (see fstep.hip).
#include "fstep_launch.hpp"

namespace sparc {

int fstep_f32_ty24_tz160(const FStepArgs<float> &a, const GatherArgs<float, float> &g, int natoms, int ncb, int nitems, int ngb,
                        bool prev, bool strm, int cblk, hipStream_t s)
{
    return fstep_dispatch<float, 24, 160>(a, g, natoms, ncb, nitems, ngb, prev, strm, cblk, s);
}

}  // namespace sparc
