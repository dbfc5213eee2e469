// Vector step kernels for double blocks on patches of 16 x 64 nodes (see fstep.hip).
#include "fstep_launch.hpp"

namespace sparc {

int fstep_f64_ty16_tz64(const FStepArgs<double> &a, const GatherArgs<double, double> &g, int natoms, int ncb, int nitems, int ngb,
                        bool prev, bool strm, int cblk, hipStream_t s)
{
    return fstep_dispatch<double, 16, 64>(a, g, natoms, ncb, nitems, ngb, prev, strm, cblk, s);
}

}  // namespace sparc
