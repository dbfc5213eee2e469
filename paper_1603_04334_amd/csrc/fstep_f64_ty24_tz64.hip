// Vector step kernels for double blocks on patches of 24 x 64 nodes (see fstep.hip).
#include "fstep_launch.hpp"

namespace sparc {

int fstep_f64_ty24_tz64(const FStepArgs<double> &a, const GatherArgs<double, double> &g, int natoms, int ncb, int nitems, int ngb,
                        bool prev, bool strm, int cblk, hipStream_t s)
{
    return fstep_dispatch<double, 24, 64>(a, g, natoms, ncb, nitems, ngb, prev, strm, cblk, s);
}

}  // namespace sparc
