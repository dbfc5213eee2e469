// Nonlocal pseudopotential term of H (Sec. 2 Eq. V_nl; Sec. 3.1 Eq.
// non-localPS:FD):  (V_nl y)(x) = sum_J sum_p chi_Jp(x) * h^3 gamma_Jp * (chi_Jp^T y).
//
// Two kernels:
//  * gather: per atom J, the projections S_Jp(c) = sum_{x in cube_J} chi_Jp(x) y(x,c)
//    as a small dense GEMM on the matrix cores, S_J^T (ns x nproj) =
//    Y_cube^T (ns x nbox) * chi_J (nbox x nproj), using
//    v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32).  The
//    cube's points (the K dimension) are split over kGatherSplit workgroups;
//    each writes its partial 16 x nproj tile.  No atomics: the partials are
//    summed in split order by the consumer.
//  * scatter: out(x,c) += alpha * sum_{J: x in cube_J} sum_p chi_Jp(x) h^3 gamma_Jp S_Jp(c)
//    over the unique nodes covered by at least one cube, grouped in blocks of
//    at most 256 nodes that touch at most kScatterSlots atoms (tables built at
//    operator creation).  A workgroup first finishes h^3 gamma S for its
//    block's atoms and eight columns into LDS (split partials summed in order),
//    then each thread updates one node for the eight columns, atoms in a fixed
//    order: deterministic even where cubes overlap.
//
// MFMA operand layout of the 16x16x4 instructions (64 lanes, lane = i + 16k,
// i in 0..15, k in 0..3): lane supplies A[i][k] (column c0+i at cube point
// k of the current group of 4) and B[k][j] (projector j at that point).  The
// FP32 accumulator keeps D[4*(lane/16) + r][lane%16] in register r; the FP64
// accumulator keeps D[lane/16 + 4*r][lane%16].
#include "nonlocal_kernel.hpp"

namespace sparc {

template <typename T, typename TI>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs<T, TI> g)
{
    __shared__ T tile[4][16][16];
    gather_item<T, TI>(g, blockIdx.x, blockIdx.y, blockIdx.z, tile, threadIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) scatter_kernel(const ScatterArgs<T> s)
{
    __shared__ T gl[kScatterSlots][kMaxProj][kScatterCols];
    scatter_item<T>(s, blockIdx.x, blockIdx.y, gl);
}

template <typename T, typename TI = T>
static int launch_gather_t(const sparc_op *op, const void *Y, int64_t ldy, int ns, void *part, hipStream_t stream,
                           const T *chi)
{
    GatherArgs<T, TI> a;
    a.Y = (const TI *)Y;
    a.ldy = ldy;
    a.ns = ns;
    a.nproj_total = op->nproj_total;
    a.atoms = op->d_atoms;
    a.box_off = op->d_box_off;
    a.chi = chi;
    a.part = (T *)part;
    dim3 grid(op->natoms, (ns + 15) / 16, kGatherSplit);
    ProfScope prof(1, stream);
    hipLaunchKernelGGL((gather_kernel<T, TI>), grid, dim3(256), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

int launch_gather_f32_to_f64(const sparc_op *op, const float *Y, int64_t ldy, int ns, double *part, hipStream_t stream)
{
    if (op->natoms == 0) return SPARC_OK;
    if ((long long)(ns + 15) / 16 > 65535) return fail(SPARC_E_SHAPE, "too many columns for one gather launch");
    return launch_gather_t<double, float>(op, Y, ldy, ns, part, stream, op->d_chi64);
}

int launch_gather(const sparc_op *op, int dtype, const void *Y, int64_t ldy, int ns, void *part, hipStream_t stream)
{
    if (op->natoms == 0) return SPARC_OK;
    if ((long long)(ns + 15) / 16 > 65535) return fail(SPARC_E_SHAPE, "too many columns for one gather launch");
    if (dtype == SPARC_F64) return launch_gather_t<double>(op, Y, ldy, ns, part, stream, op->d_chi64);
    return launch_gather_t<float>(op, Y, ldy, ns, part, stream, op->d_chi32);
}

template <typename T>
static int launch_scatter_t(const sparc_op *op, void *out, int64_t ldo, int ns, const void *part, double alpha,
                            hipStream_t stream, const T *chi, const T *hg)
{
    ScatterArgs<T> a;
    a.out = (T *)out;
    a.ldo = ldo;
    a.ns = ns;
    a.nproj_total = op->nproj_total;
    a.blk_pt = op->d_nl_blk_pt;
    a.blk_at = op->d_nl_blk_at;
    a.blk_atoms = op->d_nl_blk_atoms;
    a.pts = op->d_nl_pts;
    a.ent_off = op->d_nl_off;
    a.ent = (const int4 *)op->d_nl_ent;
    a.atoms = op->d_atoms;
    a.chi = chi;
    a.hg = hg;
    a.part = (const T *)part;
    a.alpha = (T)alpha;
    dim3 grid(op->nl_nblk, (ns + kScatterCols - 1) / kScatterCols);
    ProfScope prof(2, stream);
    hipLaunchKernelGGL(scatter_kernel<T>, grid, dim3(256), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

int launch_scatter(const sparc_op *op, int dtype, void *out, int64_t ldo, int ns, const void *part, double alpha,
                   hipStream_t stream)
{
    if (op->natoms == 0) return SPARC_OK;
    if ((ns + kScatterCols - 1) / kScatterCols > 65535) return fail(SPARC_E_SHAPE, "too many columns for one scatter launch");
    if (dtype == SPARC_F64) return launch_scatter_t<double>(op, out, ldo, ns, part, alpha, stream, op->d_chi64, op->d_hg64);
    return launch_scatter_t<float>(op, out, ldo, ns, part, alpha, stream, op->d_chi32, op->d_hg32);
}

}  // namespace sparc
