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
//    operator creation).  A workgroup first requests its nodes' out values for
//    32 FP32 / 8 FP64 columns (8 when the block tables are too large for
//    LDS), finishes h^3 gamma S for its block's atoms and those columns into
//    LDS (split partials summed in order), then each thread updates one node
//    for all of them, atoms in a fixed order: deterministic even where cubes
//    overlap.  The cube rows are short (a few tens of bytes per column), so
//    the kernel's HBM traffic is set by partial lines and its time by the
//    scattered read-modify-write of out, not by the table or chi reads.
//
// MFMA operand layout of the 16x16x4 instructions (64 lanes, lane = i + 16k,
// i in 0..15, k in 0..3): lane supplies A[i][k] (column c0+i at cube point
// k of the current group of 4) and B[k][j] (projector j at that point).  The
// FP32 accumulator keeps D[4*(lane/16) + r][lane%16] in register r; the FP64
// accumulator keeps D[lane/16 + 4*r][lane%16].
#include <algorithm>

#include "nonlocal_kernel.hpp"

namespace sparc {

template <typename T, typename TI>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs<T, TI> g)
{
    __shared__ T tile[4][16][16];
    gather_item<T, TI>(g, blockIdx.x, blockIdx.y, blockIdx.z, tile, threadIdx.x);
}

// table in dynamic LDS: [block's atoms][npm][NC]
template <typename T, int NC>
__global__ void __launch_bounds__(256) scatter_kernel(const ScatterArgs<T> s, int npm)
{
    extern __shared__ __align__(16) char scatter_lds[];
    scatter_item<T, NC>(s, blockIdx.x, blockIdx.y, (T *)scatter_lds, npm);
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
    // columns per workgroup: FP32 blocks take 32 when the table fits in 32
    // KiB of LDS (a quarter of the chi and table reads of 8 columns, same
    // time); FP64 blocks keep 8 (16 measured slower)
    constexpr int NW = sizeof(T) == 4 ? 32 : kScatterCols;
    const int npm = std::max(1, op->max_nproj);
    const size_t row = (size_t)std::max(1, op->nl_max_slots) * npm * sizeof(T);
    const bool wide = row * NW <= 32768;
    const int nc = wide ? NW : kScatterCols;
    if ((ns + nc - 1) / nc > 65535) return fail(SPARC_E_SHAPE, "too many columns for one scatter launch");
    dim3 grid(op->nl_nblk, (ns + nc - 1) / nc);
    ProfScope prof(2, stream);
    if (wide && NW != kScatterCols)
        hipLaunchKernelGGL((scatter_kernel<T, NW>), grid, dim3(256), row * NW, stream, a, npm);
    else
        hipLaunchKernelGGL((scatter_kernel<T, kScatterCols>), grid, dim3(256), row * kScatterCols, stream, a, npm);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

int launch_scatter(const sparc_op *op, int dtype, void *out, int64_t ldo, int ns, const void *part, double alpha,
                   hipStream_t stream)
{
    if (op->natoms == 0) return SPARC_OK;
    if (dtype == SPARC_F64) return launch_scatter_t<double>(op, out, ldo, ns, part, alpha, stream, op->d_chi64, op->d_hg64);
    return launch_scatter_t<float>(op, out, ldo, ns, part, alpha, stream, op->d_chi32, op->d_hg32);
}

}  // namespace sparc
