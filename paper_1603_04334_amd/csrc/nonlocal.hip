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
//    block's atoms and four columns into LDS (split partials summed in order),
//    then each thread updates one node for the four columns, atoms in a fixed
//    order: deterministic even where cubes overlap.
//
// MFMA operand layout of the 16x16x4 instructions (64 lanes, lane = i + 16k,
// i in 0..15, k in 0..3): lane supplies A[i][k] (column c0+i at cube point
// k of the current group of 4) and B[k][j] (projector j at that point).  The
// FP32 accumulator keeps D[4*(lane/16) + r][lane%16] in register r; the FP64
// accumulator keeps D[lane/16 + 4*r][lane%16].
#include "internal.hpp"

namespace sparc {

template <typename T>
struct GatherArgs {
    const T *Y;
    long long ldy;
    int ns;
    int nproj_total;
    const AtomDev *atoms;
    const int *box_off;  // grid index of every cube point, per atom from atom.box0
    const T *chi;
    T *part;             // [kGatherSplit][nproj_total][ns] partial projections
};

__device__ inline void mfma_16x16x4(const double a, const double b, double (&acc)[4])
{
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}

__device__ inline void mfma_16x16x4(const float a, const float b, float (&acc)[4])
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}

// accumulator row held by register r of this lane
template <typename T>
__device__ inline int acc_row(int lane, int r)
{
    if constexpr (sizeof(T) == 8)
        return (lane >> 4) + 4 * r;
    else
        return 4 * (lane >> 4) + r;
}

constexpr int kGatherUnroll = 8;  // groups of 4 points per wave per batch

template <typename T>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs<T> g)
{
    const int atom = blockIdx.x;
    const int c0 = blockIdx.y * 16;
    const int ks = blockIdx.z;
    const AtomDev A = g.atoms[atom];
    const int nbox = A.ext[0] * A.ext[1] * A.ext[2];
    const int chunk = (nbox + kGatherSplit - 1) / kGatherSplit;
    const int k0 = min(nbox, ks * chunk);
    const int k1 = min(nbox, k0 + chunk);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = lane & 15;
    const int k = lane >> 4;
    const int col = c0 + i;
    const bool col_ok = col < g.ns;
    const bool proj_ok = i < A.nproj;
    const T *y = g.Y + (long long)(col_ok ? col : 0) * g.ldy;
    const T *ch = g.chi + A.chi0 + (long long)(proj_ok ? i : 0) * nbox;
    const int *boff = g.box_off + A.box0;

    T acc[4] = {T(0), T(0), T(0), T(0)};
    constexpr int BATCH = 4 * kGatherUnroll;
    for (int base = k0 + wave * BATCH; base < k1; base += 4 * BATCH) {
        int off[kGatherUnroll];
        T av[kGatherUnroll], bv[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const int pt = base + 4 * u + k;
            off[u] = boff[pt < k1 ? pt : k0];
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const int pt = base + 4 * u + k;
            const bool ok = pt < k1;
            const T yv = y[off[u]];
            const T cv = ch[ok ? pt : k0];
            av[u] = (ok && col_ok) ? yv : T(0);
            bv[u] = (ok && proj_ok) ? cv : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) mfma_16x16x4(av[u], bv[u], acc);
    }

    __shared__ T tile[4][16][16];
#pragma unroll
    for (int r = 0; r < 4; ++r) tile[wave][acc_row<T>(lane, r)][lane & 15] = acc[r];
    __syncthreads();
    const int t = threadIdx.x;
    const int row = t >> 4, pj = t & 15;
    const int cc = c0 + row;
    if (cc < g.ns && pj < A.nproj) {
        const T s = ((tile[0][row][pj] + tile[1][row][pj]) + tile[2][row][pj]) + tile[3][row][pj];
        g.part[((long long)ks * g.nproj_total + A.proj0 + pj) * g.ns + cc] = s;
    }
}

constexpr int kScatterCols = 4;

template <typename T>
struct ScatterArgs {
    T *out;
    long long ldo;
    int ns;
    int nproj_total;
    const int *blk_pt;     // nblk + 1 node offsets
    const int *blk_at;     // nblk + 1 offsets into blk_atoms
    const int *blk_atoms;  // atoms touched by each block (slot order)
    const int *pts;        // unique grid nodes covered by a cube
    const int *ent_off;    // npts + 1 offsets into ent
    const int4 *ent;       // (chi index of projector 0, cube size, slot, nproj)
    const AtomDev *atoms;
    const T *chi;
    const T *hg;           // h^3 gamma per global projector
    const T *part;         // [kGatherSplit][nproj_total][ns]
    T alpha;
};

template <typename T>
__global__ void __launch_bounds__(256) scatter_kernel(const ScatterArgs<T> s)
{
    __shared__ T gl[kScatterSlots][kMaxProj][kScatterCols];
    const int b = blockIdx.x;
    const int c0 = blockIdx.y * kScatterCols;
    const int a0 = s.blk_at[b];
    const int na = s.blk_at[b + 1] - a0;
    const long long split = (long long)s.nproj_total * s.ns;
    for (int idx = threadIdx.x; idx < na * kMaxProj * kScatterCols; idx += 256) {
        const int slot = idx / (kMaxProj * kScatterCols);
        const int p = (idx / kScatterCols) % kMaxProj;
        const int cc = idx % kScatterCols;
        const AtomDev A = s.atoms[s.blk_atoms[a0 + slot]];
        T v = T(0);
        if (p < A.nproj && c0 + cc < s.ns) {
            const long long pg = A.proj0 + p;
            T sum = T(0);
#pragma unroll
            for (int q = 0; q < kGatherSplit; ++q) sum += s.part[q * split + pg * s.ns + c0 + cc];
            v = s.hg[pg] * sum;
        }
        gl[slot][p][cc] = v;
    }
    __syncthreads();
    const int pi = s.blk_pt[b] + threadIdx.x;
    if (pi >= s.blk_pt[b + 1]) return;
    T acc[kScatterCols] = {};
    const int e1 = s.ent_off[pi + 1];
    for (int e = s.ent_off[pi]; e < e1; ++e) {
        const int4 en = s.ent[e];
        for (int p = 0; p < en.w; ++p) {
            const T cv = s.chi[en.x + (long long)p * en.y];
#pragma unroll
            for (int cc = 0; cc < kScatterCols; ++cc) acc[cc] += cv * gl[en.z][p][cc];
        }
    }
    const int gpt = s.pts[pi];
#pragma unroll
    for (int cc = 0; cc < kScatterCols; ++cc)
        if (c0 + cc < s.ns) {
            T *o = s.out + (long long)(c0 + cc) * s.ldo + gpt;
            *o += s.alpha * acc[cc];
        }
}

template <typename T>
static int launch_gather_t(const sparc_op *op, const void *Y, int64_t ldy, int ns, void *part, hipStream_t stream,
                           const T *chi)
{
    GatherArgs<T> a;
    a.Y = (const T *)Y;
    a.ldy = ldy;
    a.ns = ns;
    a.nproj_total = op->nproj_total;
    a.atoms = op->d_atoms;
    a.box_off = op->d_box_off;
    a.chi = chi;
    a.part = (T *)part;
    dim3 grid(op->natoms, (ns + 15) / 16, kGatherSplit);
    ProfScope prof(1, stream);
    hipLaunchKernelGGL(gather_kernel<T>, grid, dim3(256), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
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
