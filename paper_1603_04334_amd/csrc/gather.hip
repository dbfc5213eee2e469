// Projector gather of the nonlocal operator (Sec. 3.1, Eq. non-localPS:FD):
//     G[proj0_J + p][c] = h^3 gamma_Jp * sum_{x in cube_J} chi_Jp(x) Y(x, c)
// the first half of V_nl; the fused step kernel scatters sum_p chi_Jp(x) G[.][c]
// back onto the grid.
//
// The contraction for one atom is a small GEMM, G_J^T (ns x nproj) =
// Y_box^T (ns x nbox) * chi_J (nbox x nproj), and runs on the matrix cores:
// v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (FP32).  A workgroup
// takes one atom and 16 columns; its four waves split the cube's points
// (the K dimension) into interleaved chunks of 4 and each accumulates a
// 16 x 16 tile (16 columns x up to 16 projectors); the four partial tiles
// are then summed in a fixed order through LDS, so the result does not
// depend on timing (no atomics).
//
// Operand layout of the 16x16x4 MFMA (64 lanes, lane = i + 16*k, i in 0..15,
// k in 0..3): lane supplies A[i][k] (column c0+i at the cube point k of the
// current chunk) and B[k][j] (projector j at the same point); the 16x16
// accumulator holds D[i][j] at lane j + 16*(i/4), register i%4.
#include "internal.hpp"

namespace sparc {

template <typename T>
struct GatherArgs {
    const T *Y;
    long long ldy;
    int ns;
    int n2, n3;
    const AtomDev *atoms;
    const T *chi;
    const T *hg;  // h^3 gamma per global projector
    T *G;         // [nproj_total][ns]
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

template <typename T>
__global__ void __launch_bounds__(256) gather_kernel(const GatherArgs<T> g)
{
    const int atom = blockIdx.x;
    const int c0 = blockIdx.y * 16;
    const AtomDev A = g.atoms[atom];
    const int e1 = A.ext[1], e2 = A.ext[2];
    const int nbox = A.ext[0] * e1 * e2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int i = lane & 15;  // A row (column of Y) / B column (projector)
    const int k = lane >> 4;  // position inside the chunk of 4 points
    const int col = c0 + i;
    const bool col_ok = col < g.ns;
    const bool proj_ok = i < A.nproj;
    const T *y = g.Y + (long long)(col_ok ? col : 0) * g.ldy;
    const T *ch = g.chi + A.chi0 + (long long)(proj_ok ? i : 0) * nbox;

    T acc[4] = {T(0), T(0), T(0), T(0)};
    // chunk q covers cube points 4q..4q+3; wave w takes chunks w, w+4, ...
    const int nchunk = (nbox + 3) / 4;
    for (int qc = wave; qc < nchunk; qc += 4) {
        const int pt = qc * 4 + k;
        T av = T(0), bv = T(0);
        if (pt < nbox) {
            const int iz = pt % e2;
            const int rest = pt / e2;
            const int iy = rest % e1;
            const int ix = rest / e1;
            const long long gidx = ((long long)(A.lo[0] + ix) * g.n2 + (A.lo[1] + iy)) * g.n3 + (A.lo[2] + iz);
            if (col_ok) av = y[gidx];
            if (proj_ok) bv = ch[pt];
        }
        mfma_16x16x4(av, bv, acc);
    }

    __shared__ T part[4][16][16];
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave][4 * (lane >> 4) + r][lane & 15] = acc[r];
    __syncthreads();
    // thread (row, proj) sums the four waves in fixed order
    const int t = threadIdx.x;
    const int row = t >> 4, pj = t & 15;
    const int cc = c0 + row;
    if (cc < g.ns && pj < A.nproj) {
        const T s = ((part[0][row][pj] + part[1][row][pj]) + part[2][row][pj]) + part[3][row][pj];
        g.G[(long long)(A.proj0 + pj) * g.ns + cc] = g.hg[A.proj0 + pj] * s;
    }
}

template <typename T>
static int launch_gather_t(const sparc_op *op, const void *Y, int64_t ldy, int ns, void *G, hipStream_t stream,
                           const T *chi, const T *hg)
{
    GatherArgs<T> a;
    a.Y = (const T *)Y;
    a.ldy = ldy;
    a.ns = ns;
    a.n2 = op->n[1];
    a.n3 = op->n[2];
    a.atoms = op->d_atoms;
    a.chi = chi;
    a.hg = hg;
    a.G = (T *)G;
    dim3 grid(op->natoms, (ns + 15) / 16);
    ProfScope prof(1, stream);
    hipLaunchKernelGGL(gather_kernel<T>, grid, dim3(256), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

int launch_gather(const sparc_op *op, int dtype, const void *Y, int64_t ldy, int ns, void *G, hipStream_t stream)
{
    if (op->natoms == 0) return SPARC_OK;
    if (dtype == SPARC_F64) return launch_gather_t<double>(op, Y, ldy, ns, G, stream, op->d_chi64, op->d_hg64);
    return launch_gather_t<float>(op, Y, ldy, ns, G, stream, op->d_chi32, op->d_hg32);
}

}  // namespace sparc
