// Fused Hamiltonian / Chebyshev-step kernel for gfx950.
//
// One launch computes, for every node x and every column c of an orbital
// block,
//     out(x,c) = alpha * ( (-1/2 lap_h + V_eff(x) - shift) yk(x,c) + sum_J chi_J(x)^T G_J(c) )
//                - beta * yprev(x,c)
// which is one step of the three-term Chebyshev recurrence of Sec. 3.4
// (alpha = 2 sigma_{k+1}/e, beta = sigma_k sigma_{k+1}, shift = c), the first
// step (beta = 0) or a plain application of H (alpha = 1, beta = shift = 0).
// lap_h is the 2n_o-order stencil of Sec. 3.1 Eq. FD:Laplacian with f = 0 off
// the grid; the last term is the scatter half of the nonlocal operator of Eq.
// non-localPS:FD, whose gather half G_J(c) = h^3 gamma_J chi_J^T yk(:,c) is
// produced beforehand by the gather kernel.
//
// Data movement (HBM-bound design):
//  * A workgroup owns a TY x TZ patch of the (y, z) plane of one column and
//    streams it along x (the slowest axis), so each plane of yk is fetched from
//    HBM once.  Each thread keeps a queue of 2R+1 values of its own (y, z)
//    points along x in registers, so the x-neighbours never touch LDS.
//  * The current x-plane of the patch plus a cross-shaped halo of R rows in y
//    and R columns in z is staged in LDS (double-buffered, one barrier per
//    plane); y- and z-neighbours are read from there.  Halo values belong to
//    neighbouring patches and are served by L2 when neighbours run on the same
//    XCD, which the workgroup-index remap below arranges.
//  * The next plane's queue head and halo are requested before the current
//    plane is computed, so their latency overlaps the arithmetic.
//  * yprev is read pointwise and out may alias it: each thread reads
//    yprev(x) before writing out(x), and no other thread touches that node.
//  * Lanes run along z (the contiguous axis): every global access of a wave is
//    a contiguous run along z.
#include "internal.hpp"

namespace sparc {

const TileShape kShapes[kNumShapes] = {{32, 2}, {64, 4}, {32, 4}, {64, 2}};

template <typename T>
struct StepArgs {
    const T *yk;
    const T *yprev;
    T *out;
    const T *veff;
    const T *chi;
    const T *G;
    const AtomDev *atoms;
    const int *tile_off;
    const int *tile_list;
    long long ldk, ldp, ldo;
    int n1, n2, n3;
    int tiles_y, tiles_z, nchunks, chunk_x;
    int ns;
    int nblocks;
    int has_prev;
    T c0;                 // centre coefficient of -1/2 lap_h: -3 w_0
    T cp[kMaxRadius];     // -1/2 w_p, p = 1..kMaxRadius (zero beyond the op's radius)
    T alpha, beta, shift;
};

template <typename T, int TZ, int RY>
__global__ void __launch_bounds__(kBlock) step_kernel(const StepArgs<T> a)
{
    constexpr int R = kMaxRadius;
    constexpr int NYG = kBlock / TZ;
    constexpr int TY = NYG * RY;
    constexpr int SZ = TZ + 2 * R;
    constexpr int SY = TY + 2 * R;
    constexpr int NHALO = 2 * R * TZ + 2 * R * TY;
    constexpr int NH = (NHALO + kBlock - 1) / kBlock;
    __shared__ T lds[2][SY * SZ];

    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
    // contiguous range of patches so that neighbours share its L2.
    const int nb = a.nblocks;
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int logical = xcd * (nb >> 3) + min(xcd, nb & 7) + (b >> 3);

    int t = logical;
    const int tzi = t % a.tiles_z;
    t /= a.tiles_z;
    const int tyi = t % a.tiles_y;
    t /= a.tiles_y;
    const int chunk = t % a.nchunks;
    const int col = t / a.nchunks;

    const int tid = threadIdx.x;
    const int lz = tid % TZ;
    const int lyg = tid / TZ;
    const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
    const int z0 = tzi * TZ, y0 = tyi * TY;
    const int z = z0 + lz;
    const long long P = (long long)n2 * n3;

    const T *__restrict__ yk = a.yk + (long long)col * a.ldk;
    const T *yp = a.has_prev ? a.yprev + (long long)col * a.ldp : nullptr;
    T *out = a.out + (long long)col * a.ldo;

    int yrow[RY], pofs[RY];
    bool pok[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        yrow[r] = y0 + lyg + r * NYG;
        pok[r] = (z < n3) && (yrow[r] < n2);
        pofs[r] = yrow[r] * n3 + z;
    }

    // halo slots owned by this thread: LDS index and in-plane global offset
    int hl[NH], hg[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) {
        const int e = tid + i * kBlock;
        int ly = -1, lzz = -1;
        if (e < 2 * R * TZ) {
            const int hy = e / TZ, hz = e % TZ;
            ly = hy < R ? hy : hy + TY;
            lzz = R + hz;
        } else if (e < NHALO) {
            const int e2 = e - 2 * R * TZ;
            const int zr = e2 / (2 * R), hz = e2 % (2 * R);
            ly = R + zr;
            lzz = hz < R ? hz : hz + TZ;
        }
        hl[i] = (ly >= 0) ? ly * SZ + lzz : -1;
        const int gy = y0 - R + ly, gz = z0 - R + lzz;
        hg[i] = (ly >= 0 && gy >= 0 && gy < n2 && gz >= 0 && gz < n3) ? gy * n3 + gz : -1;
    }

    const int xs = chunk * a.chunk_x;
    const int xe = min(n1, xs + a.chunk_x);

    T q[RY][2 * R + 1];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int d = 0; d <= 2 * R; ++d) {
            const int xx = xs - R + d;
            q[r][d] = (pok[r] && xx >= 0 && xx < n1) ? yk[xx * P + pofs[r]] : T(0);
        }
    T hv[NH];
#pragma unroll
    for (int i = 0; i < NH; ++i) hv[i] = (hg[i] >= 0) ? yk[xs * P + hg[i]] : T(0);

    const int tile = tyi * a.tiles_z + tzi;
    const int at_beg = a.tile_off[tile];
    const int at_end = a.tile_off[tile + 1];

    for (int x = xs; x < xe; ++x) {
        T *L = lds[(x - xs) & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) L[(R + lyg + r * NYG) * SZ + R + lz] = q[r][R];
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (hl[i] >= 0) L[hl[i]] = hv[i];
        __syncthreads();

        // request the next plane's halo and queue heads
        const int xn = x + 1;
        T qn[RY];
#pragma unroll
        for (int i = 0; i < NH; ++i) hv[i] = (xn < xe && hg[i] >= 0) ? yk[xn * P + hg[i]] : T(0);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int xx = x + R + 1;
            qn[r] = (pok[r] && xx < n1) ? yk[xx * P + pofs[r]] : T(0);
        }

#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int li = (R + lyg + r * NYG) * SZ + R + lz;
            T s = a.c0 * q[r][R];
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                const T six = (q[r][R - p] + q[r][R + p]) + (L[li - p * SZ] + L[li + p * SZ]) + (L[li - p] + L[li + p]);
                s += a.cp[p - 1] * six;
            }
            if (pok[r]) {
                const long long g = x * P + pofs[r];
                s += (a.veff[g] - a.shift) * q[r][R];
                for (int j = at_beg; j < at_end; ++j) {
                    const AtomDev &A = a.atoms[a.tile_list[j]];
                    const int ix = x - A.lo[0], iy = yrow[r] - A.lo[1], iz = z - A.lo[2];
                    if ((unsigned)ix < (unsigned)A.ext[0] && (unsigned)iy < (unsigned)A.ext[1] &&
                        (unsigned)iz < (unsigned)A.ext[2]) {
                        const long long nbox = (long long)A.ext[0] * A.ext[1] * A.ext[2];
                        const T *ch = a.chi + A.chi0 + ((long long)ix * A.ext[1] + iy) * A.ext[2] + iz;
                        const T *gg = a.G + (long long)A.proj0 * a.ns + col;
                        for (int pp = 0; pp < A.nproj; ++pp) s += ch[pp * nbox] * gg[(long long)pp * a.ns];
                    }
                }
                T res = a.alpha * s;
                if (yp) res -= a.beta * yp[g];
                out[g] = res;
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int d = 0; d < 2 * R; ++d) q[r][d] = q[r][d + 1];
            q[r][2 * R] = qn[r];
        }
    }
}

StepLaunch choose_step_launch(const sparc_op *op, int dtype, int ns)
{
    (void)dtype;
    StepLaunch L;
    const int n3 = op->n[2];
    // prefer a z extent that tiles n3 with little waste
    const int waste32 = (32 - n3 % 32) % 32;
    const int waste64 = (64 - n3 % 64) % 64;
    L.shape = (n3 >= 64 && waste64 <= waste32) ? 1 : 0;
    const TileShape &s = kShapes[L.shape];
    const long long tiles = (long long)((op->n[1] + s.ty() - 1) / s.ty()) * ((n3 + s.tz - 1) / s.tz);
    const long long per_chunk = tiles * ns;
    // split x when too few workgroups would fill the 256 CUs
    int nchunks = 1;
    while (per_chunk * nchunks < 2048 && op->n[0] / (nchunks * 2) >= 8) nchunks *= 2;
    L.chunk_x = (op->n[0] + nchunks - 1) / nchunks;
    return L;
}

template <typename T, int TZ, int RY>
static int launch_typed(const StepArgs<T> &a, hipStream_t stream)
{
    hipLaunchKernelGGL((step_kernel<T, TZ, RY>), dim3(a.nblocks), dim3(kBlock), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

template <typename T>
static int launch_step_t(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                         void *out, int64_t ldo, int ns, const void *G, const StepCoef &c, const StepLaunch &L,
                         hipStream_t stream, const T *veff, const T *chi)
{
    const TileShape &s = kShapes[L.shape];
    const TileLists &tl = op->lists[L.shape];
    StepArgs<T> a;
    a.yk = (const T *)yk;
    a.yprev = (const T *)yprev;
    a.out = (T *)out;
    a.veff = veff;
    a.chi = chi;
    a.G = (const T *)G;
    a.atoms = op->d_atoms;
    a.tile_off = tl.d_off;
    a.tile_list = tl.d_list;
    a.ldk = ldk;
    a.ldp = ldp;
    a.ldo = ldo;
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.n3 = op->n[2];
    a.tiles_y = tl.tiles_y;
    a.tiles_z = tl.tiles_z;
    a.chunk_x = L.chunk_x;
    a.nchunks = (op->n[0] + L.chunk_x - 1) / L.chunk_x;
    a.ns = ns;
    a.has_prev = c.has_prev && yprev != nullptr;
    const long long nb = (long long)ns * a.nchunks * a.tiles_y * a.tiles_z;
    if (nb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
    a.nblocks = (int)nb;
    a.c0 = (T)(-3.0 * op->w[0]);
    for (int p = 1; p <= kMaxRadius; ++p) a.cp[p - 1] = (T)(-0.5 * op->w[p]);
    a.alpha = (T)c.alpha;
    a.beta = (T)c.beta;
    a.shift = (T)c.shift;
    ProfScope prof(0, stream);
    switch (L.shape) {
        case 0: return launch_typed<T, 32, 2>(a, stream);
        case 1: return launch_typed<T, 64, 4>(a, stream);
        case 2: return launch_typed<T, 32, 4>(a, stream);
        case 3: return launch_typed<T, 64, 2>(a, stream);
    }
    (void)s;
    return fail(SPARC_E_ARG, "unknown tile shape");
}

int launch_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                void *out, int64_t ldo, int ns, const void *G, const StepCoef &c, const StepLaunch &L,
                hipStream_t stream)
{
    if (dtype == SPARC_F64)
        return launch_step_t<double>(op, yk, ldk, yprev, ldp, out, ldo, ns, G, c, L, stream, op->d_veff64,
                                     op->d_chi64);
    return launch_step_t<float>(op, yk, ldk, yprev, ldp, out, ldo, ns, G, c, L, stream, op->d_veff32,
                                op->d_chi32);
}

}  // namespace sparc
