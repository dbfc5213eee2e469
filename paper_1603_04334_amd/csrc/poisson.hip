// Electrostatic potential (Sec. 3.3): -(1/4 pi) lap_h phi = c - d on the grid
// with zero Dirichlet padding (Eq. FD:PoissonDiscrete), c = rho + b the total
// charge and d the charge correction of Eq. Phi:correction, which carries the
// values of phi just outside the grid from the multipole expansion of c to
// l_max (Eq. phi:BC:discrete and the discrete moments Q_lm that follow it).
// Solved by conjugate gradients with a block-Jacobi preconditioner (Sec. 4).
//
// Layout and kernels (everything FP64, on the device):
//  * moments: one pass over the grid, each thread accumulating all
//    (l_max+1)^2 products r^l Y_lm c (regular solid harmonics from their
//    Cartesian recurrences, expansion centre = domain centre); one partial
//    per workgroup, summed in a fixed order;
//  * boundary values of phi on the six off-grid slabs n_o nodes deep (only
//    nodes one axis step off a face are ever read by the stencil);
//  * right-hand side c - d, with d from the slabs, and the partial sums of
//    its square;
//  * CG iteration: q = A p through the fused stencil kernel of H on a
//    zero-potential operator (A = (1/2 pi) (-1/2 lap_h)), then p.q, then one
//    kernel that updates x and r, multiplies each block of r by the inverse of
//    A restricted to the block (a dense symmetric matrix, one per block shape,
//    kept in L2; blocks are taken in bricks along z so that global accesses
//    are coalesced rows) and forms the partials of r.z and r.r, then the
//    update of p.  Scalars never leave the device: every
//    workgroup finishes the partial sums it needs in the same fixed order, so
//    alpha, beta and the convergence test are bitwise the same everywhere.
//    The host enqueues iterations in chunks and reads one flag per chunk;
//    kernels after convergence return at once.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace sparc {
namespace {

constexpr int kLmax = 6;                           // largest expansion order supported
constexpr int kNM = (kLmax + 1) * (kLmax + 1);     // moments
constexpr int kPT = 256;                           // threads per workgroup
constexpr int kBjStage = 64;                       // largest block (nodes) whose inverse is staged in LDS
constexpr int kRedMax = 1024;                      // workgroups of the reduction kernels
constexpr int kChunk = 8;                          // CG iterations enqueued between convergence reads
constexpr double kFourPi = 12.566370614359172954;  // 4 pi

struct HarmNorm {
    double c[kNM];
};

struct PcgState {
    int done;
    int iters;
    double rr, bb;
};

// regular solid harmonics R_lm(x) = |x|^l Y_lm(x/|x|), index l*l + l + m:
// (x + i y)^m = C_m + i S_m, the polynomial P_l^m(z, r^2) of the associated
// Legendre recurrence in l, and R_lm = N_lm P_l^m C_m (m >= 0),
// R_l,-m = N_lm P_l^m S_m
__device__ __forceinline__ void solid_harmonics(double x, double y, double z, const HarmNorm &nrm, double (&R)[kNM])
{
    const double r2 = x * x + y * y + z * z;
    double C[kLmax + 1], S[kLmax + 1];
    C[0] = 1.0;
    S[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= kLmax; ++m) {
        C[m] = x * C[m - 1] - y * S[m - 1];
        S[m] = x * S[m - 1] + y * C[m - 1];
    }
    double dfact = 1.0;  // (2m - 1)!!
#pragma unroll
    for (int m = 0; m <= kLmax; ++m) {
        if (m > 0) dfact *= (2 * m - 1);
        double p2 = dfact, p1 = 0.0;
#pragma unroll
        for (int l = m; l <= kLmax; ++l) {
            double P;
            if (l == m) {
                P = p2;
            } else if (l == m + 1) {
                P = (2 * m + 1) * z * p2;
                p1 = P;
            } else {
                P = ((2 * l - 1) * z * p1 - (l + m - 1) * r2 * p2) / (l - m);
                p2 = p1;
                p1 = P;
            }
            R[l * l + l + m] = nrm.c[l * l + l + m] * P * C[m];
            if (m > 0) R[l * l + l - m] = nrm.c[l * l + l - m] * P * S[m];
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// sum over the 256 threads, the same value in every thread (fixed order)
__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// sum of n partials in a fixed order, the same value in every thread
__device__ __forceinline__ double sum_partials(const double *part, int n, double *red)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += kPT) v += part[i];
    return block_sum(v, red);
}

struct GridGeo {
    int n0, n1, n2;
    long long nd;
    double h;
    double c0, c1, c2;  // domain centre
};

__device__ __forceinline__ void node_pos(const GridGeo &g, long long t, int &i, int &j, int &k, double &x, double &y,
                                         double &z)
{
    k = (int)(t % g.n2);
    const long long u = t / g.n2;
    j = (int)(u % g.n1);
    i = (int)(u / g.n1);
    x = (i + 1) * g.h - g.c0;
    y = (j + 1) * g.h - g.c1;
    z = (k + 1) * g.h - g.c2;
}

__global__ void __launch_bounds__(kPT) moments_kernel(const double *__restrict__ charge, const GridGeo g,
                                                      const HarmNorm nrm, double *__restrict__ partial)
{
    double acc[kNM];
#pragma unroll
    for (int q = 0; q < kNM; ++q) acc[q] = 0.0;
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < g.nd; t += (long long)gridDim.x * kPT) {
        const double f = charge[t];
        int i, j, k;
        double x, y, z;
        node_pos(g, t, i, j, k, x, y, z);
        double R[kNM];
        solid_harmonics(x, y, z, nrm, R);
#pragma unroll
        for (int q = 0; q < kNM; ++q) acc[q] += R[q] * f;
    }
    __shared__ double red[4][kNM];
#pragma unroll
    for (int q = 0; q < kNM; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNM)
        partial[(long long)blockIdx.x * kNM + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// Q_lm = h^3 sum of the workgroup partials (fixed order); zero beyond lmax
__global__ void __launch_bounds__(kPT) moments_finish(const double *__restrict__ partial, int nparts, double h3,
                                                      int lmax, double *__restrict__ Q)
{
    const int q = threadIdx.x;
    if (q >= kNM) return;
    double v = 0.0;
    for (int b = 0; b < nparts; ++b) v += partial[(long long)b * kNM + q];
    const int l = (int)sqrtf((float)q + 0.5f);
    Q[q] = l <= lmax ? h3 * v : 0.0;
}

struct SlabGeo {
    int no;
    long long off[6];  // start of face f = 2 ax + side in the slab array
    int nu[3], nv[3];  // extent of the face coordinates (u, v) for axis ax
};

// phi of Eq. phi:BC:discrete at the off-grid nodes: face f = 2 ax + side,
// layer L = 1..no (index ax = -L on the low side, n_ax - 1 + L on the high
// side), the other two indices over the grid in order
__global__ void __launch_bounds__(kPT) slab_kernel(const GridGeo g, const SlabGeo sg, const HarmNorm nrm, int lmax,
                                                   const double *__restrict__ Q, double *__restrict__ slab,
                                                   long long total)
{
    const long long t = blockIdx.x * (long long)kPT + threadIdx.x;
    if (t >= total) return;
    int f = 0;
    while (f < 5 && t >= sg.off[f + 1]) ++f;
    const int ax = f >> 1, side = f & 1;
    const long long loc = t - sg.off[f];
    const long long per = (long long)sg.nu[ax] * sg.nv[ax];
    const int L = (int)(loc / per) + 1;
    const long long uv = loc % per;
    const int u = (int)(uv / sg.nv[ax]), v = (int)(uv % sg.nv[ax]);
    const int nax = ax == 0 ? g.n0 : (ax == 1 ? g.n1 : g.n2);
    const int ia = side ? nax - 1 + L : -L;
    int idx[3];
    idx[ax] = ia;
    idx[ax == 0 ? 1 : 0] = u;
    idx[ax == 2 ? 1 : 2] = v;
    const double x = (idx[0] + 1) * g.h - g.c0, y = (idx[1] + 1) * g.h - g.c1, z = (idx[2] + 1) * g.h - g.c2;
    double R[kNM];
    solid_harmonics(x, y, z, nrm, R);
    const double r2 = x * x + y * y + z * z;
    const double rinv2 = 1.0 / r2;
    double rl = 1.0 / sqrt(r2);  // 1 / r^(2l+1), starting at l = 0
    double phi = 0.0;
    // Q is zero beyond lmax, so the fixed-length loops add exact zeros there
#pragma unroll
    for (int l = 0; l <= kLmax; ++l) {
        double s = 0.0;
#pragma unroll
        for (int m = -l; m <= l; ++m) s += Q[l * l + l + m] * R[l * l + l + m];
        phi += kFourPi / (2 * l + 1) * rl * s;
        rl *= rinv2;
    }
    (void)lmax;
    slab[t] = phi;
}

// rhs = c - d, d = -(1/4 pi) sum of w_p phi at the off-grid neighbours
// (Eq. Phi:correction); partial sums of rhs^2 per workgroup
__global__ void __launch_bounds__(kPT) rhs_kernel(const double *__restrict__ charge, const GridGeo g,
                                                  const SlabGeo sg, const double *__restrict__ w,
                                                  const double *__restrict__ slab, double *__restrict__ rhs,
                                                  double *__restrict__ part_bb)
{
    __shared__ double red[4];
    double bb = 0.0;
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < g.nd; t += (long long)gridDim.x * kPT) {
        int id[3];
        double x, y, z;
        node_pos(g, t, id[0], id[1], id[2], x, y, z);
        const int nn[3] = {g.n0, g.n1, g.n2};
        double d = 0.0;
        for (int ax = 0; ax < 3; ++ax) {
            const int ia = id[ax];
            if (ia >= sg.no && ia < nn[ax] - sg.no) continue;
            const int u = id[ax == 0 ? 1 : 0], v = id[ax == 2 ? 1 : 2];
            const long long per = (long long)sg.nu[ax] * sg.nv[ax];
            const long long uv = (long long)u * sg.nv[ax] + v;
            for (int p = 1; p <= sg.no; ++p) {
                if (ia - p < 0) d += w[p] * slab[sg.off[2 * ax] + (long long)(p - ia - 1) * per + uv];
                if (ia + p > nn[ax] - 1) d += w[p] * slab[sg.off[2 * ax + 1] + (long long)(ia + p - nn[ax]) * per + uv];
            }
        }
        const double rv = charge[t] + d / kFourPi;
        rhs[t] = rv;
        bb += rv * rv;
    }
    const double s = block_sum(bb, red);
    if (threadIdx.x == 0) part_bb[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kPT) axpy_kernel(double *__restrict__ r, const double *__restrict__ q, double a,
                                                   long long n)
{
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < n; t += (long long)gridDim.x * kPT) r[t] += a * q[t];
}

__global__ void __launch_bounds__(kPT) fill_kernel(double *__restrict__ x, long long n)
{
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < n; t += (long long)gridDim.x * kPT) x[t] = 0.0;
}

struct BjGeo {
    int n0, n1, n2;
    int b[3];     // block edge per axis
    int nb[3];    // blocks per axis
    int last[3];  // edge of the last block per axis
    int maxm;     // b0 b1 b2
    long long nblocks;
};

// the shape code of block (bi, bj, bk): bit 2/1/0 set when it is the last
// block of a ragged axis
__device__ __forceinline__ int bj_shape(const BjGeo &q, int bi, int bj, int bk, int (&dim)[3])
{
    const int bidx[3] = {bi, bj, bk};
    int code = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool lastb = bidx[a] == q.nb[a] - 1;
        dim[a] = lastb ? q.last[a] : q.b[a];
        code = 2 * code + (lastb ? 1 : 0);
    }
    return code;
}

// block-Jacobi step over all blocks.  A workgroup takes a brick of G = 256 /
// (b0 b1 b2) blocks that follow each other along z in one (block x, block y)
// row, so its global accesses are rows of G b2 consecutive nodes (coalesced):
// thread t owns node (a, b, zz) of the brick, t = (a b1 + b) G b2 + zz.  The
// residual goes through LDS into block order, thread (slot, row) forms row
// `row` of M^-1 r for block `slot` (sum over j ascending; the interior
// blocks' inverse read from LDS), and the result goes back through LDS to the
// brick order for the coalesced store.
// UPDATE: alpha = rz_old / pq, x += alpha p, r -= alpha q; both modes:
// z = M^-1 r per block, p = z (INIT only), partials of r.z and r.r
template <bool UPDATE>
__global__ void __launch_bounds__(kPT)
    bj_kernel(const BjGeo q, const double *__restrict__ minv, double *__restrict__ x, double *__restrict__ r,
              double *__restrict__ p, const double *__restrict__ qv, double *__restrict__ z,
              const double *__restrict__ part_rz_old, int n_rz_old, const double *__restrict__ part_pq, int n_pq,
              double *__restrict__ part_rz, double *__restrict__ part_rr, const PcgState *__restrict__ state)
{
    __shared__ double red[4];
    __shared__ double rs[kPT];
    __shared__ double zs[kPT];
    // the inverse of the interior block shape (code 0), read by every row of
    // every interior block, staged once per workgroup (blocks of at most
    // kBjStage nodes)
    __shared__ double sM[kBjStage * kBjStage];
    if (UPDATE && state->done) return;
    const bool staged = q.maxm <= kBjStage;
    if (staged)
        for (int e = threadIdx.x; e < q.maxm * q.maxm; e += kPT) sM[e] = minv[e];
    double alpha = 0.0;
    if (UPDATE) alpha = sum_partials(part_rz_old, n_rz_old, red) / sum_partials(part_pq, n_pq, red);
    const int G = kPT / q.maxm;          // blocks per brick
    const int bpr = (q.nb[2] + G - 1) / G;  // bricks per (block x, block y) row
    const long long nbricks = (long long)q.nb[0] * q.nb[1] * bpr;
    // brick-order coordinates of this thread
    const int zw = G * q.b[2];
    const int ta = threadIdx.x / (q.b[1] * zw), tb = (threadIdx.x / zw) % q.b[1], tz = threadIdx.x % zw;
    const bool tin = threadIdx.x < q.b[0] * q.b[1] * zw;
    const int tslot = tz / q.b[2], tzl = tz % q.b[2];
    // block-order coordinates of this thread (compute phase)
    const int cslot = threadIdx.x / q.maxm, crow = threadIdx.x % q.maxm;
    double arz = 0.0, arr = 0.0;
    for (long long br = blockIdx.x; br < nbricks; br += gridDim.x) {
        const int bk0 = (int)(br % bpr) * G;
        const long long u = br / bpr;
        const int bj = (int)(u % q.nb[1]), bi = (int)(u / q.nb[1]);
        // load phase: this thread's node of the brick
        int dim[3] = {1, 1, 1};
        bool act = tin && bk0 + tslot < q.nb[2];
        long long node = 0;
        int lrow = 0;
        if (act) {
            (void)bj_shape(q, bi, bj, bk0 + tslot, dim);
            act = ta < dim[0] && tb < dim[1] && tzl < dim[2];
            lrow = (ta * dim[1] + tb) * dim[2] + tzl;
            node = ((long long)(bi * q.b[0] + ta) * q.n1 + (bj * q.b[1] + tb)) * q.n2 + ((bk0 + tslot) * q.b[2] + tzl);
        }
        double rv = 0.0;
        if (act) {
            if (UPDATE) {
                x[node] += alpha * p[node];
                rv = r[node] - alpha * qv[node];
                r[node] = rv;
            } else {
                rv = r[node];
            }
            rs[tslot * q.maxm + lrow] = rv;
        }
        __syncthreads();
        // compute phase: row crow of block cslot
        if (cslot < G && bk0 + cslot < q.nb[2]) {
            int cd[3];
            const int code = bj_shape(q, bi, bj, bk0 + cslot, cd);
            const int m = cd[0] * cd[1] * cd[2];
            if (crow < m) {
                const double *rb = rs + cslot * q.maxm;
                double zv = 0.0;
                if (staged && code == 0) {
#pragma unroll 8
                    for (int j = 0; j < m; ++j) zv += sM[j * m + crow] * rb[j];
                } else {
                    const double *M = minv + (long long)code * q.maxm * q.maxm;
#pragma unroll 8
                    for (int j = 0; j < m; ++j) zv += M[(long long)j * m + crow] * rb[j];
                }
                zs[cslot * q.maxm + crow] = zv;
            }
        }
        __syncthreads();
        // store phase, brick order again
        if (act) {
            const double zv = zs[tslot * q.maxm + lrow];
            z[node] = zv;
            if (!UPDATE) p[node] = zv;
            arz += rv * zv;
            arr += rv * rv;
        }
        __syncthreads();
    }
    const double s1 = block_sum(arz, red);
    const double s2 = block_sum(arr, red);
    if (threadIdx.x == 0) {
        part_rz[blockIdx.x] = s1;
        part_rr[blockIdx.x] = s2;
    }
}

// partials of p.q
__global__ void __launch_bounds__(kPT) dot_kernel(const double *__restrict__ a, const double *__restrict__ b,
                                                  long long n, double *__restrict__ part,
                                                  const PcgState *__restrict__ state)
{
    __shared__ double red[4];
    if (state->done) return;
    double s = 0.0;
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < n; t += (long long)gridDim.x * kPT) s += a[t] * b[t];
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// convergence test and p = z + beta p, beta = rz_new / rz_old
__global__ void __launch_bounds__(kPT)
    pupdate_kernel(double *__restrict__ p, const double *__restrict__ z, long long n, const double *__restrict__ rz_new,
                   const double *__restrict__ rz_old, const double *__restrict__ rr, int nbj,
                   const double *__restrict__ part_bb, int nbb, double tol2, int iter, PcgState *__restrict__ state)
{
    __shared__ double red[4];
    if (state->done) return;
    const double rrv = sum_partials(rr, nbj, red);
    const double bb = sum_partials(part_bb, nbb, red);
    if (rrv <= tol2 * bb) {
        __syncthreads();
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            state->done = 1;
            state->iters = iter + 1;
            state->rr = rrv;
            state->bb = bb;
        }
        return;
    }
    const double beta = sum_partials(rz_new, nbj, red) / sum_partials(rz_old, nbj, red);
    for (long long t = blockIdx.x * (long long)kPT + threadIdx.x; t < n; t += (long long)gridDim.x * kPT)
        p[t] = z[t] + beta * p[t];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        state->iters = iter + 1;
        state->rr = rrv;
        state->bb = bb;
    }
}

// state after the initial residual: converged already when r.r <= tol^2 b.b
__global__ void __launch_bounds__(kPT) pcg_start_kernel(const double *__restrict__ rr, int nbj,
                                                        const double *__restrict__ part_bb, int nbb, double tol2,
                                                        PcgState *__restrict__ state)
{
    __shared__ double red[4];
    const double rrv = sum_partials(rr, nbj, red);
    const double bb = sum_partials(part_bb, nbb, red);
    if (threadIdx.x == 0) {
        state->done = rrv <= tol2 * bb ? 1 : 0;
        state->iters = 0;
        state->rr = rrv;
        state->bb = bb;
    }
}

// Gauss-Jordan inverse of an SPD matrix (host, FP64, partial pivoting)
bool invert(std::vector<double> &A, int m)
{
    std::vector<double> I((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) I[(size_t)i * m + i] = 1.0;
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(A[(size_t)r * m + c]) > std::fabs(A[(size_t)piv * m + c])) piv = r;
        if (A[(size_t)piv * m + c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < m; ++k) {
                std::swap(A[(size_t)c * m + k], A[(size_t)piv * m + k]);
                std::swap(I[(size_t)c * m + k], I[(size_t)piv * m + k]);
            }
        const double d = A[(size_t)c * m + c];
        for (int k = 0; k < m; ++k) {
            A[(size_t)c * m + k] /= d;
            I[(size_t)c * m + k] /= d;
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            const double f = A[(size_t)r * m + c];
            if (f == 0.0) continue;
            for (int k = 0; k < m; ++k) {
                A[(size_t)r * m + k] -= f * A[(size_t)c * m + k];
                I[(size_t)r * m + k] -= f * I[(size_t)c * m + k];
            }
        }
    }
    A.swap(I);
    return true;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace
}  // namespace sparc

using namespace sparc;

struct sparc_poisson {
    int device = 0;
    GridGeo g{};
    SlabGeo sg{};
    BjGeo bj{};
    int lmax = 6;
    int radius = 6;
    sparc_op *op0 = nullptr;  // zero potential, no atoms: its step kernel applies -1/2 lap_h
    HarmNorm nrm{};
    double *d_minv = nullptr;
    double *d_w = nullptr;
    long long slab_total = 0;
    int nmom = 0, nred = 0, nbjg = 0;  // workgroups of the moment, reduction and block-Jacobi kernels
};

namespace {

struct PoisWs {
    double *r, *z, *p, *q, *slab, *mpart, *Q, *bb, *pq, *rz[2], *rr;
    PcgState *state;
    size_t total;
};

PoisWs carve(const sparc_poisson *P, void *ws)
{
    PoisWs W{};
    char *b = (char *)ws;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = b ? b + o : nullptr;
        o += al(bytes);
        return p;
    };
    const size_t vec = (size_t)P->g.nd * sizeof(double);
    W.r = (double *)take(vec);
    W.z = (double *)take(vec);
    W.p = (double *)take(vec);
    W.q = (double *)take(vec);
    W.slab = (double *)take((size_t)P->slab_total * sizeof(double));
    W.mpart = (double *)take((size_t)P->nmom * kNM * sizeof(double));
    W.Q = (double *)take(kNM * sizeof(double));
    W.bb = (double *)take(kRedMax * sizeof(double));
    W.pq = (double *)take(kRedMax * sizeof(double));
    W.rz[0] = (double *)take(kRedMax * sizeof(double));
    W.rz[1] = (double *)take(kRedMax * sizeof(double));
    W.rr = (double *)take(kRedMax * sizeof(double));
    W.state = (PcgState *)take(sizeof(PcgState));
    W.total = o;
    return W;
}

}  // namespace

extern "C" int sparc_poisson_create(const sparc_grid *grid, int32_t lmax, const int32_t *block, sparc_poisson **out)
{
    if (!grid || !out) return fail(SPARC_E_ARG, "null argument");
    *out = nullptr;
    if (lmax < 0 || lmax > kLmax) return fail(SPARC_E_ARG, "lmax must be in 0..6");
    int b[3] = {4, 4, 4};
    if (block)
        for (int a = 0; a < 3; ++a) b[a] = block[a];
    for (int a = 0; a < 3; ++a)
        if (b[a] < 1 || b[a] > 8) return fail(SPARC_E_ARG, "block edges must be in 1..8");
    if (b[0] * b[1] * b[2] > kPT) return fail(SPARC_E_ARG, "a block may hold at most 256 nodes");
    const int64_t nd = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    std::vector<double> zero(nd > 0 ? nd : 1, 0.0);
    sparc_op *op0 = nullptr;
    int st = sparc_op_create(grid, zero.data(), 0, nullptr, &op0);  // validates the grid
    if (st) return st;
    sparc_poisson *P = new (std::nothrow) sparc_poisson();
    if (!P) {
        sparc_op_destroy(op0);
        return fail(SPARC_E_NOMEM, "host allocation failed");
    }
    P->op0 = op0;
    (void)hipGetDevice(&P->device);
    P->lmax = lmax;
    P->radius = grid->radius;
    const int n[3] = {grid->n[0], grid->n[1], grid->n[2]};
    P->g = {n[0], n[1], n[2], (long long)nd, grid->h, 0.5 * (n[0] + 1) * grid->h, 0.5 * (n[1] + 1) * grid->h,
            0.5 * (n[2] + 1) * grid->h};
    // solid-harmonic normalisation: sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), times sqrt 2 for m != 0
    for (int l = 0; l <= kLmax; ++l)
        for (int m = 0; m <= l; ++m) {
            double ratio = 1.0;
            for (int k = l - m + 1; k <= l + m; ++k) ratio /= k;
            double c = std::sqrt((2 * l + 1) / kFourPi * ratio);
            if (m > 0) c *= std::sqrt(2.0);
            P->nrm.c[l * l + l + m] = c;
            P->nrm.c[l * l + l - m] = c;
        }
    // off-grid slabs
    SlabGeo &sg = P->sg;
    sg.no = grid->radius;
    long long off = 0;
    for (int ax = 0; ax < 3; ++ax) {
        sg.nu[ax] = n[ax == 0 ? 1 : 0];
        sg.nv[ax] = n[ax == 2 ? 1 : 2];
        for (int side = 0; side < 2; ++side) {
            sg.off[2 * ax + side] = off;
            off += (long long)sg.no * sg.nu[ax] * sg.nv[ax];
        }
    }
    P->slab_total = off;
    // block Jacobi: dense inverse of A restricted to each block shape
    BjGeo &q = P->bj;
    q.n0 = n[0];
    q.n1 = n[1];
    q.n2 = n[2];
    q.nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        q.b[a] = std::min(b[a], n[a]);
        q.nb[a] = (n[a] + q.b[a] - 1) / q.b[a];
        q.last[a] = n[a] - (q.nb[a] - 1) * q.b[a];
        q.nblocks *= q.nb[a];
    }
    q.maxm = q.b[0] * q.b[1] * q.b[2];
    const double *w = op0->w;
    std::vector<double> minv((size_t)8 * q.maxm * q.maxm, 0.0);
    for (int code = 0; code < 8; ++code) {
        int dim[3];
        for (int a = 0; a < 3; ++a) dim[a] = (code >> (2 - a)) & 1 ? q.last[a] : q.b[a];
        const int m = dim[0] * dim[1] * dim[2];
        std::vector<double> A((size_t)m * m, 0.0);
        for (int t = 0; t < m; ++t) {
            const int c[3] = {t / (dim[1] * dim[2]), (t / dim[2]) % dim[1], t % dim[2]};
            A[(size_t)t * m + t] += 6.0 * w[0];
            for (int a = 0; a < 3; ++a)
                for (int p = 1; p <= grid->radius; ++p)
                    for (int s = -1; s <= 1; s += 2) {
                        int e[3] = {c[0], c[1], c[2]};
                        e[a] += s * p;
                        if (e[a] < 0 || e[a] >= dim[a]) continue;
                        A[(size_t)t * m + (e[0] * dim[1] + e[1]) * dim[2] + e[2]] += w[p];
                    }
        }
        for (double &v : A) v *= -1.0 / kFourPi;
        if (!invert(A, m)) {
            sparc_poisson_destroy(P);
            return fail(SPARC_E_HIP, "block matrix is singular");
        }
        // symmetrise (the inverse of a symmetric matrix; removes rounding asymmetry)
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) {
                const double s = 0.5 * (A[(size_t)i * m + j] + A[(size_t)j * m + i]);
                A[(size_t)i * m + j] = A[(size_t)j * m + i] = s;
            }
        std::copy(A.begin(), A.end(), minv.begin() + (size_t)code * q.maxm * q.maxm);
    }
    std::vector<double> wv(kMaxRadius + 1, 0.0);
    for (int p = 0; p <= grid->radius; ++p) wv[p] = w[p];
    if (hipMalloc(&P->d_minv, minv.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&P->d_w, wv.size() * sizeof(double)) != hipSuccess) {
        sparc_poisson_destroy(P);
        return fail(SPARC_E_NOMEM, "device allocation failed");
    }
    if (hipMemcpy(P->d_minv, minv.data(), minv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P->d_w, wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        sparc_poisson_destroy(P);
        return fail(SPARC_E_HIP, "copy of the block inverses failed");
    }
    P->nmom = (int)std::max<long long>(1, std::min<long long>(256, (nd + kPT - 1) / kPT));
    P->nred = (int)std::max<long long>(1, std::min<long long>(kRedMax, (nd + 4 * kPT - 1) / (4 * kPT)));
    const int G = kPT / q.maxm;
    const long long bricks = (long long)q.nb[0] * q.nb[1] * ((q.nb[2] + G - 1) / G);
    P->nbjg = (int)std::max<long long>(1, std::min<long long>(kRedMax, bricks));
    *out = P;
    return SPARC_OK;
}

extern "C" int sparc_poisson_destroy(sparc_poisson *P)
{
    if (!P) return SPARC_OK;
    (void)hipFree(P->d_minv);
    (void)hipFree(P->d_w);
    sparc_op_destroy(P->op0);
    delete P;
    return SPARC_OK;
}

extern "C" size_t sparc_poisson_workspace_bytes(const sparc_poisson *P)
{
    if (!P) return 0;
    return carve(P, nullptr).total;
}

extern "C" int sparc_poisson_solve(sparc_poisson *P, const double *charge, double *phi, int32_t use_guess, double tol,
                                   int32_t max_iter, int32_t *iters, double *rel_resid, double *moments, void *ws,
                                   size_t ws_bytes, void *stream)
{
    if (!P || !charge || !phi) return fail(SPARC_E_ARG, "null argument");
    if (!(tol > 0.0) || max_iter < 0) return fail(SPARC_E_ARG, "need tol > 0 and max_iter >= 0");
    const PoisWs W = carve(P, ws);
    if (!ws || ws_bytes < W.total) return fail(SPARC_E_WORKSPACE, "workspace missing or too small");
    const long long nd = P->g.nd;
    const char *c0 = (const char *)charge, *c1 = c0 + nd * 8, *f0 = (const char *)phi, *f1 = f0 + nd * 8;
    const char *w0 = (const char *)ws, *w1 = w0 + W.total;
    if ((c0 < f1 && f0 < c1) || (w0 < f1 && f0 < w1) || (w0 < c1 && c0 < w1))
        return fail(SPARC_E_ALIAS, "charge, phi and the workspace must not overlap");
    TraceRange trace("sparc_poisson_solve");
    hipStream_t s = (hipStream_t)stream;
    const int nvec = P->nred;
    ProfScope prof(6, s);
    // multipole moments and the boundary values of phi
    hipLaunchKernelGGL(moments_kernel, dim3(P->nmom), dim3(kPT), 0, s, charge, P->g, P->nrm, W.mpart);
    hipLaunchKernelGGL(moments_finish, dim3(1), dim3(kPT), 0, s, (const double *)W.mpart, P->nmom,
                       P->g.h * P->g.h * P->g.h, P->lmax, W.Q);
    const long long sb = (P->slab_total + kPT - 1) / kPT;
    if (sb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "grid too large");
    hipLaunchKernelGGL(slab_kernel, dim3((unsigned)sb), dim3(kPT), 0, s, P->g, P->sg, P->nrm, P->lmax,
                       (const double *)W.Q, W.slab, P->slab_total);
    // right-hand side into r
    hipLaunchKernelGGL(rhs_kernel, dim3(nvec), dim3(kPT), 0, s, charge, P->g, P->sg, (const double *)P->d_w,
                       (const double *)W.slab, W.r, W.bb);
    const FLaunch V = choose_vec_launch(P->op0, SPARC_F64, 1, {nd, nd});
    const StepLaunch L = choose_step_launch(P->op0, SPARC_F64, 1);
    const StepCoef cA{1.0 / (2.0 * M_PI), 0.0, 0.0, 0};  // A = (1/2 pi)(-1/2 lap_h)
    int st;
    if (use_guess) {
        if ((st = launch_h_step(P->op0, SPARC_F64, phi, nd, nullptr, 0, W.q, nd, 1, nullptr, cA, L, s, &V))) return st;
        hipLaunchKernelGGL(axpy_kernel, dim3(nvec), dim3(kPT), 0, s, W.r, (const double *)W.q, -1.0, nd);
    } else {
        hipLaunchKernelGGL(fill_kernel, dim3(nvec), dim3(kPT), 0, s, phi, nd);
    }
    hipLaunchKernelGGL(bj_kernel<false>, dim3(P->nbjg), dim3(kPT), 0, s, P->bj, (const double *)P->d_minv, phi, W.r,
                       W.p, (const double *)nullptr, W.z, (const double *)nullptr, 0, (const double *)nullptr, 0,
                       W.rz[0], W.rr, (const PcgState *)W.state);
    const double tol2 = tol * tol;
    hipLaunchKernelGGL(pcg_start_kernel, dim3(1), dim3(kPT), 0, s, (const double *)W.rr, P->nbjg,
                       (const double *)W.bb, nvec, tol2, W.state);
    SPARC_HIP(hipGetLastError());
    PcgState hs{};
    SPARC_HIP(hipMemcpyAsync(&hs, W.state, sizeof(hs), hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    int it = 0;
    while (!hs.done && it < max_iter) {
        const int chunk = std::min(kChunk, max_iter - it);
        for (int c = 0; c < chunk; ++c, ++it) {
            const int o = it & 1;  // rz of this iteration's input in rz[o], its output in rz[1 - o]
            if ((st = launch_h_step(P->op0, SPARC_F64, W.p, nd, nullptr, 0, W.q, nd, 1, nullptr, cA, L, s, &V)))
                return st;
            hipLaunchKernelGGL(dot_kernel, dim3(nvec), dim3(kPT), 0, s, (const double *)W.p, (const double *)W.q, nd,
                               W.pq, (const PcgState *)W.state);
            hipLaunchKernelGGL(bj_kernel<true>, dim3(P->nbjg), dim3(kPT), 0, s, P->bj, (const double *)P->d_minv, phi,
                               W.r, W.p, (const double *)W.q, W.z, (const double *)W.rz[o], P->nbjg,
                               (const double *)W.pq, nvec, W.rz[1 - o], W.rr, (const PcgState *)W.state);
            hipLaunchKernelGGL(pupdate_kernel, dim3(nvec), dim3(kPT), 0, s, W.p, (const double *)W.z, nd,
                               (const double *)W.rz[1 - o], (const double *)W.rz[o], (const double *)W.rr, P->nbjg,
                               (const double *)W.bb, nvec, tol2, it, W.state);
        }
        SPARC_HIP(hipGetLastError());
        SPARC_HIP(hipMemcpyAsync(&hs, W.state, sizeof(hs), hipMemcpyDeviceToHost, s));
        SPARC_HIP(hipStreamSynchronize(s));
    }
    if (moments) {
        SPARC_HIP(hipMemcpyAsync(moments, W.Q, (size_t)(P->lmax + 1) * (P->lmax + 1) * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
        SPARC_HIP(hipStreamSynchronize(s));
    }
    if (iters) *iters = hs.iters;
    if (rel_resid) *rel_resid = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
    return SPARC_OK;
}
