// FP64 spectral-bound Lanczos, Rayleigh-Ritz projection and subspace rotation.
//
// Lanczos (Sec. 4: extremal eigenvalues of H by a few Lanczos iterations)
// runs entirely on the device: H v through the fused step kernel, then
// deterministic two-pass reductions for the inner products (one partial per
// block, then one fixed-order sum, finished by whichever kernel needs the
// value), and partial re-orthogonalisation against the stored basis, decided
// on the device by the omega recurrence.  The scalars stay on the device
// between steps, so the k steps are enqueued without host round trips; the
// tridiagonal T_k is copied back once and its eigenvalues are found on the
// host by Sturm-sequence bisection.
//
// Rayleigh-Ritz (Sec. 3.4, Eq. SubspaceGeneralizedEigenproblem): H Y is
// formed in FP64 by the fused kernels (an FP32 block is widened as it is
// loaded), H_s = Y^T (H Y) and M_s = Y^T Y come from one FP64 matrix-core
// kernel, and the symmetric-definite problem is solved on the device: in one
// workgroup (Cholesky + Jacobi) for up to 64 columns, beyond by rocSOLVER's
// Cholesky and divide-and-conquer eigensolver with the reduction to standard
// form and the back-transformation as rocBLAS triangular solves.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <map>
#include <vector>

#include "internal.hpp"

namespace sparc {

thread_local bool g_rr_rank_deficient = false;  // set by the last Rayleigh-Ritz call of this thread

constexpr int kRedBlocks = 1024;  // blocks of the first reduction pass: one partial per block
constexpr int kDotGroup = 8;      // vectors per pass over a block's segment
constexpr int kUnroll = 4;        // points per thread with loads in flight together

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// sum over the 4 waves of a 256-thread block, the same value in every thread
__device__ inline double block_sum(double v, double *red)
{
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const double t = (red[0] + red[1]) + (red[2] + red[3]);
    __syncthreads();
    return t;
}

// sum of entry i of the kRedBlocks block partials (stride per block) in one
// fixed order, so that every block that needs the value finishes it
// bitwise identically
__device__ inline double sum_partials(const double *partial, int stride, int i, double *red)
{
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < kRedBlocks / 256; ++u) v += partial[(long long)(threadIdx.x + 256 * u) * stride + i];
    return block_sum(v, red);
}

// the contiguous segment of n points owned by block b of a reduction pass
__device__ inline void block_segment(long long n, long long &beg, long long &end)
{
    const long long seg = ((n + kRedBlocks - 1) / kRedBlocks + 63) / 64 * 64;
    beg = blockIdx.x * seg;
    end = (beg + seg < n) ? beg + seg : n;
}

// block-level partial inner products: partial[b*(nv+1) + i] = sum over block
// b's points of V_i(x) w(x) for i < nv, and of w(x)^2 for i = nv.  Groups of
// 8 vectors per pass over the segment.
__device__ __forceinline__ void multidot_block(const double *__restrict__ V, long long ldv, int nv,
                                               const double *__restrict__ w, long long n,
                                               double *__restrict__ partial, double *red)
{
    long long beg, end;
    block_segment(n, beg, end);
    double *out = partial + (long long)blockIdx.x * (nv + 1);
    for (int i0 = 0; i0 <= nv; i0 += kDotGroup) {
        double acc[kDotGroup];
#pragma unroll
        for (int u = 0; u < kDotGroup; ++u) acc[u] = 0.0;
        for (long long x0 = beg + threadIdx.x; x0 < end; x0 += 256 * kUnroll) {
            double wx[kUnroll];
#pragma unroll
            for (int r = 0; r < kUnroll; ++r) {
                const long long x = x0 + 256 * r;
                wx[r] = x < end ? w[x] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kDotGroup; ++u) {
                const int i = i0 + u;
                if (i > nv) break;
                double vx[kUnroll];
#pragma unroll
                for (int r = 0; r < kUnroll; ++r) {
                    const long long x = x0 + 256 * r;
                    vx[r] = (i == nv) ? wx[r] : (x < end ? V[(long long)i * ldv + x] : 0.0);
                }
#pragma unroll
                for (int r = 0; r < kUnroll; ++r) acc[u] += vx[r] * wx[r];
            }
        }
#pragma unroll
        for (int u = 0; u < kDotGroup; ++u) {
            const double t = block_sum(acc[u], red);
            if (threadIdx.x == 0 && i0 + u <= nv) out[i0 + u] = t;
        }
    }
}

__global__ void __launch_bounds__(256) multidot_kernel(const double *__restrict__ V, long long ldv, int nv,
                                                       const double *__restrict__ w, long long n,
                                                       double *__restrict__ partial)
{
    __shared__ double red[4];
    multidot_block(V, ldv, nv, w, n, partial, red);
}

// out[i] = sum over the block partials of entry i (stride per block), one
// block per i.  alpha_out[0] = out[alpha_index] if set; mode 1 stores the
// square root.
__global__ void __launch_bounds__(256) finish_sums(const double *partial, int stride, double *out,
                                                   double *alpha_out, int alpha_index, int mode, const int *run)
{
    if (run && !*run) return;
    __shared__ double red[4];
    const int i = blockIdx.x;
    const double t = sum_partials(partial, stride, i, red);
    if (threadIdx.x == 0) {
        out[i] = mode == 1 ? sqrt(t) : t;
        if (alpha_out && i == alpha_index) alpha_out[0] = t;
    }
}

// w -= sum_i coeff[i] V_i, and partial[b] = sum over block b's points of the new w^2
__global__ void __launch_bounds__(256) orth_apply_norm(double *w, const double *__restrict__ V, long long ldv, int nv,
                                                       const double *__restrict__ coeff, long long n,
                                                       double *__restrict__ partial, const int *run)
{
    if (run && !*run) return;
    __shared__ double red[4];
    long long beg, end;
    block_segment(n, beg, end);
    double nrm = 0.0;
    for (long long x0 = beg + threadIdx.x; x0 < end; x0 += 256 * kUnroll) {
        double s[kUnroll];
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) s[r] = 0.0;
        for (int i = 0; i < nv; ++i) {
            const double c = coeff[i];
#pragma unroll
            for (int r = 0; r < kUnroll; ++r) {
                const long long x = x0 + 256 * r;
                s[r] += c * (x < end ? V[(long long)i * ldv + x] : 0.0);
            }
        }
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
            const long long x = x0 + 256 * r;
            if (x < end) {
                const double v = w[x] - s[r];
                w[x] = v;
                nrm += v * v;
            }
        }
    }
    const double t = block_sum(nrm, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// alpha_j = v_j^T H v_j from its two parts: the step kernel's workgroup
// partials of v^T (H_loc v), and the projections g_p = chi_p^T v (the
// gather's split partials, nproj of them per split), since
// v^T V_nl v = sum_p hg_p g_p^2.  One fixed order in every block.
__device__ inline double lanczos_alpha(const double *dot, int nb, const double *gpart, const double *hg, int nproj,
                                       double *red)
{
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) v += dot[b];
    for (int p = threadIdx.x; p < nproj; p += 256) {
        double g = 0.0;
#pragma unroll
        for (int q = 0; q < kGatherSplit; ++q) g += gpart[(long long)q * nproj + p];
        v += hg[p] * g * g;
    }
    return block_sum(v, red);
}

__global__ void __launch_bounds__(256) alpha_finish(const double *dot, int nb, const double *gpart, const double *hg,
                                                    int nproj, double *alpha)
{
    __shared__ double red[4];
    const double a = lanczos_alpha(dot, nb, gpart, hg, nproj, red);
    if (threadIdx.x == 0) *alpha = a;
}

// three-term Lanczos step: alpha_j is finished first (block 0 stores it),
// then w -= alpha_j v_j + beta_{j-1} v_{j-1} (bprev may be null at j = 0) and
// partial[b] = sum over block b's points of the new w^2
__global__ void __launch_bounds__(256) lanczos_3term(double *w, const double *__restrict__ vj,
                                                     const double *__restrict__ vjm, const double *dot, int nb,
                                                     const double *gpart, const double *hg, int nproj,
                                                     double *alpha, const double *bprev, long long n,
                                                     double *__restrict__ partial)
{
    __shared__ double red[4];
    const double a = lanczos_alpha(dot, nb, gpart, hg, nproj, red);
    if (blockIdx.x == 0 && threadIdx.x == 0) *alpha = a;
    const double b = bprev ? *bprev : 0.0;
    const double *vm = bprev ? vjm : vj;
    long long beg, end;
    block_segment(n, beg, end);
    double nrm = 0.0;
    for (long long x0 = beg + threadIdx.x; x0 < end; x0 += 256 * kUnroll) {
        double wv[kUnroll], v1[kUnroll], v2[kUnroll];
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
            const long long x = x0 + 256 * r;
            const bool ok = x < end;
            wv[r] = ok ? w[x] : 0.0;
            v1[r] = ok ? vj[x] : 0.0;
            v2[r] = ok ? vm[x] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
            const long long x = x0 + 256 * r;
            if (x < end) {
                const double v = wv[r] - (a * v1[r] + b * v2[r]);
                w[x] = v;
                nrm += v * v;
            }
        }
    }
    const double t = block_sum(nrm, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Partial reorthogonalisation (Simon's omega recurrence).  Row j of the
// estimates holds v_j^T v_i, i < j; after the three-term step of step j
// (coefficients alpha_j and beta_j), for i < j
//   beta_j w'_i = beta_i w_{i+1} + (alpha_i - alpha_j) w_i + beta_{i-1} w_{i-1}
//                 - beta_{j-1} w''_i  (+ eps1 (beta_i + beta_j) for rounding),
// w = row j, w'' = row j-1, and w'_j = eps1 ||T|| / beta_j.  The new vector
// is orthogonalised against the whole basis when an estimate passes sqrt(eps)
// and, after that, once more on the next step; its row then restarts at eps1.
//
// Every workgroup of this kernel finishes beta_j = sqrt(sum of the block
// partials of |w|^2) (the same fixed order as finish_sums) and evaluates the
// recurrence and the decision itself, bitwise identically; workgroup 0 stores
// beta_j, row j+1, ||T|| (anorm[j+1]), full[j] (orthogonalise now) and
// owed[j+1] (orthogonalise the next vector too).  Per-step slots keep the
// values read (owed[j], anorm[j]) apart from those written.  When the
// vector is to be orthogonalised, the workgroups go on to the inner products
// V^T w with v_0 .. v_j (partials as multidot_kernel); otherwise they exit.
__global__ void __launch_bounds__(256) omega_dots_kernel(const double *alpha, double *beta, int j, double eps1,
                                                         const double *Wp, const double *Wc, double *Wn,
                                                         int *owed, int *full, double *anorm,
                                                         const double *npart, const double *__restrict__ V,
                                                         long long ldv, const double *__restrict__ w, long long n,
                                                         double *__restrict__ partial)
{
    __shared__ double red[4];
    __shared__ int sfull;
    const double bj = sqrt(sum_partials(npart, 1, 0, red));
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const double aj = alpha[j], bjm = j > 0 ? beta[j - 1] : 0.0;
        const double an = fmax(anorm[j], fabs(aj) + bj + bjm);
        double mx = 0.0;
        for (int i = lane; i < j; i += 64) {
            double t = beta[i] * Wc[i + 1] + (alpha[i] - aj) * Wc[i] - bjm * Wp[i];
            if (i > 0) t += beta[i - 1] * Wc[i - 1];
            t += copysign(eps1 * (beta[i] + bj), t);
            mx = fmax(mx, fabs(t / bj));
        }
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
        const double dj = eps1 * an / bj;
        const bool owe = owed[j] != 0;
        const bool f = owe || fmax(mx, dj) > 1.4901161193847656e-08;  // sqrt(eps)
        if (blockIdx.x == 0) {
            // second pass for the row values (cheap, avoids holding them across the reduction)
            for (int i = lane; i < j; i += 64) {
                double t = beta[i] * Wc[i + 1] + (alpha[i] - aj) * Wc[i] - bjm * Wp[i];
                if (i > 0) t += beta[i - 1] * Wc[i - 1];
                t += copysign(eps1 * (beta[i] + bj), t);
                Wn[i] = f ? eps1 : t / bj;
            }
            if (lane == 0) {
                beta[j] = bj;
                Wn[j] = f ? eps1 : dj;
                Wn[j + 1] = 1.0;
                anorm[j + 1] = an;
                full[j] = f ? 1 : 0;
                owed[j + 1] = (f && !owe) ? 1 : 0;
            }
        }
        if (lane == 0) sfull = f ? 1 : 0;
    }
    __syncthreads();
    if (!sfull) return;
    multidot_block(V, ldv, j + 1, w, n, partial, red);
}

// rows j = 0 (1 at i = 0) and j = -1 (zero); owed[0] = 0, anorm[0] = 0
__global__ void omega_init(double *rows, int len, int *owed, double *anorm)
{
    for (int i = threadIdx.x; i < 3 * len; i += blockDim.x) rows[i] = (i == 0) ? 1.0 : 0.0;
    if (threadIdx.x == 0) {
        owed[0] = 0;
        *anorm = 0.0;
    }
}

// dst = src / nrm.  When redo is null or *redo is set, nrm = sqrt(sum of the
// block partials of |src|^2) is finished here (block 0 stores it in *norm);
// otherwise nrm = *norm.  One 256-thread block per reduction segment.
__global__ void __launch_bounds__(256) scale_by_norm(double *dst, const double *__restrict__ src, double *norm,
                                                     const double *partial, const int *redo, long long n)
{
    __shared__ double red[4];
    double nrm;
    if (!redo || *redo) {
        nrm = sqrt(sum_partials(partial, 1, 0, red));
        if (blockIdx.x == 0 && threadIdx.x == 0) *norm = nrm;
    } else {
        nrm = *norm;
    }
    const double inv = 1.0 / nrm;
    long long beg, end;
    block_segment(n, beg, end);
    for (long long x0 = beg + threadIdx.x; x0 < end; x0 += 256 * kUnroll) {
        double v[kUnroll];
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
            const long long x = x0 + 256 * r;
            v[r] = x < end ? src[x] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < kUnroll; ++r) {
            const long long x = x0 + 256 * r;
            if (x < end) dst[x] = v[r] * inv;
        }
    }
}

__global__ void f64_to_f32_dense(const double *src, float *dst, long long n)
{
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

// ---------------------------------------------------------------- Rayleigh-Ritz projection
//
// M_s = Y^T Y and H_s = Y^T (HY) in FP64 on the matrix cores
// (v_mfma_f64_16x16x4f64).  The contraction runs over the N_d grid points,
// which are split into chunks; a workgroup owns one 64 x 64 tile pair of
// (M_s, H_s) on or above the diagonal for one chunk (both matrices are
// symmetric: the lower tiles are copies), stages 32-point slices of the three
// column panels in LDS (coalesced along the contiguous grid axis) and writes
// its partial tiles, which a second kernel sums in chunk order; the upper
// triangle is then mirrored.  Each of the four waves owns a 32 x 32 quarter of
// both tiles (2 x 2 MFMA blocks each).  Workgroup indices are remapped so
// that all tile pairs of one chunk run back to back on the same XCD: the ten
// pairs that read a column panel then share it in that XCD's L2, and each
// panel of a chunk comes from HBM about once.

constexpr int kRrTile = 64;
constexpr int kRrK = 32;  // chunks of the contraction are multiples of this

// Staged slice geometry per block type.  FP32 panels stay FP32 in LDS (widened
// when read as MFMA operands).  Row strides put the 16 rows x 4 points of one
// operand read in distinct banks.
template <typename TY>
struct RrSlice {
    static constexpr int K = kRrK;                              // points per slice
    static constexpr int SA = sizeof(TY) == 4 ? K + 4 : K + 1;  // Y panel row stride (elements)
    static constexpr int SH = K + 1;                            // HY panel row stride (doubles)
    static constexpr int CPP = 256 / K;                         // columns staged per pass
    static constexpr int NP = kRrTile / CPP;                    // passes per slice
};

__device__ inline void mfma_f64(double a, double b, double (&acc)[4])
{
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}

template <typename TY>
__global__ void __launch_bounds__(256, 2) rr_project_kernel(const TY *__restrict__ Y, long long ldy,
                                                          const double *__restrict__ HY, long long ldh, long long nd,
                                                          int ns, long long kchunk, double *__restrict__ partial)
{
    using G = RrSlice<TY>;
    constexpr int KS = G::K;
    __shared__ TY sA[kRrTile][G::SA];         // Y columns of the row tile, [col][k]
    __shared__ TY sB[kRrTile][G::SA];         // Y columns of the column tile
    __shared__ double sH[kRrTile][G::SH];     // HY columns of the column tile
    // (chunk, tile pair) from the XCD-contiguous workgroup order; tile pair
    // (ti <= tj) numbered in row order: both matrices are symmetric, so only
    // the upper tiles are formed
    const int nt = (ns + kRrTile - 1) / kRrTile;
    const int npairs = nt * (nt + 1) / 2;
    const int nb = (int)gridDim.x, wg = (int)blockIdx.x, xcd = wg & 7;
    const int t = xcd * (nb >> 3) + min(xcd, nb & 7) + (wg >> 3);
    const int chunk = t / npairs;
    int ti = 0, rem = t % npairs;
    while (rem >= nt - ti) {
        rem -= nt - ti;
        ++ti;
    }
    const int tj = ti + rem;
    const long long k0 = chunk * kchunk;
    const long long k1 = (k0 + kchunk < nd) ? k0 + kchunk : nd;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;  // wave's quarter
    const int li = lane & 15, lk = lane >> 4;
    const int kk = tid % KS;
    double accM[2][2][4] = {}, accH[2][2][4] = {};
    TY ra[G::NP], rb[G::NP];  // raw values of the next slice (keeps the loads in flight)
    double rh[G::NP];

    // thread -> (column c = CPP*pass + tid/KS, point kk = tid%KS of the slice).
    // On a diagonal tile pair both Y panels are the same columns: read and
    // stage them once.
    const bool diag = ti == tj;
    // Addresses: a workgroup-uniform 64-bit base per pass (column CPP*pass of
    // the tile) plus a 32-bit lane offset (its column within the pass times
    // the leading dimension, plus the point), so no 64-bit lane addresses
    // stay live across the slice loop.
    const int cl = tid / KS;
    auto fetch = [&](long long kb) {
        const long long k = kb + kk;
        const bool kin = k < k1;
        const unsigned oy = (unsigned)(cl * ldy + k), oh = (unsigned)(cl * ldh + k);
#pragma unroll
        for (int pass = 0; pass < G::NP; ++pass) {
            const int c0 = pass * G::CPP;
            const int ca = ti * kRrTile + c0 + cl, cb = tj * kRrTile + c0 + cl;
            const TY *ya = Y + (long long)(ti * kRrTile + c0) * ldy;
            const TY *yb = Y + (long long)(tj * kRrTile + c0) * ldy;
            const double *hb = HY + (long long)(tj * kRrTile + c0) * ldh;
            ra[pass] = (kin && ca < ns) ? ya[oy] : TY(0);
            if (!diag) rb[pass] = (kin && cb < ns) ? yb[oy] : TY(0);
            rh[pass] = (kin && cb < ns) ? hb[oh] : 0.0;
        }
    };
    fetch(k0);
    for (long long kb = k0; kb < k1; kb += KS) {
        __syncthreads();
#pragma unroll
        for (int pass = 0; pass < G::NP; ++pass) {
            const int c = pass * G::CPP + tid / KS;
            sA[c][kk] = ra[pass];
            if (!diag) sB[c][kk] = rb[pass];
            sH[c][kk] = rh[pass];
        }
        __syncthreads();
        if (kb + KS < k1) fetch(kb + KS);
        const TY(*SB)[G::SA] = diag ? sA : sB;
#pragma unroll
        for (int ks = 0; ks < KS; ks += 4) {
            double a[2], b[2], h[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                a[u] = (double)sA[wi + 16 * u + li][ks + lk];
                b[u] = (double)SB[wj + 16 * u + li][ks + lk];
                h[u] = sH[wj + 16 * u + li][ks + lk];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    mfma_f64(a[u], b[v], accM[u][v]);
                    mfma_f64(a[u], h[v], accH[u][v]);
                }
        }
    }
    // partial[(chunk*2 + which)][col][row] of the full ns x ns matrices
    const long long mat = (long long)ns * ns;
    double *pm = partial + (long long)chunk * 2 * mat;
    double *ph = pm + mat;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ti * kRrTile + wi + 16 * u + (lane >> 4) + 4 * r;
                const int col = tj * kRrTile + wj + 16 * v + (lane & 15);
                if (row < ns && col < ns) {
                    pm[(long long)col * ns + row] = accM[u][v][r];
                    ph[(long long)col * ns + row] = accH[u][v][r];
                }
            }
}

// Ms, Hs (column-major ns x ns) = sum over chunks of the partial tiles, in
// chunk order, for the entries of the upper tiles (row tile <= column tile)
__global__ void rr_reduce_kernel(const double *partial, int nchunks, int ns, double *Ms, double *Hs)
{
    const long long mat = (long long)ns * ns;
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= 2 * mat) return;
    const long long which = e / mat, off = e - which * mat;
    const int row = (int)(off % ns), col = (int)(off / ns);
    if (row / kRrTile > col / kRrTile) return;
    double s = 0.0;
#pragma unroll 16
    for (int c = 0; c < nchunks; ++c) s += partial[((long long)c * 2 + which) * mat + off];
    (which == 0 ? Ms : Hs)[off] = s;
}

// the lower triangle of an ns x ns column-major matrix copied from the upper
__global__ void mirror_upper(double *A, int ns)
{
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns && j < ns && i < j) A[(long long)i * ns + j] = A[(long long)j * ns + i];
}

static dim3 stream_grid(long long n)
{
    long long b = (n + 255) / 256;
    return dim3((unsigned)std::min<long long>(b, 4096));
}

// ---------------------------------------------------------------- rotation

// out(x, c) = sum_j Y(x, j) Q(j, c) for a block of RotTile::cols output
// columns.  One thread per grid point x: the row of Y is read in chunks of
// RotTile::k values (each load coalesced along x); Q comes as a zero-padded
// copy in the block's dtype, column-major with a leading dimension that is a
// multiple of the chunk, so Q(k0.., c) is contiguous and wave-uniform (scalar
// loads); each thread keeps the sums of its point in registers and every
// output column is written coalesced along x.  HBM-bound: Y is read once and
// out written once per column block.
template <typename T>
struct RotTile;
template <>
struct RotTile<float> {
    static constexpr int cols = 64, k = 16;
};
template <>
struct RotTile<double> {
    static constexpr int cols = 32, k = 16;
};

inline int rot_ldq(int ns) { return (ns + 15) / 16 * 16; }
template <typename T>
inline int rot_ncols(int ns)
{
    return (ns + RotTile<T>::cols - 1) / RotTile<T>::cols * RotTile<T>::cols;
}

// Qp(j, c) = Q(j, c) for j, c < ns, zero elsewhere (ldq x ncp, column-major)
template <typename T>
__global__ void pad_rotation(const double *__restrict__ Q, int ns, T *__restrict__ Qp, int ldq, int ncp)
{
    const long long total = (long long)ldq * ncp;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(e % ldq), c = (int)(e / ldq);
        Qp[e] = (j < ns && c < ns) ? (T)Q[(long long)c * ns + j] : T(0);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) rotate_kernel(const T *__restrict__ Y, long long ldy, const T *__restrict__ Qp,
                                                     int ldq, T *__restrict__ out, long long ldo, long long nd, int ns)
{
    constexpr int NC = RotTile<T>::cols, KC = RotTile<T>::k;
    const long long x = blockIdx.x * 256LL + threadIdx.x;
    const int c0 = blockIdx.y * NC;
    const long long xs = x < nd ? x : nd - 1;  // loads stay in bounds; the store is masked
    T acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = T(0);
    for (int k0 = 0; k0 < ns; k0 += KC) {
        T y[KC];
#pragma unroll
        for (int j = 0; j < KC; ++j) y[j] = (k0 + j < ns) ? Y[(long long)(k0 + j) * ldy + xs] : T(0);
        const T *q = Qp + (long long)c0 * ldq + k0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            T t = acc[c];
#pragma unroll
            for (int j = 0; j < KC; ++j) t += y[j] * q[(long long)c * ldq + j];
            acc[c] = t;
        }
    }
    if (x < nd) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c0 + c < ns) out[(long long)(c0 + c) * ldo + x] = acc[c];
    }
}

// ---------------------------------------------------------------- BLAS handles

// rocBLAS handles are not safe for concurrent use, and a handle's device
// workspace stays in use until the work enqueued with it has run.  Each call
// leases a handle from a per-device pool: one last used on the same stream
// (stream order protects its workspace) or one whose completion event has
// fired; otherwise a new handle is made.  Returning a lease records the event
// on the call's stream.  Handles are kept until the process ends.
namespace {
struct PooledBlas {
    rocblas_handle h = nullptr;
    hipEvent_t done = nullptr;
    hipStream_t last = nullptr;
};
std::mutex g_blas_mu;
std::map<int, std::vector<PooledBlas>> g_blas_free;

struct BlasLease {
    int dev = 0;
    hipStream_t stream;
    PooledBlas e;
    rocblas_handle h = nullptr;
    explicit BlasLease(hipStream_t s) : stream(s)
    {
        (void)hipGetDevice(&dev);
        bool found = false;
        {
            std::lock_guard<std::mutex> lk(g_blas_mu);
            auto &v = g_blas_free[dev];
            for (size_t i = 0; i < v.size(); ++i) {
                bool idle = v[i].last == s;
                if (!idle) {
                    const hipError_t q = hipEventQuery(v[i].done);
                    idle = q == hipSuccess;
                    // a pending event is the expected answer, not an error of
                    // this thread's later calls
                    if (q == hipErrorNotReady) (void)hipGetLastError();
                }
                if (idle) {
                    e = v[i];
                    v.erase(v.begin() + (long)i);
                    found = true;
                    break;
                }
            }
        }
        if (!found) {
            // handles are created one at a time (creation is not documented as thread-safe)
            std::lock_guard<std::mutex> lk(g_blas_mu);
            if (rocblas_create_handle(&e.h) != rocblas_status_success) {
                e.h = nullptr;
                return;
            }
            if (hipEventCreateWithFlags(&e.done, hipEventDisableTiming) != hipSuccess) {
                rocblas_destroy_handle(e.h);
                e.h = nullptr;
                return;
            }
            // no atomics: results must not depend on scheduling
            rocblas_set_atomics_mode(e.h, rocblas_atomics_not_allowed);
        }
        rocblas_set_stream(e.h, s);
        h = e.h;
    }
    ~BlasLease()
    {
        if (!h) return;
        (void)hipEventRecord(e.done, stream);
        e.last = stream;
        std::lock_guard<std::mutex> lk(g_blas_mu);
        g_blas_free[dev].push_back(e);
    }
    BlasLease(const BlasLease &) = delete;
    BlasLease &operator=(const BlasLease &) = delete;
};
// A HIP error state left behind by a library call that itself reported
// success.  The one code seen so far (hipErrorStreamCaptureUnsupported, after
// rocSOLVER's generalized eigensolver on worker threads that capture nothing)
// is cleared and
// counted, with its first occurrences written to stderr; any other code fails
// the call.
std::atomic<long long> g_cleared_errors{0};

int note_library_error(const char *call, hipError_t e)
{
    if (e != hipErrorStreamCaptureUnsupported)
        return fail(SPARC_E_HIP, std::string(call) + " returned success but left HIP error: " + hipGetErrorString(e));
    const long long n = ++g_cleared_errors;
    if (n <= 8)
        fprintf(stderr, "sparc: cleared HIP error left by %s after success (%s), occurrence %lld\n", call,
                hipGetErrorString(e), n);
    return SPARC_OK;
}
}  // namespace

// ---------------------------------------------------------------- tridiagonal eigenvalues

// number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
static int sturm_count(const double *alpha, const double *beta, int k, double x)
{
    int count = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double b2 = i > 0 ? beta[i - 1] * beta[i - 1] : 0.0;
        q = (alpha[i] - x) - (i > 0 ? b2 / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0) ++count;
    }
    return count;
}

static void tridiag_eigenvalues(const double *alpha, const double *beta, int k, double *theta)
{
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(beta[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(beta[i]) : 0.0);
        lo = std::min(lo, alpha[i] - r);
        hi = std::max(hi, alpha[i] + r);
    }
    const double pad = 1e-12 * std::max(1.0, std::max(std::fabs(lo), std::fabs(hi)));
    lo -= pad;
    hi += pad;
    for (int j = 0; j < k; ++j) {
        // the (j+1)-th smallest eigenvalue: smallest x with count(x) > j
        double a = lo, b = hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (a + b);
            if (mid <= a || mid >= b) break;
            if (sturm_count(alpha, beta, k, mid) > j)
                b = mid;
            else
                a = mid;
        }
        theta[j] = 0.5 * (a + b);
    }
}

}  // namespace sparc

using namespace sparc;

extern "C" {

size_t sparc_lanczos_workspace_bytes(const sparc_op *op, int32_t k)
{
    if (!op || k < 1) return 0;
    size_t b = align_up((size_t)op->nd * (k + 1) * sizeof(double));  // basis V_0..V_{k-1} and w
    b += gather_bytes(op, SPARC_F64, 1);                                  // gathered projections
    b += align_up((size_t)(4 * k + 8) * sizeof(double));                  // alpha, beta, coeff, norm
    b += align_up((size_t)kRedBlocks * (k + 3) * sizeof(double));         // block partial sums
    b += align_up((size_t)step_dot_blocks(op) * sizeof(double));           // v^T H_loc v partials
    b += align_up((size_t)(3 * (k + 2) + k + 1) * sizeof(double));        // omega rows, ||T|| per step
    b += align_up((size_t)(2 * k + 1) * sizeof(int));                       // reorthogonalisation flags per step
    return b;
}

// Lanczos with partial re-orthogonalisation: w = H v_j, alpha_j = v_j^T H v_j,
// w -= alpha_j v_j + beta_{j-1} v_{j-1}, beta_j = |w|; when the omega
// recurrence (omega_dots_kernel) estimates a loss of orthogonality beyond sqrt(eps),
// one classical Gram-Schmidt pass against v_0 .. v_j (c = V^T w, w -= V c) and
// a new beta_j; v_{j+1} = w / beta_j.  Every step is enqueued without a host
// round trip: the conditional pass reads its flag on the device.
int sparc_lanczos(const sparc_op *op, int32_t k, const double *v0, double *alpha, double *beta, double *theta,
                  void *ws, size_t ws_bytes, void *stream)
{
    if (!op || !v0 || !theta) return fail(SPARC_E_ARG, "null argument");
    if (k < 1 || k > op->nd) return fail(SPARC_E_ARG, "need 1 <= k <= N_d");
    const size_t need = sparc_lanczos_workspace_bytes(op, k);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    TraceRange trace("sparc_lanczos");
    hipStream_t s = (hipStream_t)stream;
    const long long n = op->nd;
    char *p = (char *)ws;
    double *V = (double *)p;  // k+1 vectors of n (the last is w)
    p += align_up((size_t)n * (k + 1) * sizeof(double));
    double *G = (double *)p;
    p += gather_bytes(op, SPARC_F64, 1);
    double *d_alpha = (double *)p;
    double *d_beta = d_alpha + k;
    double *d_coeff = d_beta + k;       // k + 1 entries (coefficients and |w|^2)
    double *d_norm = d_coeff + k + 2;
    p += align_up((size_t)(4 * k + 8) * sizeof(double));
    double *partial = (double *)p;                        // inner products, k + 2 per block
    double *npart = partial + (size_t)kRedBlocks * (k + 2);  // |w|^2, one per block
    p += align_up((size_t)kRedBlocks * (k + 3) * sizeof(double));
    double *dotp = (double *)p;  // step kernel partials of v_j^T H_loc v_j
    const int ndot = (int)step_dot_blocks(op);
    p += align_up((size_t)ndot * sizeof(double));
    double *rows = (double *)p;  // three rows of orthogonality estimates, k + 2 entries each
    double *d_anorm = rows + 3 * (k + 2);  // ||T|| estimate after each step (k + 1)
    p += align_up((size_t)(3 * (k + 2) + k + 1) * sizeof(double));
    int *d_owed = (int *)p;     // k + 1: orthogonalise the vector of step j regardless
    int *d_full = d_owed + k + 1;  // k: the vector of step j is orthogonalised
    double *w = V + (long long)k * n;
    const double eps1 = 0.5 * std::sqrt((double)n) * 2.220446049250313e-16;

    const dim3 rg(kRedBlocks), tb(256);
    int st;
    hipLaunchKernelGGL(omega_init, dim3(1), tb, 0, s, rows, k + 2, d_owed, d_anorm);
    // V_0 = v0 / |v0|
    hipLaunchKernelGGL(multidot_kernel, rg, tb, 0, s, v0, (long long)n, 0, v0, n, npart);
    hipLaunchKernelGGL(scale_by_norm, rg, tb, 0, s, V, v0, d_norm, (const double *)npart, (const int *)nullptr, n);
    const int nproj = op->nproj_total;
    for (int j = 0; j < k; ++j) {
        double *vj = V + (long long)j * n;
        // w = H v_j, with the two parts of alpha_j = v_j^T H v_j left as partials
        if ((st = launch_lanczos_h_f64(op, vj, w, dotp, G, s))) return st;
        if ((st = launch_scatter(op, SPARC_F64, w, n, 1, G, 1.0, s))) return st;
        if (j + 1 == k) {
            hipLaunchKernelGGL(alpha_finish, dim3(1), tb, 0, s, (const double *)dotp, ndot, (const double *)G,
                               (const double *)op->d_hg64, nproj, d_alpha + j);
            break;
        }
        // alpha_j; w -= alpha_j v_j + beta_{j-1} v_{j-1}; partials of |w|^2
        hipLaunchKernelGGL(lanczos_3term, rg, tb, 0, s, w, (const double *)vj, (const double *)(vj - (j > 0 ? n : 0)),
                           (const double *)dotp, ndot, (const double *)G, (const double *)op->d_hg64, nproj,
                           d_alpha + j, (const double *)(j > 0 ? d_beta + j - 1 : nullptr), n, npart);
        // beta_j, the orthogonality estimates and, when they ask for it, the
        // inner products of one classical Gram-Schmidt pass against
        // v_0 .. v_j, whose new |w|^2 partials the scaling kernel finishes
        // into beta_j
        const double *Wc = rows + (size_t)(j % 3) * (k + 2);
        const double *Wp = rows + (size_t)((j + 2) % 3) * (k + 2);
        double *Wn = rows + (size_t)((j + 1) % 3) * (k + 2);
        const int nv = j + 1;
        const int *full = d_full + j;
        hipLaunchKernelGGL(omega_dots_kernel, rg, tb, 0, s, (const double *)d_alpha, d_beta, j, eps1, Wp, Wc, Wn,
                           d_owed, d_full, d_anorm, (const double *)npart, (const double *)V, (long long)n,
                           (const double *)w, n, partial);
        hipLaunchKernelGGL(finish_sums, dim3(nv), tb, 0, s, (const double *)partial, nv + 1, d_coeff, nullptr, -1, 0,
                           full);
        hipLaunchKernelGGL(orth_apply_norm, rg, tb, 0, s, w, V, (long long)n, nv, d_coeff, n, npart, full);
        hipLaunchKernelGGL(scale_by_norm, rg, tb, 0, s, vj + n, (const double *)w, d_beta + j, (const double *)npart,
                           full, n);
        SPARC_HIP(hipGetLastError());
    }
    SPARC_HIP(hipGetLastError());
    std::vector<double> ha(k), hb(std::max(1, k - 1));
    SPARC_HIP(hipMemcpyAsync(ha.data(), d_alpha, k * sizeof(double), hipMemcpyDeviceToHost, s));
    if (k > 1) SPARC_HIP(hipMemcpyAsync(hb.data(), d_beta, (k - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    for (int j = 0; j + 1 < k; ++j)
        if (!(hb[j] > 0.0) || !std::isfinite(hb[j])) return fail(SPARC_E_BREAKDOWN, "Lanczos breakdown at step " + std::to_string(j));
    for (int j = 0; j < k; ++j)
        if (!std::isfinite(ha[j])) return fail(SPARC_E_BREAKDOWN, "non-finite Lanczos coefficient");
    tridiag_eigenvalues(ha.data(), hb.data(), k, theta);
    if (alpha) std::copy(ha.begin(), ha.end(), alpha);
    if (beta && k > 1) std::copy(hb.begin(), hb.begin() + (k - 1), beta);
    return SPARC_OK;
}

static long long rr_chunk(long long nd, int ns)
{
    // at least 512 workgroups in total (upper tile pairs x chunks) and at
    // least 8 chunks per XCD; chunks a multiple of the staged slice
    const long long nt = (ns + kRrTile - 1) / kRrTile;
    const long long tiles = nt * (nt + 1) / 2;
    long long nch = std::max<long long>(64, (512 + tiles - 1) / tiles);
    nch = std::max<long long>(1, std::min<long long>(nch, nd / kRrK));
    long long c = (nd + nch - 1) / nch;
    c = (c + kRrK - 1) / kRrK * kRrK;
    return std::max<long long>(c, kRrK);
}

size_t sparc_rr_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns)
{
    if (!op || ns < 1) return 0;
    size_t b = 0;
    b += align_up((size_t)op->nd * ns * sizeof(double));                           // H Y
    b += gather_bytes(op, SPARC_F64, ns);                                           // gathered projections
    b += 2 * align_up((size_t)ns * ns * sizeof(double));                           // H_s, M_s
    b += 2 * align_up((size_t)ns * sizeof(double)) + align_up(sizeof(int));       // D, E, info
    const long long nch = (op->nd + rr_chunk(op->nd, ns) - 1) / rr_chunk(op->nd, ns);
    b += align_up((size_t)nch * 2 * ns * ns * sizeof(double));                     // projection partials
    return b;
}

int sparc_rayleigh_ritz(const sparc_op *op, int32_t dtype, const void *Y, int64_t ldy, int32_t ns, double *theta,
                        double *evec, void *ws, size_t ws_bytes, void *stream)
{
    g_rr_rank_deficient = false;
    if (!op || !Y || !theta) return fail(SPARC_E_ARG, "null argument");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "bad dtype");
    if (ns < 1 || ldy < op->nd) return fail(SPARC_E_SHAPE, "ns < 1 or ldy < N_d");
    // the projection addresses a lane's point by a 32-bit element offset from
    // its pass's first column
    if ((long long)RrSlice<double>::CPP * ldy + op->nd >= (1LL << 32))
        return fail(SPARC_E_SHAPE, "ldy too large for the projection kernel");
    const size_t need = sparc_rr_workspace_bytes(op, dtype, ns);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    TraceRange trace("sparc_rayleigh_ritz");
    hipStream_t s = (hipStream_t)stream;
    const long long nd = op->nd;
    char *p = (char *)ws;
    double *HY = (double *)p;
    p += align_up((size_t)nd * ns * sizeof(double));
    double *G = (double *)p;
    p += gather_bytes(op, SPARC_F64, ns);
    double *Hs = (double *)p;
    p += align_up((size_t)ns * ns * sizeof(double));
    double *Ms = (double *)p;
    p += align_up((size_t)ns * ns * sizeof(double));
    double *D = (double *)p;
    p += align_up((size_t)ns * sizeof(double));
    double *E = (double *)p;
    p += align_up((size_t)ns * sizeof(double));
    int *info = (int *)p;
    p += align_up(sizeof(int));
    double *partial = (double *)p;

    int st;
    StepLaunch L = choose_step_launch(op, SPARC_F64, ns);
    StepCoef hc{1.0, 0.0, 0.0, 0};
    const long long kc = rr_chunk(nd, ns);
    const int nch = (int)((nd + kc - 1) / kc);
    const int nt = (ns + kRrTile - 1) / kRrTile;
    const dim3 pg((unsigned)(nch * (nt * (nt + 1) / 2)), 1, 1);
    if (dtype == SPARC_F64) {
        const FLaunch V = choose_vec_launch(op, SPARC_F64, ns, {ldy, nd});
        if ((st = launch_h_step(op, SPARC_F64, Y, ldy, nullptr, 0, HY, nd, ns, G, hc, L, s, &V))) return st;
        hipLaunchKernelGGL(rr_project_kernel<double>, pg, dim3(256), 0, s, (const double *)Y, (long long)ldy,
                           (const double *)HY, nd, nd, ns, kc, partial);
    } else {
        // H in FP64 on the FP32 values, widened as they are loaded
        const float *Yf = (const float *)Y;
        if ((st = launch_gather_f32_to_f64(op, Yf, ldy, ns, G, s))) return st;
        if ((st = launch_step_f32_to_f64(op, Yf, ldy, HY, nd, ns, hc, choose_mixed_launch(op, ns), s))) return st;
        if ((st = launch_scatter(op, SPARC_F64, HY, nd, ns, G, 1.0, s))) return st;
        hipLaunchKernelGGL(rr_project_kernel<float>, pg, dim3(256), 0, s, Yf, (long long)ldy, (const double *)HY, nd,
                           nd, ns, kc, partial);
    }
    const long long tot = 2LL * ns * ns;
    hipLaunchKernelGGL(rr_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, partial, nch, ns, Ms, Hs);
    dim3 tb(16, 16), tg((ns + 15) / 16, (ns + 15) / 16);
    hipLaunchKernelGGL(mirror_upper, tg, tb, 0, s, Hs, ns);
    hipLaunchKernelGGL(mirror_upper, tg, tb, 0, s, Ms, ns);
    SPARC_HIP(hipGetLastError());

    if (ns <= 64) {
        // one-workgroup Cholesky + Jacobi; eigenvectors land in Hs
        if ((st = launch_small_sygv(Hs, Ms, ns, D, Hs, info, s))) return st;
    } else {
        BlasLease lease(s);
        rocblas_handle hb = lease.h;
        if (!hb) return fail(SPARC_E_HIP, "rocblas_create_handle failed");
        // anything still pending here was left by an earlier call of this thread
        const hipError_t before = hipGetLastError();
        if (before != hipSuccess)
            return fail(SPARC_E_HIP, std::string("HIP error pending before the eigensolver: ") + hipGetErrorString(before));
        // M_s = U^T U (rocSOLVER Cholesky); the reduction to the standard
        // problem C = U^-T H_s U^-1 and the back-transformation q = U^-1 z by
        // blocked triangular solves (rocBLAS trsm); C z = theta z by rocSOLVER's
        // divide-and-conquer symmetric eigensolver.  (rocsolver_dsygvd's own
        // reduction issues ~600 matrix-vector solves per call at N_s = 600.)
        auto lib_call = [&](const char *what, rocblas_status rs) -> int {
            const hipError_t after = hipGetLastError();
            if (rs != rocblas_status_success)
                return fail(SPARC_E_HIP, std::string(what) + " failed: " + rocblas_status_to_string(rs) +
                                             (after != hipSuccess ? std::string(", HIP: ") + hipGetErrorString(after) : ""));
            if (after != hipSuccess) return note_library_error(what, after);
            return SPARC_OK;
        };
        if ((st = lib_call("rocsolver_dpotrf", rocsolver_dpotrf(hb, rocblas_fill_upper, ns, Ms, ns, info)))) return st;
        int pinfo = 0;
        SPARC_HIP(hipMemcpyAsync(&pinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
        SPARC_HIP(hipStreamSynchronize(s));
        if (pinfo != 0) {
            g_rr_rank_deficient = true;
            return fail(SPARC_E_BREAKDOWN, "Cholesky of M_s failed (info=" + std::to_string(pinfo) +
                                               "): the filtered block is numerically rank deficient");
        }
        const double one = 1.0;
        if ((st = lib_call("rocblas_dtrsm", rocblas_dtrsm(hb, rocblas_side_left, rocblas_fill_upper,
                                                          rocblas_operation_transpose, rocblas_diagonal_non_unit, ns,
                                                          ns, &one, Ms, ns, Hs, ns))))
            return st;
        if ((st = lib_call("rocblas_dtrsm", rocblas_dtrsm(hb, rocblas_side_right, rocblas_fill_upper,
                                                          rocblas_operation_none, rocblas_diagonal_non_unit, ns, ns,
                                                          &one, Ms, ns, Hs, ns))))
            return st;
        if ((st = lib_call("rocsolver_dsyevd",
                           rocsolver_dsyevd(hb, evec ? rocblas_evect_original : rocblas_evect_none, rocblas_fill_upper,
                                            ns, Hs, ns, D, E, info))))
            return st;
        if (evec && (st = lib_call("rocblas_dtrsm", rocblas_dtrsm(hb, rocblas_side_left, rocblas_fill_upper,
                                                                 rocblas_operation_none, rocblas_diagonal_non_unit, ns,
                                                                 ns, &one, Ms, ns, Hs, ns))))
            return st;
    }
    int hinfo = 0;
    SPARC_HIP(hipMemcpyAsync(theta, D, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    if (evec) SPARC_HIP(hipMemcpyAsync(evec, Hs, (size_t)ns * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) {
        if (ns <= 64 && hinfo == ns + 1)
            return fail(SPARC_E_BREAKDOWN, "Jacobi eigensolver did not converge within its sweep limit");
        if (ns > 64)
            return fail(SPARC_E_BREAKDOWN, "rocsolver_dsyevd: the tridiagonal eigensolver did not converge (info=" +
                                               std::to_string(hinfo) + ")");
        // the small solver's Cholesky factorisation of M_s failed (info = the
        // failing column)
        g_rr_rank_deficient = true;
        return fail(SPARC_E_BREAKDOWN, "Cholesky of M_s failed (info=" + std::to_string(hinfo) +
                                           "): the filtered block is numerically rank deficient");
    }
    return SPARC_OK;
}

int64_t sparc_cleared_hip_errors(void) { return g_cleared_errors.load(); }

size_t sparc_rotate_workspace_bytes(int32_t dtype, int32_t ns)
{
    if (ns < 1) return 0;
    if (dtype == SPARC_F64) return (size_t)rot_ldq(ns) * rot_ncols<double>(ns) * sizeof(double);
    if (dtype == SPARC_F32) return (size_t)rot_ldq(ns) * rot_ncols<float>(ns) * sizeof(float);
    return 0;
}

int sparc_rotate(int32_t dtype, const void *Y, int64_t ldy, int64_t nd, int32_t ns, const double *Q, void *out,
                 int64_t ldo, void *ws, size_t ws_bytes, void *stream)
{
    if (!Y || !Q || !out) return fail(SPARC_E_ARG, "null argument");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "bad dtype");
    if (ns < 1 || nd < 1 || ldy < nd || ldo < nd) return fail(SPARC_E_SHAPE, "bad shape");
    const size_t es = elem_size(dtype);
    const size_t by = (size_t)((ns - 1) * ldy + nd) * es, bo = (size_t)((ns - 1) * ldo + nd) * es;
    const char *pa = (const char *)Y, *pb = (const char *)out;
    if (pa < pb + bo && pb < pa + by) return fail(SPARC_E_ALIAS, "Y and out overlap");
    const size_t need = sparc_rotate_workspace_bytes(dtype, ns);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    const char *pw = (const char *)ws;
    if ((pw < pa + by && pa < pw + need) || (pw < pb + bo && pb < pw + need))
        return fail(SPARC_E_ALIAS, "workspace overlaps Y or out");
    TraceRange trace("sparc_rotate");
    hipStream_t s = (hipStream_t)stream;
    const unsigned gx = (unsigned)((nd + 255) / 256);
    const int ldq = rot_ldq(ns);
    // Blocks wider than one column block of the kernel below would re-read Y
    // once per block of output columns; the product is then a plain GEMM on
    // the matrix cores (rocBLAS, atomics off: deterministic).
    const bool gemm = ns > (dtype == SPARC_F64 ? RotTile<double>::cols : RotTile<float>::cols) &&
                      nd <= 0x7fffffffLL && ldy <= 0x7fffffffLL && ldo <= 0x7fffffffLL;
    if (gemm) {
        BlasLease lease(s);
        if (!lease.h) return fail(SPARC_E_HIP, "rocblas_create_handle failed");
        rocblas_status rs;
        if (dtype == SPARC_F64) {
            hipLaunchKernelGGL(pad_rotation<double>, stream_grid((long long)ldq * ns), dim3(256), 0, s, Q, ns,
                               (double *)ws, ldq, ns);
            const double one = 1.0, zero = 0.0;
            rs = rocblas_dgemm(lease.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)nd, ns, ns, &one,
                               (const double *)Y, (rocblas_int)ldy, (const double *)ws, ldq, &zero, (double *)out,
                               (rocblas_int)ldo);
        } else {
            hipLaunchKernelGGL(pad_rotation<float>, stream_grid((long long)ldq * ns), dim3(256), 0, s, Q, ns,
                               (float *)ws, ldq, ns);
            const float one = 1.0f, zero = 0.0f;
            rs = rocblas_sgemm(lease.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)nd, ns, ns, &one,
                               (const float *)Y, (rocblas_int)ldy, (const float *)ws, ldq, &zero, (float *)out,
                               (rocblas_int)ldo);
        }
        const hipError_t after = hipGetLastError();
        if (rs != rocblas_status_success)
            return fail(SPARC_E_HIP, std::string("rocBLAS GEMM of the rotation failed: ") + rocblas_status_to_string(rs));
        if (after != hipSuccess) return fail(SPARC_E_HIP, std::string("rotation: ") + hipGetErrorString(after));
        return SPARC_OK;
    }
    if (dtype == SPARC_F64) {
        const int ncp = rot_ncols<double>(ns);
        hipLaunchKernelGGL(pad_rotation<double>, stream_grid((long long)ldq * ncp), dim3(256), 0, s, Q, ns,
                           (double *)ws, ldq, ncp);
        hipLaunchKernelGGL(rotate_kernel<double>, dim3(gx, ncp / RotTile<double>::cols), dim3(256), 0, s,
                           (const double *)Y, (long long)ldy, (const double *)ws, ldq, (double *)out, (long long)ldo,
                           (long long)nd, ns);
    } else {
        const int ncp = rot_ncols<float>(ns);
        hipLaunchKernelGGL(pad_rotation<float>, stream_grid((long long)ldq * ncp), dim3(256), 0, s, Q, ns,
                           (float *)ws, ldq, ncp);
        hipLaunchKernelGGL(rotate_kernel<float>, dim3(gx, ncp / RotTile<float>::cols), dim3(256), 0, s,
                           (const float *)Y, (long long)ldy, (const float *)ws, ldq, (float *)out, (long long)ldo,
                           (long long)nd, ns);
    }
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

}  // extern "C"
