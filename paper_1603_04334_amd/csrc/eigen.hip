// Small generalized symmetric-definite eigensolver on the device, FP64.
//
// Solves H_s q = theta M_s q (the subspace problem of Sec. 3.4, Eq.
// SubspaceGeneralizedEigenproblem) for n <= kEigMax in a single workgroup
// with every matrix in LDS:
//   1. Cholesky factorisation M_s = L L^T (column by column);
//   2. X = L^{-1} by forward substitution, row by row with every column and
//      16 partial sums per entry in parallel, then C = X H_s X^T by two
//      small products (each thread a 2 x 2 block);
//   3. cyclic Jacobi on C with the round-robin (circle) ordering, so the n/2
//      rotations of a round touch disjoint rows/columns; the pairs of every
//      round are tabulated in LDS once.  A round is applied as one two-sided
//      update: one wave computes the round's rotations, and the thread owning
//      row pair k and column pair l maps the 2 x 2 block of C at (rows of k,
//      columns of l) through the row rotation of k and then the column
//      rotation of l, reading C from one LDS buffer and writing the other
//      (two barriers per round, C read and written once); the same thread
//      applies the column rotation of l to rows 2k, 2k+1 of Z, so the
//      rotation is read once per thread.
//      Sweeps stop when the off-diagonal mass is below 1e-30 of the total
//      (relative 1e-15 in norm) or after max_sweeps;
//   4. eigenvalues sorted ascending (stable), eigenvectors back-transformed
//      q = X^T z so that Q^T M_s Q = I.
// Rotation for the pair (p, q): with tau = (c_qq - c_pp) / (2 c_pq), the
// smaller root t = sign(tau) / (|tau| + sqrt(1 + tau^2)) of t^2 + 2 tau t = 1
// gives c = 1/sqrt(1 + t^2), s = t c; rows and columns p, q are replaced by
// (c x_p - s x_q, s x_p + c x_q), which zeroes c_pq.  Evaluated as
// d = c_qq - c_pp, e = 2 c_pq, r = sqrt(d^2 + e^2), u = |d| + r,
// c = u / sqrt(2 r u), s = sign(d) e / sqrt(2 r u) (the same t = sign(d) e / u,
// with two square roots and one division on the dependent path).
#include "internal.hpp"

namespace sparc {

constexpr int kEigMax = 64;
constexpr int kEigThreads = 1024;

__device__ inline double block_sum_eig(double v, double *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kEigThreads / 64; ++w) t += red[w];
    return t;
}

// D = op(A) op(B) (op: optional transpose) for n x n matrices in LDS, each
// thread a 2 x 2 block of D; entries of D beyond n are not written.  The
// caller synchronises.
__device__ inline void lds_gemm(const double (*A)[kEigMax + 1], const double (*B)[kEigMax + 1],
                                double (*D)[kEigMax + 1], int n, bool transa, bool transb)
{
    const int half = (n + 1) / 2;
    for (int e = threadIdx.x; e < half * half; e += blockDim.x) {
        const int r0 = 2 * (e / half), c0 = 2 * (e % half);
        const int r1 = min(r0 + 1, n - 1), c1 = min(c0 + 1, n - 1);
        double d00 = 0.0, d01 = 0.0, d10 = 0.0, d11 = 0.0;
        for (int k = 0; k < n; ++k) {
            const double a0 = transa ? A[k][r0] : A[r0][k], a1 = transa ? A[k][r1] : A[r1][k];
            const double b0 = transb ? B[c0][k] : B[k][c0];
            const double b1 = transb ? B[c1][k] : B[k][c1];
            d00 += a0 * b0;
            d01 += a0 * b1;
            d10 += a1 * b0;
            d11 += a1 * b1;
        }
        D[r0][c0] = d00;
        if (c0 + 1 < n) D[r0][c0 + 1] = d01;
        if (r0 + 1 < n) D[r0 + 1][c0] = d10;
        if (r0 + 1 < n && c0 + 1 < n) D[r0 + 1][c0 + 1] = d11;
    }
}

// Jacobi rotation (c, s) annihilating C[p][q], for a pair of the round;
// the identity for the padding pair of an odd n
__device__ inline void jacobi_params(const double (*C)[kEigMax + 1], int p, int q, int n, double &c, double &s)
{
    c = 1.0;
    s = 0.0;
    if (q < n && C[p][q] != 0.0) {
        const double e = 2.0 * C[p][q];
        const double d = C[q][q] - C[p][p];
        const double r = sqrt(d * d + e * e);
        if (r > 0.0) {  // zero only if both underflow: leave the pair
            const double u = fabs(d) + r;
            const double inv = 1.0 / sqrt(2.0 * r * u);
            c = u * inv;
            s = (d >= 0.0 ? e : -e) * inv;
        }
    }
}

// indices (p < q) of pair k in round r of the circle ordering over np indices
__device__ inline void round_pair(int np, int r, int k, int &p, int &q)
{
    if (k == 0) {
        p = np - 1;
        q = r;
    } else {
        p = (r + k) % (np - 1);
        q = (r - k + np - 1) % (np - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

__global__ void __launch_bounds__(kEigThreads) small_sygv_kernel(const double *__restrict__ Hs,
                                                                  const double *__restrict__ Ms, int n,
                                                                  double *theta, double *evec, int *info,
                                                                  int max_sweeps)
{
    __shared__ double CB[2][kEigMax][kEigMax + 1];  // C, double-buffered across Jacobi rounds
    __shared__ double Z[kEigMax][kEigMax + 1];
    __shared__ double L[kEigMax][kEigMax + 1];
    __shared__ double red[kEigThreads / 64];
    __shared__ double lam[kEigMax];
    __shared__ double2 rcs[kEigMax / 2];                 // (c, s) of each pair of the round
    __shared__ unsigned short rpq[kEigMax - 1][kEigMax / 2];  // p | q << 8 per round and pair
    __shared__ int rank[kEigMax];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int np = n + (n & 1);
    double (*C)[kEigMax + 1] = CB[0];

    for (int e = tid; e < np * np; e += nt) {
        const int i = e % np, j = e / np;  // column-major input, zero padding row/column for odd n
        const bool in = i < n && j < n;
        L[i][j] = in ? Ms[(long long)j * n + i] : 0.0;
        C[i][j] = in ? Hs[(long long)j * n + i] : 0.0;
    }
    if (tid == 0) bad = 0;
    __syncthreads();

    // 1. Cholesky, lower triangle of L
    for (int j = 0; j < n; ++j) {
        if (tid == 0) {
            const double d = L[j][j];
            if (!(d > 0.0)) bad = j + 1;
            L[j][j] = sqrt(d > 0.0 ? d : 1.0);
        }
        __syncthreads();
        if (bad) break;
        const double piv = L[j][j];
        for (int i = j + 1 + tid; i < n; i += nt) L[i][j] /= piv;
        __syncthreads();
        const int m = n - j - 1;
        for (int e = tid; e < m * m; e += nt) {
            const int i = j + 1 + e / m, k = j + 1 + e % m;
            if (k <= i) L[i][k] -= L[i][j] * L[k][j];
        }
        __syncthreads();
    }
    if (bad) {
        if (tid == 0) info[0] = bad;
        return;
    }

    // 2. X = L^{-1} (in Z): row i needs rows k < i; 16 lanes share each entry
    for (int i = 0; i < n; ++i) {
        const int c = tid >> 4, part = tid & 15;
        double acc = 0.0;
        if (c < i)
            for (int k = c + part; k < i; k += 16) acc += L[i][k] * Z[k][c];
        for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
        if (part == 0 && c < n) Z[i][c] = c < i ? -acc / L[i][i] : (c == i ? 1.0 / L[i][i] : 0.0);
        __syncthreads();
    }
    // W = X H_s (CB[1]), C = W X^T (CB[0]), symmetrised
    double (*W)[kEigMax + 1] = CB[1];
    lds_gemm(Z, C, W, n, false, false);
    __syncthreads();
    lds_gemm(W, Z, C, n, false, true);
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) {
        const int i = e % n, j = e / n;
        if (i < j) {
            const double v = 0.5 * (C[i][j] + C[j][i]);
            C[i][j] = v;
            C[j][i] = v;
        }
    }
    // keep X for the back-transform in L (the factor is no longer needed)
    for (int e = tid; e < n * n; e += nt) {
        const int i = e % n, j = e / n;
        L[i][j] = Z[i][j];
    }
    __syncthreads();
    for (int e = tid; e < n * np; e += nt) {
        const int i = e % n, j = e / n;
        Z[i][j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();

    // 3. cyclic Jacobi.  The work split is the same in every round: thread
    // (k, l) owns the block of row pair k and column pair l of C and rows
    // 2k, 2k+1 of Z.
    const int half = np / 2;
    for (int e = tid; e < (np - 1) * half; e += nt) {
        int p, q;
        round_pair(np, e / half, e % half, p, q);
        rpq[e / half][e % half] = (unsigned short)(p | (q << 8));
    }
    __syncthreads();
    const bool has_blk = tid < half * half;
    const int bk = has_blk ? tid / half : 0, bl = has_blk ? tid % half : 0;
    const int z0 = 2 * bk, z1 = 2 * bk + 1;
    int cur = 0;
    bool converged = n == 1;
    for (int sweep = 0; sweep <= max_sweeps && n > 1; ++sweep) {
        const double(*A)[kEigMax + 1] = CB[cur];
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < n * n; e += nt) {
            const int i = e % n, j = e / n;
            const double v = A[i][j] * A[i][j];
            tot += v;
            if (i != j) off += v;
        }
        off = block_sum_eig(off, red);
        tot = block_sum_eig(tot, red);
        if (!(off > 1e-30 * tot)) {
            converged = true;
            break;
        }
        // the test above also runs after the last sweep
        if (sweep == max_sweeps) break;
        for (int r = 0; r < np - 1; ++r) {
            const double(*S)[kEigMax + 1] = CB[cur];
            double(*D)[kEigMax + 1] = CB[cur ^ 1];
            if (tid < half) {
                const int pq = rpq[r][tid];
                double c, s;
                jacobi_params(S, pq & 255, pq >> 8, n, c, s);
                rcs[tid] = make_double2(c, s);
            }
            __syncthreads();
            if (has_blk) {
                const int pqk = rpq[r][bk], pql = rpq[r][bl];
                const int pk = pqk & 255, qk = pqk >> 8, pl = pql & 255, ql = pql >> 8;
                const double2 rk = rcs[bk], rl = rcs[bl];
                const double ck = rk.x, sk = rk.y, cl = rl.x, sl = rl.y;
                const double a = S[pk][pl], b = S[pk][ql], d = S[qk][pl], g = S[qk][ql];
                const double a1 = ck * a - sk * d, b1 = ck * b - sk * g;
                const double d1 = sk * a + ck * d, g1 = sk * b + ck * g;
                D[pk][pl] = cl * a1 - sl * b1;
                D[pk][ql] = sl * a1 + cl * b1;
                D[qk][pl] = cl * d1 - sl * g1;
                D[qk][ql] = sl * d1 + cl * g1;
                if (z0 < n) {
                    const double za = Z[z0][pl], zb = Z[z0][ql];
                    Z[z0][pl] = cl * za - sl * zb;
                    Z[z0][ql] = sl * za + cl * zb;
                }
                if (z1 < n) {
                    const double za = Z[z1][pl], zb = Z[z1][ql];
                    Z[z1][pl] = cl * za - sl * zb;
                    Z[z1][ql] = sl * za + cl * zb;
                }
            }
            cur ^= 1;
            __syncthreads();
        }
    }
    C = CB[cur];

    // 4. sort (stable ascending) and back-transform q = X^T z (into the other buffer)
    double(*Q)[kEigMax + 1] = CB[cur ^ 1];
    if (tid < n) lam[tid] = C[tid][tid];
    __syncthreads();
    if (tid < n) {
        int rk = 0;
        const double li = lam[tid];
        for (int j = 0; j < n; ++j) rk += (lam[j] < li) || (lam[j] == li && j < tid);
        rank[tid] = rk;
        theta[rk] = li;
    }
    __syncthreads();
    // Q = X^T Z
    lds_gemm(L, Z, Q, n, true, false);
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) {
        const int k = e % n, c = e / n;
        evec[(long long)rank[c] * n + k] = Q[k][c];
    }
    // n + 1: the off-diagonal mass was still above the tolerance after max_sweeps
    if (tid == 0) info[0] = converged ? 0 : n + 1;
}

int launch_small_sygv(const double *Hs, const double *Ms, int n, double *theta, double *evec, int *info,
                      hipStream_t stream)
{
    if (n < 1 || n > kEigMax) return fail(SPARC_E_ARG, "small eigensolver needs 1 <= n <= 64");
    hipLaunchKernelGGL(small_sygv_kernel, dim3(1), dim3(kEigThreads), 0, stream, Hs, Ms, n, theta, evec, info, 40);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

}  // namespace sparc
