/*
 * CPU FP64 oracle for the Chebyshev-filter hot path of real-space Kohn-Sham DFT
 * (Ghosh & Suryanarayana, "SPARC: Accurate and efficient finite-difference
 * formulation and parallel implementation of Density Functional Theory.
 * Part I: Isolated clusters", arXiv:1603.04334).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library: the finite-difference
 * weights, the operator and the filter recurrence are written out here again,
 * plainly, in the order the paper states them.  No blocking, no fusion.
 *
 * Layout: a grid function is n1*n2*n3 doubles with linear index
 * k + n3*(j + n2*i) (z fastest).  An orbital block is column-major: column c
 * starts at c*ld.
 *
 * Boundary conditions:
 *   bc = 0  zero Dirichlet: f = 0 at every index that is not a grid node
 *           (Sec. 3.1, the paragraph after Eq. FD:gradient).
 *   bc = 1  odd reflection about the walls at i = 0 and i = n+1 (1-based),
 *           a test-only mode under which discrete sine vectors are exact
 *           eigenvectors of the stencil; it is not part of the method.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ weights */

/* Laplacian weights, Sec. 3.1 Eq. weightsLap:
 *   w_0 = -(1/h^2) sum_{q=1}^{n_o} 1/q^2
 *   w_p = 2 (-1)^{p+1} (n_o!)^2 / (h^2 p^2 (n_o-p)! (n_o+p)!),  p = 1..n_o   */
static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

void oracle_fd_weights(int no, double h, double *w)
{
    double s = 0.0;
    for (int q = 1; q <= no; ++q) s += 1.0 / ((double)q * (double)q);
    w[0] = -s / (h * h);
    for (int p = 1; p <= no; ++p) {
        double sign = (p % 2 == 1) ? 1.0 : -1.0; /* (-1)^{p+1} */
        double num = 2.0 * sign * factorial(no) * factorial(no);
        double den = h * h * (double)p * (double)p * factorial(no - p) * factorial(no + p);
        w[p] = num / den;
    }
}

/* ------------------------------------------------------------- grid access */

/* value of f at 0-based index (i,j,k), which may lie off the grid */
static double fval(const double *f, int n1, int n2, int n3, int i, int j, int k, int bc)
{
    int idx[3] = {i, j, k};
    int n[3] = {n1, n2, n3};
    double sign = 1.0;
    for (int d = 0; d < 3; ++d) {
        int a = idx[d];
        if (a >= 0 && a < n[d]) continue;
        if (bc == 0) return 0.0;
        /* odd extension with period 2(n+1) in 1-based index a+1 */
        int per = 2 * (n[d] + 1);
        int r = (a + 1) % per;
        if (r < 0) r += per;
        if (r == 0 || r == n[d] + 1) return 0.0;
        if (r <= n[d]) {
            idx[d] = r - 1;
        } else {
            idx[d] = per - r - 1;
            sign = -sign;
        }
    }
    return sign * f[(int64_t)idx[2] + (int64_t)n3 * ((int64_t)idx[1] + (int64_t)n2 * idx[0])];
}

/* ------------------------------------------------------------ Laplacian */

/* Eq. FD:Laplacian: at each node, sum over p = 0..n_o of w_p times the six
 * values at distance p along the three axes.  The p = 0 term contributes the
 * centre value six times. */
void oracle_laplacian(int n1, int n2, int n3, double h, int no, int bc,
                      const double *f, double *out)
{
    double w[16];
    oracle_fd_weights(no, h, w);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            for (int k = 0; k < n3; ++k) {
                double s = 0.0;
                for (int p = 0; p <= no; ++p) {
                    double six = fval(f, n1, n2, n3, i + p, j, k, bc) + fval(f, n1, n2, n3, i - p, j, k, bc)
                               + fval(f, n1, n2, n3, i, j + p, k, bc) + fval(f, n1, n2, n3, i, j - p, k, bc)
                               + fval(f, n1, n2, n3, i, j, k + p, bc) + fval(f, n1, n2, n3, i, j, k - p, bc);
                    s += w[p] * six;
                }
                out[(int64_t)k + (int64_t)n3 * ((int64_t)j + (int64_t)n2 * i)] = s;
            }
}

/* ------------------------------------------------------------ nonlocal */

/* Atom description: box lower corner lo[3] (0-based), extents ext[3], nproj
 * projectors; chi holds nproj*ext0*ext1*ext2 values (projector slowest, then
 * x, y, z fastest), gamma holds nproj energies. */
typedef struct {
    int lo[3], ext[3], nproj;
    const double *chi;
    const double *gamma;
} oracle_atom;

/* Sec. 3.1 Eq. non-localPS:FD:
 *   (V_nl f)(x) = h^3 sum_J sum_lm gamma_Jl chi_Jlm(x) sum_{x'} chi_Jlm(x') f(x')
 * accumulated into out. */
static void vnl_add(int n1, int n2, int n3, double h, int natoms, const oracle_atom *atoms,
                    const double *f, double *out)
{
    (void)n1;
    double h3 = h * h * h;
    for (int J = 0; J < natoms; ++J) {
        const oracle_atom *a = &atoms[J];
        int64_t nbox = (int64_t)a->ext[0] * a->ext[1] * a->ext[2];
        for (int p = 0; p < a->nproj; ++p) {
            const double *chi = a->chi + (int64_t)p * nbox;
            double dot = 0.0;
            for (int bi = 0; bi < a->ext[0]; ++bi)
                for (int bj = 0; bj < a->ext[1]; ++bj)
                    for (int bk = 0; bk < a->ext[2]; ++bk) {
                        int64_t g = (int64_t)(a->lo[2] + bk)
                                  + (int64_t)n3 * ((int64_t)(a->lo[1] + bj) + (int64_t)n2 * (a->lo[0] + bi));
                        dot += chi[((int64_t)bi * a->ext[1] + bj) * a->ext[2] + bk] * f[g];
                    }
            double coef = h3 * a->gamma[p] * dot;
            for (int bi = 0; bi < a->ext[0]; ++bi)
                for (int bj = 0; bj < a->ext[1]; ++bj)
                    for (int bk = 0; bk < a->ext[2]; ++bk) {
                        int64_t g = (int64_t)(a->lo[2] + bk)
                                  + (int64_t)n3 * ((int64_t)(a->lo[1] + bj) + (int64_t)n2 * (a->lo[0] + bi));
                        out[g] += coef * chi[((int64_t)bi * a->ext[1] + bj) * a->ext[2] + bk];
                    }
        }
    }
}

/* ------------------------------------------------------------ Hamiltonian */

/* H f = -1/2 lap_h f + V_eff f + V_nl f  (Sec. 2 Eq. EL with V_eff = V_xc + phi,
 * discretised as in Sec. 3.1).  One column. */
static void h_apply_col(int n1, int n2, int n3, double h, int no, int bc, const double *veff,
                        int natoms, const oracle_atom *atoms, const double *f, double *out)
{
    int64_t nd = (int64_t)n1 * n2 * n3;
    oracle_laplacian(n1, n2, n3, h, no, bc, f, out);
    for (int64_t g = 0; g < nd; ++g) out[g] = -0.5 * out[g] + veff[g] * f[g];
    vnl_add(n1, n2, n3, h, natoms, atoms, f, out);
}

void oracle_h_apply(int n1, int n2, int n3, double h, int no, int bc, const double *veff,
                    int natoms, const oracle_atom *atoms,
                    const double *X, int64_t ldx, double *Y, int64_t ldy, int ns)
{
    for (int c = 0; c < ns; ++c)
        h_apply_col(n1, n2, n3, h, no, bc, veff, natoms, atoms, X + (int64_t)c * ldx, Y + (int64_t)c * ldy);
}

/* ------------------------------------------------------------ Chebyshev filter */

/* Sec. 3.4 Eq. ChebFilter and Alg. 2, in the scaled three-term form of the
 * Chebyshev-filtered subspace iteration the paper cites.  As printed, Alg. 2
 * reuses the first-step update sigma <- sigma/(2 - sigma^2) at every step and
 * multiplies by 2*sigma/e with the old sigma; that is exact only for the
 * first step, so the general recurrence of the cited method is used:
 *   e = (b - a)/2,  c = (b + a)/2,  sigma_1 = e/(a0 - c),  tau = 2/sigma_1
 *   Y_0 = X,  Y_1 = (sigma_1/e)(H - cI) X
 *   for k = 1..m-1:  sigma_{k+1} = 1/(tau - sigma_k)
 *                    Y_{k+1} = (2 sigma_{k+1}/e)(H - cI) Y_k - sigma_k sigma_{k+1} Y_{k-1}
 * so that Y_m = C_m((H - c)/e) X / C_m((a0 - c)/e).
 * scaled = 0 instead runs the plain recurrence of Eq. ChebFilter,
 *   Y_1 = ((H - cI)/e) X,  Y_{k+1} = 2((H - cI)/e) Y_k - Y_{k-1},
 * giving C_m((H - c)/e) X without the normalisation. */
void oracle_cheb_filter(int n1, int n2, int n3, double h, int no, int bc, const double *veff,
                        int natoms, const oracle_atom *atoms,
                        const double *X, int64_t ldx, double *Y, int64_t ldy, int ns,
                        int m, double a0, double a, double b, int scaled)
{
    int64_t nd = (int64_t)n1 * n2 * n3;
    double e = (b - a) / 2.0;
    double c = (b + a) / 2.0;
    double sigma1 = e / (a0 - c);
    double tau = 2.0 / sigma1;
    for (int col = 0; col < ns; ++col) {
        const double *x = X + (int64_t)col * ldx;
        double *y = Y + (int64_t)col * ldy;
        double *prev = (double *)malloc(sizeof(double) * nd);
        double *cur = (double *)malloc(sizeof(double) * nd);
        double *hv = (double *)malloc(sizeof(double) * nd);
        memcpy(prev, x, sizeof(double) * nd);
        /* Y_1 */
        h_apply_col(n1, n2, n3, h, no, bc, veff, natoms, atoms, prev, hv);
        double sigma = sigma1;
        double f1 = scaled ? sigma1 / e : 1.0 / e;
        for (int64_t g = 0; g < nd; ++g) cur[g] = f1 * (hv[g] - c * prev[g]);
        for (int k = 1; k < m; ++k) {
            h_apply_col(n1, n2, n3, h, no, bc, veff, natoms, atoms, cur, hv);
            double alpha, beta;
            double sigma_next = 1.0 / (tau - sigma);
            if (scaled) {
                alpha = 2.0 * sigma_next / e;
                beta = sigma * sigma_next;
            } else {
                alpha = 2.0 / e;
                beta = 1.0;
            }
            for (int64_t g = 0; g < nd; ++g) {
                double nxt = alpha * (hv[g] - c * cur[g]) - beta * prev[g];
                prev[g] = cur[g];
                cur[g] = nxt;
            }
            sigma = sigma_next;
        }
        memcpy(y, cur, sizeof(double) * nd);
        free(prev);
        free(cur);
        free(hv);
    }
}

/* number of OpenMP threads the oracle uses (reported with CPU timings) */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
