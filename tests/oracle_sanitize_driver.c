/*
 * Driver for the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_oracle_sanitizers.py; test infrastructure).
 *
 * Every entry point of oracle/sparc_oracle.c runs on grids whose stencil reaches
 * past the walls (radius 6 on 3-5 nodes, and a 9 x 8 x 7 grid), under both
 * boundary modes, with projector cubes that touch the low and the high walls,
 * padded leading dimensions, and the scaled and plain filter recurrences.  Besides
 * staying clean under the sanitizers, the runs check two facts that hold for any
 * correct implementation: H is symmetric under zero Dirichlet conditions
 * (Sec. 3.1 stencil and Eq. non-localPS:FD), and the degree-1 filter is the
 * shifted, scaled operator (Sec. 3.4, first step of the recurrence).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int lo[3], ext[3], nproj;
    const double *chi;
    const double *gamma;
} oracle_atom;

void oracle_fd_weights(int no, double h, double *w);
void oracle_laplacian(int n1, int n2, int n3, double h, int no, int bc, const double *f, double *out);
void oracle_h_apply(int n1, int n2, int n3, double h, int no, int bc, const double *veff, int natoms,
                    const oracle_atom *atoms, const double *X, int64_t ldx, double *Y, int64_t ldy, int ns);
void oracle_cheb_filter(int n1, int n2, int n3, double h, int no, int bc, const double *veff, int natoms,
                        const oracle_atom *atoms, const double *X, int64_t ldx, double *Y, int64_t ldy, int ns,
                        int m, double a0, double a, double b, int scaled);

static uint64_t rng_state = 0x9e3779b97f4a7c15ULL;

static double urand(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    z ^= z >> 31;
    return (double)(z >> 11) / 9007199254740992.0 - 0.5;
}

static double *fill(int64_t n)
{
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!p) exit(3);
    for (int64_t i = 0; i < n; ++i) p[i] = urand();
    return p;
}

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static int run_grid(int n1, int n2, int n3, double h)
{
    const int no = 6;
    const int64_t nd = (int64_t)n1 * n2 * n3;
    const int64_t ld = nd + 3; /* padded columns */
    const int ns = 3;
    double w[16];
    for (int o = 1; o <= no; ++o) oracle_fd_weights(o, h, w);

    /* two atoms: one cube at the low corner, one ending at the high walls */
    oracle_atom at[2];
    double *chi[2], *gam[2];
    for (int J = 0; J < 2; ++J) {
        at[J].ext[0] = n1 < 3 ? n1 : 3;
        at[J].ext[1] = n2 < 2 ? n2 : 2;
        at[J].ext[2] = n3 < 4 ? n3 : 4;
        for (int d = 0; d < 3; ++d) {
            const int n = d == 0 ? n1 : (d == 1 ? n2 : n3);
            at[J].lo[d] = J == 0 ? 0 : n - at[J].ext[d];
        }
        at[J].nproj = 4;
        chi[J] = fill((int64_t)at[J].nproj * at[J].ext[0] * at[J].ext[1] * at[J].ext[2]);
        gam[J] = fill(at[J].nproj);
        at[J].chi = chi[J];
        at[J].gamma = gam[J];
    }
    double *veff = fill(nd);
    double *X = fill(ld * ns);
    double *Y = fill(ld * ns);
    double *Z = fill(ld * ns);
    int bad = 0;

    for (int bc = 0; bc <= 1; ++bc) {
        oracle_laplacian(n1, n2, n3, h, no, bc, X, Y);
        oracle_h_apply(n1, n2, n3, h, no, bc, veff, 2, at, X, ld, Y, ld, ns);
        for (int scaled = 0; scaled <= 1; ++scaled)
            oracle_cheb_filter(n1, n2, n3, h, no, bc, veff, 2, at, X, ld, Z, ld, ns, 5, -2.0, 1.0, 40.0, scaled);
        for (int64_t i = 0; i < ld * ns; ++i)
            if (!isfinite(Y[i]) || !isfinite(Z[i])) bad = 1;
    }

    /* symmetry of H (zero Dirichlet): <x0, H x1> = <H x0, x1> */
    oracle_h_apply(n1, n2, n3, h, no, 0, veff, 2, at, X, ld, Y, ld, 2);
    const double l = dot(X, Y + ld, nd), r = dot(Y, X + ld, nd);
    const double scale = sqrt(dot(X, X, nd) * dot(Y + ld, Y + ld, nd)) + 1e-300;
    if (fabs(l - r) > 1e-12 * scale) {
        printf("H not symmetric on %dx%dx%d: %.17g vs %.17g\n", n1, n2, n3, l, r);
        bad = 1;
    }

    /* degree 1: Y_1 = (sigma_1/e)(H - c) X with sigma_1 = e/(a0 - c) */
    const double a0 = -2.0, a = 1.0, b = 40.0, e = (b - a) / 2.0, c = (b + a) / 2.0, s1 = e / (a0 - c);
    oracle_cheb_filter(n1, n2, n3, h, no, 0, veff, 2, at, X, ld, Z, ld, 1, 1, a0, a, b, 1);
    oracle_h_apply(n1, n2, n3, h, no, 0, veff, 2, at, X, ld, Y, ld, 1);
    double err = 0.0, mag = 0.0;
    for (int64_t g = 0; g < nd; ++g) {
        const double ref = (s1 / e) * (Y[g] - c * X[g]);
        err = fmax(err, fabs(Z[g] - ref));
        mag = fmax(mag, fabs(ref));
    }
    if (err > 1e-13 * (mag + 1.0)) {
        printf("degree-1 filter differs from (sigma_1/e)(H - c)X by %.3g\n", err);
        bad = 1;
    }

    for (int J = 0; J < 2; ++J) {
        free(chi[J]);
        free(gam[J]);
    }
    free(veff);
    free(X);
    free(Y);
    free(Z);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run_grid(3, 4, 5, 0.7);
    bad |= run_grid(9, 8, 7, 0.5);
    bad |= run_grid(1, 1, 13, 0.4);
    printf(bad ? "oracle sanitizer driver: FAILED\n" : "oracle sanitizer driver: ok\n");
    return bad;
}
