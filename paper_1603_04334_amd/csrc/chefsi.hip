// Repeated CheFSI passes (Sec. 3.4) on a resident orbital block.
//
// One pass: the Chebyshev filter with bounds (a0, lambda_c, b), the FP64
// Rayleigh-Ritz step, the Fermi level of the Ritz values (Eq.
// FermiEnergyConstraintFormulation) and the subspace rotation, which leaves
// the Ritz vectors in X.  The first SCF iteration of a calculation repeats the
// pass about three times from a random block, without a density update in
// between (Sec. 3.4, last paragraph); every later SCF iteration runs one
// pass.  The cutoff of a pass is the previous pass's Fermi level plus 0.1 Ha
// (Sec. 4); the first pass takes the caller's cutoff (from the Lanczos
// bounds).  b stays fixed: H does not change while the density is not
// updated.  a0 (the estimate of lambda_1) stays fixed unless a cutoff falls at
// or below it, which happens when the Lanczos estimate had not converged on a
// low state the filtered block then found: a0 becomes the lowest Ritz value
// of the previous pass (an upper bound of lambda_1 below that pass's Fermi
// level).  a0 only scales the filter's output, so the filtered subspace and
// the Ritz values do not depend on it.
//
// The passes are the paper's guard against rank loss: one filter of high
// degree concentrates every column on the lowest eigenvectors until the block
// is linearly dependent, and the orthogonalisation of each Rayleigh-Ritz step
// restores it.  When a pass still loses rank at the working precision (the
// Cholesky factorisation of M_s fails; in FP32 a random block filtered at the
// full degree can get there) the same pass is redone from the same input at
// half the degree, the same remedy one step further: the block is never
// promoted to a wider type.
#include <vector>

#include "internal.hpp"

namespace sparc {

constexpr double kCutoffShift = 0.1;  // lambda_c = previous Fermi level + 0.1 Ha (Sec. 4)

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ChefsiLayout {
    size_t y, fws, rr, evec, rot, occ, total;
};

ChefsiLayout chefsi_layout(const sparc_op *op, int dtype, int ns)
{
    ChefsiLayout L{};
    L.y = align256((size_t)op->nd * ns * elem_size(dtype));
    L.fws = align256(sparc_workspace_bytes(op, dtype, ns, 1));
    L.rr = align256(sparc_rr_workspace_bytes(op, dtype, ns));
    L.evec = align256((size_t)ns * ns * sizeof(double));
    L.rot = align256(sparc_rotate_workspace_bytes(dtype, ns));
    L.occ = align256((size_t)ns * sizeof(double));
    L.total = L.y + L.fws + L.rr + L.evec + L.rot + L.occ;
    return L;
}

}  // namespace

int chefsi_run(const sparc_op *op, int dtype, void *X, int64_t ldx, int ns, int m, int passes, double ne, double kT,
               double &a0, double a, double b, const ChefsiBuffers &B, double *theta, double *lambda_f,
               int32_t *degrees, double *rho, hipStream_t s, int *halvings)
{
    if (passes < 1) return fail(SPARC_E_ARG, "passes must be >= 1");
    if (m < 1 || !(a0 < a && a < b)) return fail(SPARC_E_BOUNDS, "need m >= 1 and a0 < a < b");
    if (!(kT > 0.0)) return fail(SPARC_E_ARG, "k_B T must be positive");
    if (!(ne > 0.0 && ne < 2.0 * ns)) return fail(SPARC_E_ARG, "need 0 < N_e < 2 ns");
    std::vector<double> th(ns), occ(ns);
    double cut = a, lf = 0.0;
    int st;
    for (int p = 0; p < passes; ++p) {
        TraceRange pass("chefsi pass");
        if (p > 0) {
            cut = lf + kCutoffShift;
            if (cut <= a0) a0 = th[0];  // th: the previous pass's Ritz values
            if (!(a0 < cut && cut < b))
                return fail(SPARC_E_BOUNDS, "cutoff from the Fermi level leaves the filter interval (a0, b)");
        }
        int deg = m;
        for (;;) {
            if ((st = sparc_cheb_filter(op, dtype, X, ldx, B.Y, B.ldy, ns, deg, a0, cut, b, B.fws, B.fws_bytes, s)))
                return st;
            st = sparc_rayleigh_ritz(op, dtype, B.Y, B.ldy, ns, th.data(), B.evec, B.rr, B.rr_bytes, s);
            if (st == SPARC_E_BREAKDOWN && g_rr_rank_deficient && deg > 1) {
                deg = (deg + 1) / 2;  // X is untouched until the rotation: filter it again
                if (halvings) ++*halvings;
                continue;
            }
            if (st) return st;
            break;
        }
        if ((st = sparc_fermi_level(th.data(), ns, ne, kT, &lf, occ.data()))) return st;
        if ((st = sparc_rotate(dtype, B.Y, B.ldy, op->nd, ns, B.evec, X, ldx, B.rot, B.rot_bytes, s))) return st;
        if (theta) std::copy(th.begin(), th.end(), theta + (size_t)p * ns);
        if (lambda_f) lambda_f[p] = lf;
        if (degrees) degrees[p] = deg;
    }
    if (rho) {
        SPARC_HIP(hipMemcpyAsync(B.occ, occ.data(), (size_t)ns * sizeof(double), hipMemcpyHostToDevice, s));
        if ((st = sparc_density(dtype, X, ldx, op->nd, ns, B.occ, op->h, rho, s))) return st;
    }
    SPARC_HIP(hipStreamSynchronize(s));  // the rotation is done and occ was read
    return SPARC_OK;
}

}  // namespace sparc

using namespace sparc;

extern "C" size_t sparc_chefsi_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns)
{
    if (!op || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32)) return 0;
    return chefsi_layout(op, dtype, ns).total;
}

extern "C" int sparc_chefsi(const sparc_op *op, int32_t dtype, void *X, int64_t ldx, int32_t ns, int32_t m,
                            int32_t passes, double ne, double kT, double a0, double a, double b, double *theta,
                            double *lambda_f, int32_t *degrees, double *rho, void *ws, size_t ws_bytes, void *stream)
{
    if (!op || !X || (dtype != SPARC_F64 && dtype != SPARC_F32)) return fail(SPARC_E_ARG, "bad arguments");
    if (ns < 1 || ldx < op->nd) return fail(SPARC_E_SHAPE, "ns < 1 or ldx < N_d");
    const ChefsiLayout L = chefsi_layout(op, dtype, ns);
    if (!ws || ws_bytes < L.total) return fail(SPARC_E_WORKSPACE, "workspace missing or too small");
    const size_t es = elem_size(dtype);
    const char *x0 = (const char *)X, *x1 = x0 + ((size_t)(ns - 1) * ldx + op->nd) * es;
    const char *w0 = (const char *)ws, *w1 = w0 + L.total;
    if (x0 < w1 && w0 < x1) return fail(SPARC_E_ALIAS, "X overlaps the workspace");
    if (rho) {
        const char *r0 = (const char *)rho, *r1 = r0 + (size_t)op->nd * sizeof(double);
        if ((r0 < x1 && x0 < r1) || (r0 < w1 && w0 < r1)) return fail(SPARC_E_ALIAS, "rho overlaps X or the workspace");
    }
    char *p = (char *)ws;
    ChefsiBuffers B{};
    B.Y = p;
    B.ldy = op->nd;
    p += L.y;
    B.fws = p;
    B.fws_bytes = L.fws;
    p += L.fws;
    B.rr = p;
    B.rr_bytes = L.rr;
    p += L.rr;
    B.evec = (double *)p;
    p += L.evec;
    B.rot = p;
    B.rot_bytes = L.rot;
    p += L.rot;
    B.occ = (double *)p;
    double a0w = a0;
    return chefsi_run(op, dtype, X, ldx, ns, m, passes, ne, kT, a0w, a, b, B, theta, lambda_f, degrees, rho,
                      (hipStream_t)stream, nullptr);
}
