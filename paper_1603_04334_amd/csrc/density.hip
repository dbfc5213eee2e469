// Occupations, Fermi energy and electron density (Sec. 3.4).
//
// After the Rayleigh-Ritz step the Fermi energy lambda_f is the root of the
// electron-count constraint 2 sum_n g_n = N_e (Eq.
// FermiEnergyConstraintFormulation), g_n the Fermi-Dirac occupation of Ritz
// value theta_n at smearing k_B T.  It is found on the host by Brent's method
// (the paper's choice, Sec. 4) over N_s scalars; no device work is involved.
//
// The density rho = (2/h^3) sum_n g_n psi_n^2 is one streaming pass over the
// rotated block: every lane owns one 16-byte run of grid points (4 FP32 or 2
// FP64 values), walks the N_s columns in ascending order with eight column
// loads in flight, and accumulates in FP64, so the result does not depend on
// the launch shape.  The pass reads s N_d N_s bytes and writes 8 N_d; it is
// bound by HBM bandwidth.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "internal.hpp"

namespace sparc {
namespace {

// The constraint 2 sum g_n - N_e, evaluated without cancellation: with
// n_below levels at or below l, it equals
//   2 ((n_below - N_e/2) + sum_{theta > l} g_n - sum_{theta <= l} (1 - g_n)),
// and both kinds of tail term are exp(-|theta - l|/kT) / (1 + exp(...)), so
// they stay accurate (down to underflow) however far the level lies from l.
double count_residual(const double *theta, int ns, double ne, double kT, double l)
{
    long below = 0;
    double above_tail = 0.0, below_tail = 0.0;
    for (int n = 0; n < ns; ++n) {
        const double d = theta[n] - l;
        const double e = std::exp(-std::fabs(d) / kT);
        const double t = e / (1.0 + e);
        if (d > 0) {
            above_tail += t;
        } else {
            ++below;
            below_tail += t;
        }
    }
    return 2.0 * (((double)below - 0.5 * ne) + (above_tail - below_tail));
}

// Brent's root finder (inverse quadratic interpolation, secant and bisection
// steps, keeping a sign-changing bracket [b, c]; R. P. Brent, Algorithms for
// Minimization without Derivatives, 1973, ch. 4).  f(lo) < 0 < f(hi).
template <typename F>
double brent_root(F f, double lo, double hi, double flo, double fhi, double abs_tol)
{
    double a = lo, fa = flo, b = hi, fb = fhi;
    double c = a, fc = fa, step = b - a, prev_step = step;
    for (int it = 0; it < 300; ++it) {
        if ((fb > 0) == (fc > 0)) {  // keep the root between b and c
            c = a;
            fc = fa;
            step = prev_step = b - a;
        }
        if (std::fabs(fc) < std::fabs(fb)) {  // b is the best estimate so far
            a = b;
            b = c;
            c = a;
            fa = fb;
            fb = fc;
            fc = fa;
        }
        const double tol = 2.0 * DBL_EPSILON * std::fabs(b) + 0.5 * abs_tol;
        const double half = 0.5 * (c - b);
        if (std::fabs(half) <= tol || fb == 0.0) return b;
        if (std::fabs(prev_step) >= tol && std::fabs(fa) > std::fabs(fb)) {
            // interpolate: secant through (a, b), or an inverse quadratic
            // through a, b and c when all three differ
            double p, q;
            const double s = fb / fa;
            if (a == c) {
                p = 2.0 * half * s;
                q = 1.0 - s;
            } else {
                const double qa = fa / fc, r = fb / fc;
                p = s * (2.0 * half * qa * (qa - r) - (b - a) * (r - 1.0));
                q = (qa - 1.0) * (r - 1.0) * (s - 1.0);
            }
            if (p > 0)
                q = -q;
            else
                p = -p;
            // accept the interpolated point only if it falls well inside the
            // bracket and the steps keep shrinking; otherwise bisect
            if (2.0 * p < std::min(3.0 * half * q - std::fabs(tol * q), std::fabs(prev_step * q))) {
                prev_step = step;
                step = p / q;
            } else {
                step = prev_step = half;
            }
        } else {
            step = prev_step = half;
        }
        a = b;
        fa = fb;
        b += std::fabs(step) > tol ? step : (half > 0 ? tol : -tol);
        fb = f(b);
    }
    return b;
}

template <typename T>
struct DenVec;
template <>
struct DenVec<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};
template <>
struct DenVec<double> {
    typedef double V __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};

constexpr int kDenThreads = 256;
constexpr int kDenUnroll = 8;  // column loads in flight per lane

// rho[i] = scale * sum_n occ[n] * psi_n[i]^2, columns in ascending order.
// Lane t owns points [N t, N t + N); VEC: full 16-byte runs (ld and the
// block's address are multiples of N elements / 16 bytes), else scalar loads.
template <typename T, bool VEC>
__global__ void __launch_bounds__(kDenThreads)
    density_kernel(const T *__restrict__ psi, long long ld, long long nd, int ns, const double *__restrict__ occ,
                   double scale, double *__restrict__ rho)
{
    constexpr int N = DenVec<T>::N;
    using V = typename DenVec<T>::V;
    const long long i0 = ((long long)blockIdx.x * kDenThreads + threadIdx.x) * N;
    if (i0 >= nd) return;
    double acc[N];
#pragma unroll
    for (int p = 0; p < N; ++p) acc[p] = 0.0;
    if (VEC && i0 + N <= nd) {
        const V *col = (const V *)(psi + i0);
        const long long ldv = ld / N;
        int n = 0;
        for (; n + kDenUnroll <= ns; n += kDenUnroll) {
            V x[kDenUnroll];
#pragma unroll
            for (int j = 0; j < kDenUnroll; ++j) x[j] = col[(long long)(n + j) * ldv];
#pragma unroll
            for (int j = 0; j < kDenUnroll; ++j) {
                const double g = occ[n + j];
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    const double v = (double)x[j][p];
                    acc[p] += g * v * v;
                }
            }
        }
        for (; n < ns; ++n) {
            const V x = col[(long long)n * ldv];
            const double g = occ[n];
#pragma unroll
            for (int p = 0; p < N; ++p) {
                const double v = (double)x[p];
                acc[p] += g * v * v;
            }
        }
    } else {
        const int np = (int)std::min<long long>(N, nd - i0);
        for (int n = 0; n < ns; ++n) {
            const double g = occ[n];
            const T *c = psi + (long long)n * ld + i0;
#pragma unroll
            for (int p = 0; p < N; ++p)
                if (p < np) {
                    const double v = (double)c[p];
                    acc[p] += g * v * v;
                }
        }
    }
#pragma unroll
    for (int p = 0; p < N; ++p)
        if (i0 + p < nd) rho[i0 + p] = scale * acc[p];
}

template <typename T>
int launch_density(const T *psi, long long ld, long long nd, int ns, const double *occ, double scale, double *rho,
                   hipStream_t s)
{
    constexpr int N = DenVec<T>::N;
    const long long lanes = (nd + N - 1) / N;
    const long long blocks = (lanes + kDenThreads - 1) / kDenThreads;
    if (blocks > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "grid too large for one density launch");
    const bool vec = ld % N == 0 && (uintptr_t)psi % 16 == 0;
    ProfScope prof(4, s);
    if (vec)
        hipLaunchKernelGGL((density_kernel<T, true>), dim3((unsigned)blocks), dim3(kDenThreads), 0, s, psi, ld, nd, ns,
                           occ, scale, rho);
    else
        hipLaunchKernelGGL((density_kernel<T, false>), dim3((unsigned)blocks), dim3(kDenThreads), 0, s, psi, ld, nd,
                           ns, occ, scale, rho);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

}  // namespace
}  // namespace sparc

using namespace sparc;

extern "C" int sparc_fermi_level(const double *theta, int32_t ns, double ne, double kT, double *lambda_f, double *occ)
{
    if (!theta || !lambda_f || ns < 1) return fail(SPARC_E_ARG, "bad arguments");
    if (!(kT > 0.0) || !std::isfinite(kT)) return fail(SPARC_E_ARG, "k_B T must be positive");
    if (!(ne > 0.0 && ne < 2.0 * ns)) return fail(SPARC_E_ARG, "need 0 < N_e < 2 N_s");
    double tmin = theta[0], tmax = theta[0];
    for (int n = 0; n < ns; ++n) {
        if (!std::isfinite(theta[n])) return fail(SPARC_E_ARG, "non-finite eigenvalue");
        tmin = std::min(tmin, theta[n]);
        tmax = std::max(tmax, theta[n]);
    }
    auto f = [&](double l) { return count_residual(theta, ns, ne, kT, l); };
    // the residual rises monotonically from -N_e to 2 N_s - N_e: widen a
    // bracket around the spectrum until it changes sign
    double lo = tmin - 40.0 * kT, hi = tmax + 40.0 * kT;
    double flo = f(lo), fhi = f(hi);
    for (int k = 0; k < 64 && flo >= 0; ++k) flo = f(lo -= 40.0 * kT * (1 << std::min(k, 20)));
    for (int k = 0; k < 64 && fhi <= 0; ++k) fhi = f(hi += 40.0 * kT * (1 << std::min(k, 20)));
    if (flo >= 0 || fhi <= 0) return fail(SPARC_E_BOUNDS, "no sign change of the electron-count residual");
    const double lf = brent_root(f, lo, hi, flo, fhi, 1e-15 * kT);
    *lambda_f = lf;
    if (occ)
        for (int n = 0; n < ns; ++n) {
            const double x = (theta[n] - lf) / kT;
            occ[n] = x > 0 ? std::exp(-x) / (1.0 + std::exp(-x)) : 1.0 / (1.0 + std::exp(x));
        }
    return SPARC_OK;
}

extern "C" int sparc_density(int32_t dtype, const void *psi, int64_t ld, int64_t nd, int32_t ns, const double *occ,
                             double h, double *rho, void *stream)
{
    if (!psi || !occ || !rho || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32))
        return fail(SPARC_E_ARG, "bad arguments");
    if (nd < 1 || ld < nd || !(h > 0.0)) return fail(SPARC_E_SHAPE, "need nd >= 1, ld >= nd, h > 0");
    const size_t es = elem_size(dtype);
    const char *p0 = (const char *)psi, *p1 = p0 + ((size_t)(ns - 1) * ld + nd) * es;
    const char *r0 = (const char *)rho, *r1 = r0 + (size_t)nd * sizeof(double);
    if (p0 < r1 && r0 < p1) return fail(SPARC_E_ALIAS, "rho overlaps the orbital block");
    const double scale = 2.0 / (h * h * h);
    TraceRange trace("sparc_density");
    hipStream_t s = (hipStream_t)stream;
    return dtype == SPARC_F64 ? launch_density((const double *)psi, ld, nd, ns, occ, scale, rho, s)
                              : launch_density((const float *)psi, ld, nd, ns, occ, scale, rho, s);
}
