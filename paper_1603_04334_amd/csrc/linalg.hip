// FP64 spectral-bound Lanczos, Rayleigh-Ritz projection and subspace rotation.
//
// Lanczos (Sec. 4: extremal eigenvalues of H by a few Lanczos iterations)
// runs entirely on the device: H v through the fused step kernel, then
// deterministic two-pass reductions for the inner products (per-block partial
// sums, then one fixed-order sum), and full re-orthogonalisation against the
// stored basis.  The scalars stay on the device between steps, so the k steps
// are enqueued without host round trips; the tridiagonal T_k is copied back
// once and its eigenvalues are found on the host by Sturm-sequence bisection.
//
// Rayleigh-Ritz (Sec. 3.4, Eq. SubspaceGeneralizedEigenproblem): the block is
// promoted to FP64, H Y is formed by the fused kernel, H_s = Y^T (H Y) and
// M_s = Y^T Y are plain FP64 GEMMs (rocBLAS), and the symmetric-definite
// problem is solved on the device by rocSOLVER's dsygvd.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <map>

#include "internal.hpp"

namespace sparc {

constexpr int kRedBlocks = 512;  // blocks of the first reduction pass

// partial[b*nv + i] = sum over block b's points of V_i(x) * w(x)
__global__ void __launch_bounds__(256) multidot_kernel(const double *__restrict__ V, long long ldv, int nv,
                                                       const double *__restrict__ w, long long n,
                                                       double *__restrict__ partial)
{
    __shared__ double red[4];
    const long long chunk = (n + gridDim.x - 1) / gridDim.x;
    const long long beg = blockIdx.x * chunk;
    const long long end = (beg + chunk < n) ? beg + chunk : n;
    for (int i = 0; i < nv; ++i) {
        const double *v = V + (long long)i * ldv;
        double s = 0.0;
        for (long long x = beg + threadIdx.x; x < end; x += blockDim.x) s += v[x] * w[x];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) partial[(long long)blockIdx.x * nv + i] = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
    }
}

// out[i] = sum_b partial[b*nv + i] (fixed order); mode 1 stores sqrt of the sum
__global__ void multidot_finish(const double *partial, int nblocks, int nv, double *out, int mode)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * nv + i];
    out[i] = mode == 1 ? sqrt(s) : s;
}

// w -= alpha_j v_j + beta_{j-1} v_{j-1}
__global__ void lanczos_update(double *w, const double *vj, const double *vjm1, const double *alpha_j,
                               const double *beta_jm1, long long n)
{
    const double al = *alpha_j;
    const double be = beta_jm1 ? *beta_jm1 : 0.0;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x) {
        double r = w[x] - al * vj[x];
        if (vjm1) r -= be * vjm1[x];
        w[x] = r;
    }
}

// w -= sum_i coeff[i] V_i
__global__ void reorth_apply(double *w, const double *V, long long ldv, int nv, const double *coeff, long long n)
{
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < nv; ++i) s += coeff[i] * V[(long long)i * ldv + x];
        w[x] -= s;
    }
}

// dst = src / *norm
__global__ void scale_by_inverse(double *dst, const double *src, const double *norm, long long n)
{
    const double inv = 1.0 / *norm;
    for (long long x = blockIdx.x * (long long)blockDim.x + threadIdx.x; x < n; x += (long long)gridDim.x * blockDim.x)
        dst[x] = src[x] * inv;
}

__global__ void f32_to_f64(const float *src, long long lds, double *dst, long long ldd, long long nd, int ns)
{
    const long long total = nd * ns;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
        const long long c = t / nd, x = t - c * nd;
        dst[c * ldd + x] = (double)src[c * lds + x];
    }
}

__global__ void f64_to_f32_dense(const double *src, float *dst, long long n)
{
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}

// symmetrise an ns x ns matrix in place: A = (A + A^T)/2
__global__ void symmetrize(double *A, int ns)
{
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns && j < ns && i < j) {
        const double v = 0.5 * (A[(long long)j * ns + i] + A[(long long)i * ns + j]);
        A[(long long)j * ns + i] = v;
        A[(long long)i * ns + j] = v;
    }
}

static dim3 stream_grid(long long n)
{
    long long b = (n + 255) / 256;
    return dim3((unsigned)std::min<long long>(b, 4096));
}

// ---------------------------------------------------------------- BLAS handles

namespace {
std::mutex g_blas_mu;
std::map<int, rocblas_handle> g_blas;  // one handle per device
}  // namespace

static rocblas_handle blas_handle()
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto it = g_blas.find(dev);
    if (it != g_blas.end()) return it->second;
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
    g_blas[dev] = h;
    return h;
}

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
    b += align_up((size_t)std::max(1, op->nproj_total) * sizeof(double));  // gathered coefficients
    b += align_up((size_t)(3 * k + 4) * sizeof(double));                  // alpha, beta, coeff, norm
    b += align_up((size_t)kRedBlocks * (k + 1) * sizeof(double));         // partial sums
    return b;
}

int sparc_lanczos(const sparc_op *op, int32_t k, const double *v0, double *alpha, double *beta, double *theta,
                  void *ws, size_t ws_bytes, void *stream)
{
    if (!op || !v0 || !theta) return fail(SPARC_E_ARG, "null argument");
    if (k < 1 || k > op->nd) return fail(SPARC_E_ARG, "need 1 <= k <= N_d");
    const size_t need = sparc_lanczos_workspace_bytes(op, k);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const long long n = op->nd;
    char *p = (char *)ws;
    double *V = (double *)p;  // k+1 vectors of n (the last is w)
    p += align_up((size_t)n * (k + 1) * sizeof(double));
    double *G = (double *)p;
    p += align_up((size_t)std::max(1, op->nproj_total) * sizeof(double));
    double *d_alpha = (double *)p;
    double *d_beta = d_alpha + k;
    double *d_coeff = d_beta + k;
    double *d_norm = d_coeff + k;
    p += align_up((size_t)(3 * k + 4) * sizeof(double));
    double *partial = (double *)p;
    double *w = V + (long long)k * n;

    const dim3 sg = stream_grid(n);
    auto dots = [&](const double *Vb, int nv, const double *vec, double *outv, int mode) -> int {
        hipLaunchKernelGGL(multidot_kernel, dim3(kRedBlocks), dim3(256), 0, s, Vb, (long long)n, nv, vec, n, partial);
        hipLaunchKernelGGL(multidot_finish, dim3((nv + 63) / 64), dim3(64), 0, s, partial, kRedBlocks, nv, outv, mode);
        SPARC_HIP(hipGetLastError());
        return SPARC_OK;
    };
    int st;
    // V_0 = v0 / |v0|
    if ((st = dots(v0, 1, v0, d_norm, 1))) return st;
    hipLaunchKernelGGL(scale_by_inverse, sg, dim3(256), 0, s, V, v0, d_norm, n);
    StepLaunch L = choose_step_launch(op, SPARC_F64, 1);
    StepCoef hc{1.0, 0.0, 0.0, 0};
    for (int j = 0; j < k; ++j) {
        double *vj = V + (long long)j * n;
        if ((st = launch_gather(op, SPARC_F64, vj, n, 1, G, s))) return st;
        if ((st = launch_step(op, SPARC_F64, vj, n, nullptr, 0, w, n, 1, G, hc, L, s))) return st;
        if ((st = dots(vj, 1, w, d_alpha + j, 0))) return st;
        hipLaunchKernelGGL(lanczos_update, sg, dim3(256), 0, s, w, vj, j > 0 ? vj - n : nullptr, d_alpha + j,
                           j > 0 ? d_beta + (j - 1) : nullptr, n);
        for (int pass = 0; pass < 2; ++pass) {
            if ((st = dots(V, j + 1, w, d_coeff, 0))) return st;
            hipLaunchKernelGGL(reorth_apply, sg, dim3(256), 0, s, w, V, (long long)n, j + 1, d_coeff, n);
        }
        if (j + 1 < k) {
            if ((st = dots(w, 1, w, d_beta + j, 1))) return st;
            hipLaunchKernelGGL(scale_by_inverse, sg, dim3(256), 0, s, vj + n, w, d_beta + j, n);
        }
        SPARC_HIP(hipGetLastError());
    }
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

size_t sparc_rr_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns)
{
    if (!op || ns < 1) return 0;
    size_t b = 0;
    if (dtype == SPARC_F32) b += align_up((size_t)op->nd * ns * sizeof(double));  // promoted Y
    b += align_up((size_t)op->nd * ns * sizeof(double));                           // H Y
    b += align_up((size_t)std::max(1, op->nproj_total) * ns * sizeof(double));     // gathered coefficients
    b += 2 * align_up((size_t)ns * ns * sizeof(double));                           // H_s, M_s
    b += 2 * align_up((size_t)ns * sizeof(double)) + align_up(sizeof(int));       // D, E, info
    return b;
}

int sparc_rayleigh_ritz(const sparc_op *op, int32_t dtype, const void *Y, int64_t ldy, int32_t ns, double *theta,
                        double *evec, void *ws, size_t ws_bytes, void *stream)
{
    if (!op || !Y || !theta) return fail(SPARC_E_ARG, "null argument");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "bad dtype");
    if (ns < 1 || ldy < op->nd) return fail(SPARC_E_SHAPE, "ns < 1 or ldy < N_d");
    if (ldy > 0x7fffffffLL || op->nd > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "leading dimension exceeds 32 bits");
    const size_t need = sparc_rr_workspace_bytes(op, dtype, ns);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const long long nd = op->nd;
    char *p = (char *)ws;
    const double *Y64 = (const double *)Y;
    long long ld64 = ldy;
    if (dtype == SPARC_F32) {
        double *y = (double *)p;
        p += align_up((size_t)nd * ns * sizeof(double));
        hipLaunchKernelGGL(f32_to_f64, stream_grid(nd * ns), dim3(256), 0, s, (const float *)Y, (long long)ldy, y, nd, nd, ns);
        Y64 = y;
        ld64 = nd;
    }
    double *HY = (double *)p;
    p += align_up((size_t)nd * ns * sizeof(double));
    double *G = (double *)p;
    p += align_up((size_t)std::max(1, op->nproj_total) * ns * sizeof(double));
    double *Hs = (double *)p;
    p += align_up((size_t)ns * ns * sizeof(double));
    double *Ms = (double *)p;
    p += align_up((size_t)ns * ns * sizeof(double));
    double *D = (double *)p;
    p += align_up((size_t)ns * sizeof(double));
    double *E = (double *)p;
    p += align_up((size_t)ns * sizeof(double));
    int *info = (int *)p;

    int st;
    StepLaunch L = choose_step_launch(op, SPARC_F64, ns);
    if ((st = launch_gather(op, SPARC_F64, Y64, ld64, ns, G, s))) return st;
    StepCoef hc{1.0, 0.0, 0.0, 0};
    if ((st = launch_step(op, SPARC_F64, Y64, ld64, nullptr, 0, HY, nd, ns, G, hc, L, s))) return st;

    std::lock_guard<std::mutex> lk(g_blas_mu);
    rocblas_handle hb = blas_handle();
    if (!hb) return fail(SPARC_E_HIP, "rocblas_create_handle failed");
    rocblas_set_stream(hb, s);
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(hb, rocblas_operation_transpose, rocblas_operation_none, ns, ns, (int)nd, &one, Y64, (int)ld64,
                      HY, (int)nd, &zero, Hs, ns) != rocblas_status_success ||
        rocblas_dgemm(hb, rocblas_operation_transpose, rocblas_operation_none, ns, ns, (int)nd, &one, Y64, (int)ld64,
                      Y64, (int)ld64, &zero, Ms, ns) != rocblas_status_success)
        return fail(SPARC_E_HIP, "rocblas_dgemm failed");
    dim3 tb(16, 16), tg((ns + 15) / 16, (ns + 15) / 16);
    hipLaunchKernelGGL(symmetrize, tg, tb, 0, s, Hs, ns);
    hipLaunchKernelGGL(symmetrize, tg, tb, 0, s, Ms, ns);
    if (rocsolver_dsygvd(hb, rocblas_eform_ax, evec ? rocblas_evect_original : rocblas_evect_none, rocblas_fill_upper,
                         ns, Hs, ns, Ms, ns, D, E, info) != rocblas_status_success)
        return fail(SPARC_E_HIP, "rocsolver_dsygvd failed");
    int hinfo = 0;
    SPARC_HIP(hipMemcpyAsync(theta, D, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s));
    if (evec) SPARC_HIP(hipMemcpyAsync(evec, Hs, (size_t)ns * ns * sizeof(double), hipMemcpyDeviceToDevice, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (hinfo != 0) return fail(SPARC_E_HIP, "generalized eigensolver failed (info=" + std::to_string(hinfo) + ")");
    return SPARC_OK;
}

int sparc_rotate(int32_t dtype, const void *Y, int64_t ldy, int64_t nd, int32_t ns, const double *Q, void *out,
                 int64_t ldo, void *ws, size_t ws_bytes, void *stream)
{
    if (!Y || !Q || !out) return fail(SPARC_E_ARG, "null argument");
    if (ns < 1 || nd < 1 || ldy < nd || ldo < nd) return fail(SPARC_E_SHAPE, "bad shape");
    if (ldy > 0x7fffffffLL || ldo > 0x7fffffffLL || nd > 0x7fffffffLL)
        return fail(SPARC_E_SHAPE, "dimension exceeds 32 bits");
    const size_t es = elem_size(dtype);
    const size_t by = (size_t)((ns - 1) * ldy + nd) * es, bo = (size_t)((ns - 1) * ldo + nd) * es;
    const char *pa = (const char *)Y, *pb = (const char *)out;
    if (pa < pb + bo && pb < pa + by) return fail(SPARC_E_ALIAS, "Y and out overlap");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_blas_mu);
    rocblas_handle hb = blas_handle();
    if (!hb) return fail(SPARC_E_HIP, "rocblas_create_handle failed");
    rocblas_set_stream(hb, s);
    if (dtype == SPARC_F64) {
        const double one = 1.0, zero = 0.0;
        if (rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)nd, ns, ns, &one, (const double *)Y,
                          (int)ldy, Q, ns, &zero, (double *)out, (int)ldo) != rocblas_status_success)
            return fail(SPARC_E_HIP, "rocblas_dgemm failed");
        return SPARC_OK;
    }
    if (dtype != SPARC_F32) return fail(SPARC_E_ARG, "bad dtype");
    if (!ws || ws_bytes < (size_t)ns * ns * sizeof(float)) return fail(SPARC_E_WORKSPACE, "workspace too small");
    hipLaunchKernelGGL(f64_to_f32_dense, stream_grid((long long)ns * ns), dim3(256), 0, s, Q, (float *)ws,
                       (long long)ns * ns);
    const float one = 1.0f, zero = 0.0f;
    if (rocblas_sgemm(hb, rocblas_operation_none, rocblas_operation_none, (int)nd, ns, ns, &one, (const float *)Y,
                      (int)ldy, (const float *)ws, ns, &zero, (float *)out, (int)ldo) != rocblas_status_success)
        return fail(SPARC_E_HIP, "rocblas_sgemm failed");
    return SPARC_OK;
}

}  // extern "C"
