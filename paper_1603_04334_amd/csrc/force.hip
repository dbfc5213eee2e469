// Nonlocal component of the atomic forces (Sec. 3.6, Eqs.
// NonlocForce:Discrete and NonLocForce:U:W; Alg. 4):
//   f_J = -4 sum_n g_n sum_lm gamma_Jl Y_Jnlm W_Jnlm,
//   Y_Jnlm = h^3 sum_x psi_n chi_Jlm,  W_Jnlm = h^3 sum_x (grad_h psi_n) chi_Jlm,
// with grad_h the finite-difference gradient of Eq. gradient:approximate and
// zero Dirichlet padding.
//
// Design.  The paper forms grad_h psi_n on each atom's cube and contracts it
// with chi.  With zero padding the gradient matrix is antisymmetric, so
//   W_Jnlm[d] = h^3 sum_x psi_n(x) F_Jlm,d(x),  F_Jlm,d = -grad_h,d chi_Jlm,
// exactly: F lives on the cube widened by the stencil radius along d, is a
// property of the operator, and is built once (host, FP64) on the first call.
// Y and the three W components are then four projector-like contractions of
// the same block, which run on the matrix cores through the gather of the
// nonlocal operator (one gather record per atom and contraction, 4 natoms
// records in one launch), reading each orbital once per record instead of
// forming 3 N_s gradient fields.  A second kernel, one workgroup per atom,
// sums the split partials in a fixed order and reduces over orbitals and
// projectors in a fixed order, so the forces are reproducible bit for bit.
// FP32 blocks are widened as they are loaded; all sums are FP64.
#include <algorithm>
#include <vector>

#include "nonlocal_kernel.hpp"

namespace sparc {
namespace {

// w~_1..w~_no of Eq. gradient:approximate, the factorial ratio accumulated as
// a product of q factors (no - q + i) / (no + i)
void gradient_weights(int no, double h, double *w)
{
    for (int q = 1; q <= no; ++q) {
        double ratio = 1.0;
        for (int i = 1; i <= q; ++i) ratio *= double(no - q + i) / double(no + i);
        w[q] = ((q & 1) ? 1.0 : -1.0) * ratio / (h * q);
    }
}

int build_force_tables(const sparc_op *op)
{
    const int natoms = op->natoms;
    const int R = op->radius;
    double w[kMaxRadius + 1] = {0};
    gradient_weights(R, op->h, w);
    int64_t chi_total = 0;
    for (const AtomDev &a : op->atoms) chi_total += (int64_t)a.ext[0] * a.ext[1] * a.ext[2] * a.nproj;
    std::vector<double> chi(chi_total);
    SPARC_HIP(hipMemcpy(chi.data(), op->d_chi64, chi_total * sizeof(double), hipMemcpyDeviceToHost));

    std::vector<AtomDev> rec;
    std::vector<int> boff;
    std::vector<double> fun;
    rec.reserve(4 * natoms);
    for (int J = 0; J < natoms; ++J) {
        const AtomDev &A = op->atoms[J];
        const int cube = A.ext[0] * A.ext[1] * A.ext[2];
        // chi of atom J at grid node z (zero off the cube)
        auto chi_at = [&](int p, const int z[3]) {
            for (int e = 0; e < 3; ++e)
                if (z[e] < A.lo[e] || z[e] >= A.lo[e] + A.ext[e]) return 0.0;
            const int idx = ((z[0] - A.lo[0]) * A.ext[1] + (z[1] - A.lo[1])) * A.ext[2] + (z[2] - A.lo[2]);
            return chi[A.chi0 + (int64_t)p * cube + idx];
        };
        for (int r = 0; r < 4; ++r) {
            AtomDev F = A;
            const int d = r - 1;
            if (r > 0) {
                F.lo[d] = std::max(0, A.lo[d] - R);
                F.ext[d] = std::min(op->n[d], A.lo[d] + A.ext[d] + R) - F.lo[d];
            }
            F.proj0 = 4 * A.proj0 + r * A.nproj;
            if (boff.size() > 0x7fffffffULL) return fail(SPARC_E_SHAPE, "force tables too large");
            F.box0 = (int)boff.size();
            F.chi0 = (long long)fun.size();
            const int nb = F.ext[0] * F.ext[1] * F.ext[2];
            for (int i = 0; i < F.ext[0]; ++i)
                for (int j = 0; j < F.ext[1]; ++j)
                    for (int k = 0; k < F.ext[2]; ++k)
                        boff.push_back(((F.lo[0] + i) * op->n[1] + (F.lo[1] + j)) * op->n[2] + (F.lo[2] + k));
            fun.resize(fun.size() + (size_t)nb * A.nproj);
            double *out = fun.data() + F.chi0;
            for (int p = 0; p < A.nproj; ++p) {
                int t = 0;
                for (int i = 0; i < F.ext[0]; ++i)
                    for (int j = 0; j < F.ext[1]; ++j)
                        for (int k = 0; k < F.ext[2]; ++k, ++t) {
                            const int y[3] = {F.lo[0] + i, F.lo[1] + j, F.lo[2] + k};
                            double v;
                            if (r == 0) {
                                v = chi_at(p, y);
                            } else {
                                // -grad_d chi = sum_q w_q (chi(y - q e_d) - chi(y + q e_d))
                                v = 0.0;
                                for (int q = 1; q <= R; ++q) {
                                    int zm[3] = {y[0], y[1], y[2]}, zp[3] = {y[0], y[1], y[2]};
                                    zm[d] -= q;
                                    zp[d] += q;
                                    v += w[q] * (chi_at(p, zm) - chi_at(p, zp));
                                }
                            }
                            out[(size_t)p * nb + t] = v;
                        }
            }
            rec.push_back(F);
        }
    }
    std::vector<double> gam(op->gamma.begin(), op->gamma.end());
    if (hipMalloc(&op->d_fatoms, rec.size() * sizeof(AtomDev)) != hipSuccess ||
        hipMalloc(&op->d_fbox_off, boff.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&op->d_ffun, fun.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&op->d_fgamma, gam.size() * sizeof(double)) != hipSuccess) {
        for (void **p : {(void **)&op->d_fatoms, (void **)&op->d_fbox_off, (void **)&op->d_ffun,
                         (void **)&op->d_fgamma}) {
            (void)hipFree(*p);
            *p = nullptr;
        }
        return fail(SPARC_E_NOMEM, "allocation of the force tables failed");
    }
    SPARC_HIP(hipMemcpy(op->d_fatoms, rec.data(), rec.size() * sizeof(AtomDev), hipMemcpyHostToDevice));
    SPARC_HIP(hipMemcpy(op->d_fbox_off, boff.data(), boff.size() * sizeof(int), hipMemcpyHostToDevice));
    SPARC_HIP(hipMemcpy(op->d_ffun, fun.data(), fun.size() * sizeof(double), hipMemcpyHostToDevice));
    SPARC_HIP(hipMemcpy(op->d_fgamma, gam.data(), gam.size() * sizeof(double), hipMemcpyHostToDevice));
    op->force_ready = true;
    return SPARC_OK;
}

template <typename TI>
__global__ void __launch_bounds__(256) force_gather_kernel(const GatherArgs<double, TI> g)
{
    __shared__ double tile[4][16][16];
    gather_item<double, TI>(g, blockIdx.x, blockIdx.y, blockIdx.z, tile, threadIdx.x);
}

// one workgroup per atom: f[3J + d] = scale * sum_n occ[n] sum_p gamma_p S_0p(n) S_dp(n),
// S_rp(n) the record-r contraction of projector p with orbital n (split
// partials summed in split order); orbitals are dealt n = t + 256 i to thread
// t, and the per-thread sums meet in a fixed butterfly and wave order
__global__ void __launch_bounds__(256) force_finish_kernel(const double *__restrict__ part, int nrec_proj, int ns,
                                                           const AtomDev *__restrict__ atoms,
                                                           const double *__restrict__ gamma,
                                                           const double *__restrict__ occ, double scale,
                                                           double *__restrict__ force)
{
    const AtomDev A = atoms[blockIdx.x];
    const long long split = (long long)nrec_proj * ns;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int n = threadIdx.x; n < ns; n += 256) {
        const double g = occ[n];
        double s3[3] = {0.0, 0.0, 0.0};
        for (int p = 0; p < A.nproj; ++p) {
            double S[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long base = (long long)(4 * A.proj0 + r * A.nproj + p) * ns + n;
                double v = 0.0;
                for (int ks = 0; ks < kGatherSplit; ++ks) v += part[ks * split + base];
                S[r] = v;
            }
            const double gy = gamma[A.proj0 + p] * S[0];
#pragma unroll
            for (int d = 0; d < 3; ++d) s3[d] += gy * S[1 + d];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[d] += g * s3[d];
    }
    __shared__ double red[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double v = acc[d];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0) red[d][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int d = threadIdx.x;
        force[3 * blockIdx.x + d] = scale * ((red[d][0] + red[d][1]) + (red[d][2] + red[d][3]));
    }
}

size_t force_part_bytes(const sparc_op *op, int ns)
{
    return (size_t)kGatherSplit * 4 * op->nproj_total * ns * sizeof(double);
}

}  // namespace
}  // namespace sparc

using namespace sparc;

extern "C" size_t sparc_force_workspace_bytes(const sparc_op *op, int32_t ns)
{
    if (!op || ns < 1) return 0;
    return std::max<size_t>(force_part_bytes(op, ns), 256);
}

extern "C" int sparc_nonlocal_force(const sparc_op *op, int32_t dtype, const void *psi, int64_t ld, int32_t ns,
                                    const double *occ, double *force, void *ws, size_t ws_bytes, void *stream)
{
    if (!op || !psi || !occ || (op->natoms > 0 && !force) || (dtype != SPARC_F64 && dtype != SPARC_F32))
        return fail(SPARC_E_ARG, "bad arguments");
    if (ns < 1 || ld < op->nd) return fail(SPARC_E_SHAPE, "ns < 1 or ld < N_d");
    if ((ns + 15) / 16 > 65535) return fail(SPARC_E_SHAPE, "too many columns for one launch");
    if (op->natoms == 0) return SPARC_OK;
    const size_t need = force_part_bytes(op, ns);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace missing or too small");
    const size_t es = elem_size(dtype);
    const char *p0 = (const char *)psi, *p1 = p0 + ((size_t)(ns - 1) * ld + op->nd) * es;
    const char *w0 = (const char *)ws, *w1 = w0 + need;
    const char *f0 = (const char *)force, *f1 = f0 + (size_t)op->natoms * 3 * sizeof(double);
    if ((w0 < p1 && p0 < w1) || (f0 < p1 && p0 < f1) || (f0 < w1 && w0 < f1))
        return fail(SPARC_E_ALIAS, "psi, the workspace and the forces overlap");
    {
        std::lock_guard<std::mutex> lk(op->force_mu);
        if (!op->force_ready) {
            int st = build_force_tables(op);
            if (st) return st;
        }
    }
    TraceRange trace("sparc_nonlocal_force");
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid(4 * op->natoms, (ns + 15) / 16, kGatherSplit);
    const double h3 = op->h * op->h * op->h;
    ProfScope prof(5, s);
    if (dtype == SPARC_F64) {
        GatherArgs<double, double> a{(const double *)psi, ld, ns, 4 * op->nproj_total, op->d_fatoms, op->d_fbox_off,
                                     op->d_ffun, (double *)ws};
        hipLaunchKernelGGL(force_gather_kernel<double>, grid, dim3(256), 0, s, a);
    } else {
        GatherArgs<double, float> a{(const float *)psi, ld, ns, 4 * op->nproj_total, op->d_fatoms, op->d_fbox_off,
                                    op->d_ffun, (double *)ws};
        hipLaunchKernelGGL(force_gather_kernel<float>, grid, dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(force_finish_kernel, dim3(op->natoms), dim3(256), 0, s, (const double *)ws,
                       4 * op->nproj_total, ns, op->d_atoms, op->d_fgamma, occ, -4.0 * h3 * h3, force);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}
