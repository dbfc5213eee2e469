// Launch code of the fused step kernel, instantiated per storage type in
// step_f32.hip, step_f64.hip and step_mixed.hip (separate translation units,
// so the many kernel variants compile in parallel).
#pragma once

#include <type_traits>

#include "nonlocal_kernel.hpp"
#include "step_kernel.hpp"

namespace sparc {

// fixed-order workgroup sum of the per-thread products of a DOT launch
template <typename T, int NT>
__device__ __forceinline__ void store_dot(T v, T *dot, int b)
{
    __shared__ T red[NT / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = red[0];
        for (int i = 1; i < NT / 64; ++i) t += red[i];
        dot[b] = t;
    }
}

template <typename T, int TZ, int RY, int NT, bool PREV, bool STREAM, typename TI, bool DOT = false>
__global__ void __launch_bounds__(NT) step_kernel(const StepArgs<T, TI> a)
{
    using K = StepKernel<T, TZ, RY, NT, PREV, STREAM, TI, DOT>;
    __shared__ T lds[2][K::SY * K::SZ];
    K k(a);
    k.run(blockIdx.x, lds);
    if constexpr (DOT) store_dot<T, NT>(k.dacc, a.dot, blockIdx.x);
}

// One filter step with the projector gather of the same Y_k in one launch:
// the first a.nblocks workgroups run the step (its XCD-aware index remap sees
// the hardware round-robin unchanged), the last ngb run NT/256 gather items
// each, 256 threads apiece (item = atom + natoms (column group + ncb split),
// the standalone gather's grid order; a group past the last item only joins
// the item's barrier), filling CUs as the step's workgroups drain.
template <typename T, int TZ, int RY, int NT, bool PREV, bool STREAM>
__global__ void __launch_bounds__(NT) step_gather_kernel(const StepArgs<T, T> a, const GatherArgs<T, T> g,
                                                         int natoms, int ncb, int nitems)
{
    if ((int)blockIdx.x >= a.nblocks) {
        constexpr int G = NT / 256;
        __shared__ T tile[G][4][16][16];
        const int sub = threadIdx.x >> 8;
        const int item = ((int)blockIdx.x - a.nblocks) * G + sub;
        if (item < nitems)
            gather_item<T, T>(g, item % natoms, (item / natoms) % ncb, item / (natoms * ncb), tile[sub],
                              threadIdx.x & 255);
        else
            __syncthreads();
        return;
    }
    using K = StepKernel<T, TZ, RY, NT, PREV, STREAM, T>;
    __shared__ T lds[2][K::SY * K::SZ];
    K k(a);
    k.run(blockIdx.x, lds);
}

// gather launch data for launch_typed (ngb == 0: plain step)
template <typename T>
struct GatherPlan {
    GatherArgs<T, T> g;
    int natoms = 0, ncb = 0, nitems = 0, ngb = 0;
};

template <typename T, int TZ, int RY, int NT, typename TI>
inline int launch_typed(const StepArgs<T, TI> &a, bool prev, bool strm, hipStream_t stream,
                        const GatherPlan<T> *gp = nullptr)
{
    if constexpr (std::is_same<T, TI>::value) {
        if (gp && gp->ngb > 0) {
            const dim3 grid(a.nblocks + gp->ngb), blk(NT);
#define SPARC_SG(P, S)                                                                                           \
    hipLaunchKernelGGL((step_gather_kernel<T, TZ, RY, NT, P, S>), grid, blk, 0, stream, a, gp->g, gp->natoms, \
                       gp->ncb, gp->nitems)
            if (prev && strm)
                SPARC_SG(true, true);
            else if (prev)
                SPARC_SG(true, false);
            else if (strm)
                SPARC_SG(false, true);
            else
                SPARC_SG(false, false);
#undef SPARC_SG
            SPARC_HIP(hipGetLastError());
            return SPARC_OK;
        }
    }
    const dim3 g(a.nblocks), b(NT);
    if constexpr (std::is_same<T, TI>::value) {
        if (prev && strm)
            hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, true, true, TI>), g, b, 0, stream, a);
        else if (prev)
            hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, true, false, TI>), g, b, 0, stream, a);
    }
    if (!prev) {
        if (strm)
            hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, false, true, TI>), g, b, 0, stream, a);
        else
            hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, false, false, TI>), g, b, 0, stream, a);
    }
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

template <typename T, typename TI = T>
int launch_step_t(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                         void *out, int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L,
                         hipStream_t stream, const T *veff, void *part = nullptr, const T *chi = nullptr)
{
    const TileShape &s = kShapes[L.shape];
    StepArgs<T, TI> a;
    a.yk = (const TI *)yk;
    a.yprev = (const T *)yprev;
    a.out = (T *)out;
    a.veff = veff;
    a.ldk = ldk;
    a.ldp = ldp;
    a.ldo = ldo;
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.n3 = op->n[2];
    a.tiles_y = (op->n[1] + s.ty() - 1) / s.ty();
    a.tiles_z = (op->n[2] + s.tz - 1) / s.tz;
    a.chunk_x = L.chunk_x;
    a.nchunks = (op->n[0] + L.chunk_x - 1) / L.chunk_x;
    const bool prev = c.has_prev && yprev != nullptr;
    const long long nb = (long long)ns * a.nchunks * a.tiles_y * a.tiles_z;
    if (nb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
    a.nblocks = (int)nb;
    a.remap = 1;
    a.dot = nullptr;
    a.c0 = (T)(-3.0 * op->w[0]);
    for (int p = 1; p <= kMaxRadius; ++p) a.cp[p - 1] = (T)(-0.5 * op->w[p]);
    a.alpha = (T)c.alpha;
    a.beta = (T)c.beta;
    a.shift = (T)c.shift;
    // blocks the last-level cache cannot keep between steps are streamed
    const bool strm = (double)op->nd * ns * (2 * sizeof(T) + sizeof(TI)) > kStreamBytes;
    GatherPlan<T> gp;
    if (part && op->natoms > 0) {
        if ((long long)(ns + 15) / 16 > 65535) return fail(SPARC_E_SHAPE, "too many columns for one gather launch");
        gp.g.Y = (const T *)yk;
        gp.g.ldy = ldk;
        gp.g.ns = ns;
        gp.g.nproj_total = op->nproj_total;
        gp.g.atoms = op->d_atoms;
        gp.g.box_off = op->d_box_off;
        gp.g.chi = chi;
        gp.g.part = (T *)part;
        gp.natoms = op->natoms;
        gp.ncb = (ns + 15) / 16;
        gp.nitems = op->natoms * gp.ncb * kGatherSplit;
        const int per = kShapes[L.shape].nt / 256;
        gp.ngb = (gp.nitems + per - 1) / per;
        if ((long long)a.nblocks + gp.ngb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
    }
    ProfScope prof(prev ? 0 : 3, stream);
    switch (L.shape) {
        case 0: return launch_typed<T, 32, 2, 256, TI>(a, prev, strm, stream, &gp);
        case 1: return launch_typed<T, 32, 2, 512, TI>(a, prev, strm, stream, &gp);
    }
    return fail(SPARC_E_ARG, "unknown tile shape");
}


}  // namespace sparc
