// Launch code of the vector step kernels, instantiated per storage type and
// patch height in fstep_<type>_ty<TY>.hip (separate translation units, so the
// kernel variants compile in parallel).
#pragma once

#include "fstep_kernel.hpp"
#include "nonlocal_kernel.hpp"

namespace sparc {

// One launch: the first a.nblocks workgroups run the vector step, the last
// ngb run NT/256 projector-gather items of yk each (item = atom + natoms *
// (column block + ncb * split), 256 threads apiece; a group past the last
// item only joins the item's barrier), filling CUs as the step drains.
template <typename T, int TY, int TZ, bool PREV, bool STREAM, bool TAIL, int B>
__global__ void __launch_bounds__((TZ / VecTraits<T>::N) * TY)
    fstep_kernel(const FStepArgs<T> a, const GatherArgs<T, T> g, int natoms, int ncb, int nitems)
{
    constexpr int NT = (TZ / VecTraits<T>::N) * TY;
    if constexpr (TAIL) {
        if ((int)blockIdx.x >= a.nblocks) {
            // G whole groups of 256 threads; threads past them (NT not a
            // multiple of 256) only join the items' barrier
            constexpr int G = NT / 256;
            __shared__ T tile[G][4][16][16];
            const int sub = threadIdx.x >> 8;
            const int item = ((int)blockIdx.x - a.nblocks) * G + sub;
            if (sub < G && item < nitems)
                gather_item<T, T>(g, item % natoms, (item / natoms) % ncb, item / (natoms * ncb), tile[sub],
                                  threadIdx.x & 255);
            else
                __syncthreads();
            return;
        }
    }
    using K = FStep<T, TY, PREV, STREAM, B, TZ>;
    __shared__ __align__(16) typename K::Shared sh;
    K k(a);
    k.run(blockIdx.x, sh);
}

template <typename T, int TY, int TZ, int B>
int fstep_dispatch_b(const FStepArgs<T> &a, const GatherArgs<T, T> &g, int natoms, int ncb, int nitems, int ngb,
                     bool prev, bool strm, hipStream_t s)
{
    constexpr int NT = (TZ / VecTraits<T>::N) * TY;
    const dim3 grid(a.nblocks + ngb), b(NT);
#define SPARC_FS(P, S, G) \
    hipLaunchKernelGGL((fstep_kernel<T, TY, TZ, P, S, G, B>), grid, b, 0, s, a, g, natoms, ncb, nitems)
    // patches of fewer than 256 threads cannot host a gather item
    if (ngb > 0 && NT < 256) return fail(SPARC_E_ARG, "gather tail needs 256-thread workgroups");
    if constexpr (NT < 256) {
        if (prev && strm)
            SPARC_FS(true, true, false);
        else if (prev)
            SPARC_FS(true, false, false);
        else if (strm)
            SPARC_FS(false, true, false);
        else
            SPARC_FS(false, false, false);
    } else if (ngb > 0) {
        if (prev && strm)
            SPARC_FS(true, true, true);
        else if (prev)
            SPARC_FS(true, false, true);
        else if (strm)
            SPARC_FS(false, true, true);
        else
            SPARC_FS(false, false, true);
    } else {
        if (prev && strm)
            SPARC_FS(true, true, false);
        else if (prev)
            SPARC_FS(true, false, false);
        else if (strm)
            SPARC_FS(false, true, false);
        else
            SPARC_FS(false, false, false);
    }
#undef SPARC_FS
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

// cblk: columns per workgroup (1 or 2; 2 only for patches of at most 512
// threads, whose waves can hold two register queues)
template <typename T, int TY, int TZ = kFTZ>
int fstep_dispatch(const FStepArgs<T> &a, const GatherArgs<T, T> &g, int natoms, int ncb, int nitems, int ngb,
                   bool prev, bool strm, int cblk, hipStream_t s)
{
    constexpr int NT = (TZ / VecTraits<T>::N) * TY;
    if constexpr (NT <= 512) {
        if (cblk == 2) return fstep_dispatch_b<T, TY, TZ, 2>(a, g, natoms, ncb, nitems, ngb, prev, strm, s);
    } else {
        if (cblk == 2) return fail(SPARC_E_ARG, "two columns per workgroup need patches of at most 512 threads");
    }
    return fstep_dispatch_b<T, TY, TZ, 1>(a, g, natoms, ncb, nitems, ngb, prev, strm, s);
}

// per (type, patch height) launches, one translation unit each
#define SPARC_FSTEP_DECL(name, T) \
    int name(const FStepArgs<T> &, const GatherArgs<T, T> &, int, int, int, int, bool, bool, int, hipStream_t);
SPARC_FSTEP_DECL(fstep_f32_ty16, float)
SPARC_FSTEP_DECL(fstep_f32_ty32, float)
SPARC_FSTEP_DECL(fstep_f32_ty64, float)
SPARC_FSTEP_DECL(fstep_f64_ty8, double)
SPARC_FSTEP_DECL(fstep_f64_ty16, double)
SPARC_FSTEP_DECL(fstep_f64_ty32, double)
SPARC_FSTEP_DECL(fstep_f32_ty16_tz64, float)
SPARC_FSTEP_DECL(fstep_f32_ty32_tz64, float)
SPARC_FSTEP_DECL(fstep_f64_ty8_tz64, double)
SPARC_FSTEP_DECL(fstep_f64_ty16_tz64, double)
SPARC_FSTEP_DECL(fstep_f32_ty24_tz160, float)
SPARC_FSTEP_DECL(fstep_f32_ty32_tz80, float)
SPARC_FSTEP_DECL(fstep_f64_ty24_tz64, double)
#undef SPARC_FSTEP_DECL

}  // namespace sparc
