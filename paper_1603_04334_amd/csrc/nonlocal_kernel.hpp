// Device side of the nonlocal gather and scatter (see nonlocal.hip for the
// design); shared by the standalone launches and the batched persistent kernel.
#pragma once

#include "internal.hpp"

namespace sparc {

// TI: storage type of Y (FP32 blocks may be projected in FP64)
template <typename T, typename TI = T>
struct GatherArgs {
    const TI *Y;
    long long ldy;
    int ns;
    int nproj_total;
    const AtomDev *atoms;
    const int *box_off;  // grid index of every cube point, per atom from atom.box0
    const T *chi;
    T *part;             // [kGatherSplit][nproj_total][ns] partial projections
};

__device__ inline void mfma_16x16x4(const double a, const double b, double (&acc)[4])
{
    typedef double v4d __attribute__((ext_vector_type(4)));
    v4d c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}

__device__ inline void mfma_16x16x4(const float a, const float b, float (&acc)[4])
{
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f c = {acc[0], acc[1], acc[2], acc[3]};
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    acc[0] = c[0];
    acc[1] = c[1];
    acc[2] = c[2];
    acc[3] = c[3];
}

// accumulator row held by register r of this lane
template <typename T>
__device__ inline int acc_row(int lane, int r)
{
    if constexpr (sizeof(T) == 8)
        return (lane >> 4) + 4 * r;
    else
        return 4 * (lane >> 4) + r;
}

constexpr int kGatherUnroll = 8;  // groups of 4 points per wave per batch

// tid: this thread's index within the 256 threads (4 waves) that run the
// item; the item has one workgroup barrier
template <typename T, typename TI = T>
__device__ __forceinline__ void gather_item(const GatherArgs<T, TI> &g, int atom, int cb, int ks, T (*tile)[16][16],
                                            int tid)
{
    const int c0 = cb * 16;
    const AtomDev A = g.atoms[atom];
    const int nbox = A.ext[0] * A.ext[1] * A.ext[2];
    const int chunk = (nbox + kGatherSplit - 1) / kGatherSplit;
    const int k0 = min(nbox, ks * chunk);
    const int k1 = min(nbox, k0 + chunk);
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int i = lane & 15;
    const int k = lane >> 4;
    const int col = c0 + i;
    const bool col_ok = col < g.ns;
    const bool proj_ok = i < A.nproj;
    const TI *y = g.Y + (long long)(col_ok ? col : 0) * g.ldy;
    const T *ch = g.chi + A.chi0 + (long long)(proj_ok ? i : 0) * nbox;
    const int *boff = g.box_off + A.box0;

    T acc[4] = {T(0), T(0), T(0), T(0)};
    constexpr int BATCH = 4 * kGatherUnroll;
    for (int base = k0 + wave * BATCH; base < k1; base += 4 * BATCH) {
        int off[kGatherUnroll];
        T av[kGatherUnroll], bv[kGatherUnroll];
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const int pt = base + 4 * u + k;
            off[u] = boff[pt < k1 ? pt : k0];
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) {
            const int pt = base + 4 * u + k;
            const bool ok = pt < k1;
            const T yv = (T)y[off[u]];
            const T cv = ch[ok ? pt : k0];
            av[u] = (ok && col_ok) ? yv : T(0);
            bv[u] = (ok && proj_ok) ? cv : T(0);
        }
#pragma unroll
        for (int u = 0; u < kGatherUnroll; ++u) mfma_16x16x4(av[u], bv[u], acc);
    }

#pragma unroll
    for (int r = 0; r < 4; ++r) tile[wave][acc_row<T>(lane, r)][lane & 15] = acc[r];
    __syncthreads();
    const int row = tid >> 4, pj = tid & 15;
    const int cc = c0 + row;
    if (cc < g.ns && pj < A.nproj) {
        const T s = ((tile[0][row][pj] + tile[1][row][pj]) + tile[2][row][pj]) + tile[3][row][pj];
        g.part[((long long)ks * g.nproj_total + A.proj0 + pj) * g.ns + cc] = s;
    }
}

constexpr int kScatterCols = 8;  // columns per scatter item of the batched kernel

template <typename T>
struct ScatterArgs {
    T *out;
    long long ldo;
    int ns;
    int nproj_total;
    const int *blk_pt;     // nblk + 1 node offsets
    const int *blk_at;     // nblk + 1 offsets into blk_atoms
    const int *blk_atoms;  // atoms touched by each block (slot order)
    const int *pts;        // unique grid nodes covered by a cube
    const int *ent_off;    // npts + 1 offsets into ent
    const int4 *ent;       // (chi index of projector 0, cube size, slot, nproj)
    const AtomDev *atoms;
    const T *chi;
    const T *hg;           // h^3 gamma per global projector
    const T *part;         // [kGatherSplit][nproj_total][ns]
    T alpha;
};

// One node block b (at most 256 nodes) and NC columns from cg * NC.  gl: the
// block's table h^3 gamma S, [slot][npm][NC] (npm >= every atom's projector
// count).  The out values of all NC columns are requested before the table
// is built, so their latency overlaps it.  Per node and column the sum runs
// over the node's entries and projectors in table order whatever NC is, so
// every column count gives the same bits.
template <typename T, int NC>
__device__ __forceinline__ void scatter_item(const ScatterArgs<T> &s, int b, int cg, T *gl, int npm)
{
    const int c0 = cg * NC;
    const int a0 = s.blk_at[b];
    const int na = s.blk_at[b + 1] - a0;
    const long long split = (long long)s.nproj_total * s.ns;
    const int pi = s.blk_pt[b] + threadIdx.x;
    const bool own = pi < s.blk_pt[b + 1];
    int gpt = 0, e0 = 0, e1 = 0;
    T cur[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) cur[cc] = T(0);
    if (own) {
        gpt = s.pts[pi];
        e0 = s.ent_off[pi];
        e1 = s.ent_off[pi + 1];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
            if (c0 + cc < s.ns) cur[cc] = s.out[(long long)(c0 + cc) * s.ldo + gpt];
    }
    for (int idx = threadIdx.x; idx < na * npm * NC; idx += 256) {
        const int slot = idx / (npm * NC);
        const int p = (idx / NC) % npm;
        const int cc = idx % NC;
        const AtomDev A = s.atoms[s.blk_atoms[a0 + slot]];
        T v = T(0);
        if (p < A.nproj && c0 + cc < s.ns) {
            const long long pg = A.proj0 + p;
            T sum = T(0);
#pragma unroll
            for (int q = 0; q < kGatherSplit; ++q) sum += s.part[q * split + pg * s.ns + c0 + cc];
            v = s.hg[pg] * sum;
        }
        gl[idx] = v;
    }
    __syncthreads();
    if (!own) return;
    T acc[NC];
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) acc[cc] = T(0);
    for (int e = e0; e < e1; ++e) {
        const int4 en = s.ent[e];
        for (int p = 0; p < en.w; ++p) {
            const T cv = s.chi[en.x + (long long)p * en.y];
            const T *row = gl + (en.z * npm + p) * NC;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) acc[cc] += cv * row[cc];
        }
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc)
        if (c0 + cc < s.ns) s.out[(long long)(c0 + cc) * s.ldo + gpt] = cur[cc] + s.alpha * acc[cc];
}

}  // namespace sparc
