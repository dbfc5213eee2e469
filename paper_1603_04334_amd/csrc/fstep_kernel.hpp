// Device side of the vector step: stencil, local potential and Chebyshev
// recurrence in one pass over an orbital block with 16-byte accesses (see
// fstep.hip for the design).  Shared by the standalone launches and the
// batched persistent kernel.
#pragma once

#include "step_kernel.hpp"

namespace sparc {

constexpr int kFTZ = 32;  // default patch extent along z (grid points)

template <typename T>
struct VecTraits;
template <>
struct VecTraits<float> {
    static constexpr int N = 4;
    typedef float V __attribute__((ext_vector_type(4)));
};
template <>
struct VecTraits<double> {
    static constexpr int N = 2;
    typedef double V __attribute__((ext_vector_type(2)));
};
typedef unsigned U4 __attribute__((ext_vector_type(4)));

// 16-byte raw buffer accesses (see plane_rsrc for the range check)
template <typename T, int AUX>
__device__ __forceinline__ typename VecTraits<T>::V vload(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(typename VecTraits<T>::V, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX));
}

template <typename T, int AUX>
__device__ __forceinline__ void vstore(typename VecTraits<T>::V v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, off, 0, AUX);
}

template <typename T>
struct FStepArgs {
    const T *yk;
    const T *yprev;
    T *out;
    const T *veff;
    long long ldk, ldp, ldo;
    int n1, n2, n3;
    int tiles_y, tiles_z, nchunks, chunk_x;
    int nblocks;
    int remap;
    int ns, cgroup;    // columns; consecutive workgroups take cgroup columns of one patch
    T c0;              // -3 w_0
    T cp[kMaxRadius];  // -1/2 w_p
    T alpha, beta, shift;
};

// B: columns per workgroup.  With B = 2 the two columns of one patch share
// the V_eff loads, the halo offsets and the plane loop (orbital blocking).
template <typename T, int TY, bool PREV, bool STREAM, int B = 1, int TZ = kFTZ>
struct FStep {
    static constexpr int R = kMaxRadius;
    static constexpr int VZ = VecTraits<T>::N;
    using V = typename VecTraits<T>::V;
    static constexpr int LPR = TZ / VZ;  // lanes per row of the patch
    static constexpr int NT = LPR * TY;
    static constexpr int NW = NT / 64;
    static constexpr int PADZ = (R + VZ - 1) / VZ * VZ;  // z halo per side, whole units
    static constexpr int ZU = PADZ / VZ;
    static constexpr int SZ = TZ + 2 * PADZ;
    static constexpr int SY = TY + 2 * R;
    static constexpr int QL = 2 * R + 1;
    static constexpr int NHALO = 2 * R * LPR + TY * 2 * ZU;  // halo units per plane
    static constexpr int NH = (NHALO + NT - 1) / NT;
    static constexpr int WU = 2 * ZU + 1;  // units of a lane's z window
    static_assert(NT % 64 == 0, "whole waves");
    // the z window reads an edge unit whole or one aligned half of it: the
    // used range must start and end on half-unit boundaries
    static_assert(VZ == 1 || ((PADZ - R) % (VZ / 2) == 0 && (PADZ + VZ + R) % (VZ / 2) == 0),
                  "z window edges must fall on half units");
    static_assert(B == 1 || B == 2, "one or two columns per workgroup");

    struct Shared {
        T plane[2][B][SY * SZ];
    };

    const FStepArgs<T> &a;
    const T *yk[B];
    const T *yp[B];
    T *out[B];
    long long P;
    int col, chunk, xs, xe, ly, lz, y, zg;
    unsigned pofs;      // in-plane byte offset of the lane's unit, or kOutside
    unsigned sofs[B];   // store offset per column (kOutside for a column past the block)
    unsigned hofs[NH];  // halo units: in-plane byte offsets, or kOutside
    int hl[NH];         // halo units: LDS element index, or -1
    V q[B][QL];  // per column, the lane's unit at planes x-R .. x+R (one vector per plane)
    // the two load stages (values for one plane: its halo, the queue head at
    // plane t+R, V_eff and yprev at the lane's unit), one named member per
    // stage and only whole-vector accesses at constant indices, so that they
    // stay in registers
    struct Stage {
        V h[B][NH];
        V qh[B], p[B];
        V v;
    };
    Stage st0, st1;
    template <int S>
    __device__ __forceinline__ Stage &stage()
    {
        if constexpr (S == 0)
            return st0;
        else
            return st1;
    }

    __device__ FStep(const FStepArgs<T> &args) : a(args) {}

    template <int Q>
    static constexpr int slot(int d) { return (Q + d) % QL; }

    template <int S>
    __device__ __forceinline__ void load_stage(int t)
    {
        Stage &s = stage<S>();
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const auto rk = plane_rsrc(yk[b], t, a.n1, P);
#pragma unroll
            for (int i = 0; i < NH; ++i) s.h[b][i] = vload<T, 0>(rk, hofs[i]);
            s.qh[b] = vload<T, 0>(plane_rsrc(yk[b], t + R, a.n1, P), pofs);
        }
        s.v = vload<T, 0>(plane_rsrc(a.veff, t, a.n1, P), pofs);
        if constexpr (PREV) {
#pragma unroll
            for (int b = 0; b < B; ++b) s.p[b] = vload<T, STREAM ? kNonTemporal : 0>(plane_rsrc(yp[b], t, a.n1, P), pofs);
        }
    }

    template <int S, int Q>
    __device__ __forceinline__ void plane(int x, Shared &sh)
    {
        // publish the centre plane and its halo of every column
#pragma unroll
        for (int b = 0; b < B; ++b) {
            T *L = sh.plane[S][b];
            q[b][slot<Q>(2 * R)] = stage<S>().qh[b];
            *(V *)&L[(R + ly) * SZ + PADZ + VZ * lz] = q[b][slot<Q>(R)];
#pragma unroll
            for (int i = 0; i < NH; ++i)
                if (hl[i] >= 0) *(V *)&L[hl[i]] = stage<S>().h[b][i];
        }
        __syncthreads();

        const V vv = stage<S>().v;
        V pv[B];
#pragma unroll
        for (int b = 0; b < B; ++b) pv[b] = PREV ? stage<S>().p[b] : V{};
        // request plane x+2 into the stage just consumed
        load_stage<S>(x + 2);

#pragma unroll
        for (int b = 0; b < B; ++b) {
            const T *L = sh.plane[S][b];
            const V cen = q[b][slot<Q>(R)];
            // z window: PADZ values on each side of the lane's unit.  Only
            // [PADZ - R, PADZ + VZ - 1 + R] is used: the centre unit is the
            // lane's own (registers), an edge unit of which only an aligned
            // half is used reads that half
            T w[WU * VZ];
            const T *row = &L[(R + ly) * SZ + VZ * lz];
            constexpr int WLO = PADZ - R, WHI = PADZ + VZ - 1 + R;
#pragma unroll
            for (int u = 0; u < WU; ++u) {
                const int u0 = u * VZ, u1 = u0 + VZ - 1;
                const int b0 = u0 > WLO ? u0 : WLO, b1 = u1 < WHI ? u1 : WHI;
                if (u == ZU) {
#pragma unroll
                    for (int j = 0; j < VZ; ++j) w[u0 + j] = cen[j];
                } else if (b0 == u0 && b1 == u1) {
                    const V t = *(const V *)&row[u0];
#pragma unroll
                    for (int j = 0; j < VZ; ++j) w[u0 + j] = t[j];
                } else if (b0 <= b1) {
                    constexpr int H = VZ / 2;
                    const int h0 = (b0 - u0) / H * H;  // the aligned half holding b0 .. b1
                    typedef T VH __attribute__((ext_vector_type(VZ / 2)));
                    const VH t = *(const VH *)&row[u0 + h0];
#pragma unroll
                    for (int j = 0; j < H; ++j) w[u0 + h0 + j] = t[j];
                }
            }
            T acc[VZ];
#pragma unroll
            for (int j = 0; j < VZ; ++j) acc[j] = a.c0 * cen[j];
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                const V ym = *(const V *)&L[(R + ly - p) * SZ + PADZ + VZ * lz];
                const V yq = *(const V *)&L[(R + ly + p) * SZ + PADZ + VZ * lz];
#pragma unroll
                for (int j = 0; j < VZ; ++j) {
                    const T six = (q[b][slot<Q>(R - p)][j] + q[b][slot<Q>(R + p)][j]) + (ym[j] + yq[j]) +
                                  (w[PADZ + j - p] + w[PADZ + j + p]);
                    acc[j] += a.cp[p - 1] * six;
                }
            }
#pragma unroll
            for (int j = 0; j < VZ; ++j) acc[j] += (vv[j] - a.shift) * cen[j];

            V rv;
#pragma unroll
            for (int j = 0; j < VZ; ++j) {
                T r = a.alpha * acc[j];
                if constexpr (PREV) r -= a.beta * pv[b][j];
                rv[j] = r;
            }
            // written once; units outside the grid are dropped by the range check
            vstore<T, STREAM ? kNonTemporal : 0>(rv, plane_rsrc((const T *)out[b], x, a.n1, P), sofs[b]);
        }
    }

    template <int U>
    __device__ __forceinline__ void run_block(int x0, int xend, Shared &sh)
    {
        if constexpr (U < 2 * QL) {
            if (x0 + U >= xend) return;
            plane<U % 2, U % QL>(x0 + U, sh);
            run_block<U + 1>(x0, xend, sh);
        }
    }

    // b: workgroup index within the launch (or work item within a batch)
    __device__ __forceinline__ void run(int wg, Shared &sh)
    {
        const int nb = a.nblocks;
        const int xcd = wg & 7;
        int t = a.remap ? xcd * (nb >> 3) + min(xcd, nb & 7) + (wg >> 3) : wg;
        // cgroup consecutive indices are the same patch of consecutive
        // column blocks, so they share the patch's V_eff in L2
        const int cg = t % a.cgroup;
        t /= a.cgroup;
        const int tzi = t % a.tiles_z;
        t /= a.tiles_z;
        const int tyi = t % a.tiles_y;
        t /= a.tiles_y;
        chunk = t % a.nchunks;
        col = ((t / a.nchunks) * a.cgroup + cg) * B;
        if (col >= a.ns) return;  // the padding of the last column group

        const int tid = threadIdx.x;
        lz = tid % LPR;
        ly = tid / LPR;
        const int z0 = tzi * TZ, y0 = tyi * TY;
        y = y0 + ly;
        zg = z0 + VZ * lz;
        P = (long long)a.n2 * a.n3;
        const bool own_ok = (zg < a.n3) && (y < a.n2);
        pofs = own_ok ? (unsigned)(y * a.n3 + zg) * (unsigned)sizeof(T) : kOutside;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            // a column past the block repeats the last one and stores nothing
            const int c = min(col + b, a.ns - 1);
            yk[b] = a.yk + (size_t)c * a.ldk;
            yp[b] = PREV ? a.yprev + (size_t)c * a.ldp : nullptr;
            out[b] = a.out + (size_t)c * a.ldo;
            sofs[b] = col + b < a.ns ? pofs : kOutside;
        }
        xs = chunk * a.chunk_x;
        xe = min(a.n1, xs + a.chunk_x);

        run_planes(tid, z0, y0, sh);
    }

    __device__ __forceinline__ void run_planes(int tid, int z0, int y0, Shared &sh)
    {
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int e = tid + i * NT;
            int lrow = -1, lcol = 0;
            if (e < 2 * R * LPR) {
                const int hy = e / LPR, hu = e % LPR;
                lrow = hy < R ? hy : hy + TY;
                lcol = PADZ + VZ * hu;
            } else if (e < NHALO) {
                const int e2 = e - 2 * R * LPR;
                const int r = e2 / (2 * ZU), hu = e2 % (2 * ZU);
                lrow = R + r;
                lcol = hu < ZU ? VZ * hu : PADZ + TZ + VZ * (hu - ZU);
            }
            hl[i] = lrow >= 0 ? lrow * SZ + lcol : -1;
            const int gy = y0 - R + lrow, gz = z0 - PADZ + lcol;
            const bool hok = lrow >= 0 && gy >= 0 && gy < a.n2 && gz >= 0 && gz < a.n3;
            hofs[i] = hok ? (unsigned)(gy * a.n3 + gz) * (unsigned)sizeof(T) : kOutside;
        }

        // queue: planes xs-R .. xs+R-1 (heads are filled from the stages)
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int d = 0; d < 2 * R; ++d) q[b][d] = vload<T, 0>(plane_rsrc(yk[b], xs - R + d, a.n1, P), pofs);
        load_stage<0>(xs);
        load_stage<1>(xs + 1);
        for (int x0 = xs; x0 < xe; x0 += 2 * QL) run_block<0>(x0, xe, sh);
    }
};

}  // namespace sparc
