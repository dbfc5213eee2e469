// Device side of the fused stencil / local-potential / recurrence step (see
// stencil.hip for the design); shared by the standalone launch and the
// batched persistent kernel.
#pragma once

#include "internal.hpp"

namespace sparc {

// TI: storage type of Y_k (FP32 blocks may feed an FP64 application of H)
template <typename T, typename TI = T>
struct StepArgs {
    const TI *yk;
    const T *yprev;
    T *out;
    const T *veff;
    long long ldk, ldp, ldo;
    int n1, n2, n3;
    int tiles_y, tiles_z, nchunks, chunk_x;
    int nblocks;
    int remap;         // 1: spread consecutive block indices over the XCDs' patch ranges
    T *dot;            // DOT launches: per-workgroup sum of yk (H_loc yk) over its points
    T c0;              // centre coefficient of -1/2 lap_h: -3 w_0
    T cp[kMaxRadius];  // -1/2 w_p, p = 1..kMaxRadius (zero beyond the op's radius)
    T alpha, beta, shift;
};

// Global accesses are raw buffer loads and stores through one descriptor per
// plane: the plane's base address and byte size (zero for a plane outside
// the grid), with 32-bit in-plane byte offsets kept in registers.  A point
// outside the grid carries the offset kOutside, which the descriptor's range
// check turns into a load of zero or a dropped store, so neither the bounds
// selects nor 64-bit address arithmetic are spent per access.  A plane
// stays below 2 GiB (checked when the op is built), so kOutside is always
// out of range.
constexpr unsigned kOutside = 0x80000000u;
constexpr int kBufWord3 = 0x00020000;  // raw (untyped) buffer, 32-bit data format
constexpr int kNonTemporal = 2;        // cache-policy bit: non-temporal

template <typename E>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const E *col, int t, int n1, long long P)
{
    const bool in = t >= 0 && t < n1;
    const E *base = col + (in ? (long long)t * P : 0LL);
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, in ? (int)(P * (long long)sizeof(E)) : 0, kBufWord3);
}

template <typename E, int AUX>
__device__ __forceinline__ E buf_load(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(E) == 4)
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
    else
        return __builtin_bit_cast(E, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}

template <typename E, int AUX>
__device__ __forceinline__ void buf_store(E v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(E) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, AUX);
    } else {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, AUX);
    }
}

// STREAM: Y_{k-1} and the output bypass the caches (non-temporal accesses)
// DOT: each thread also accumulates yk(x) * out(x) over its points (dacc)
template <typename T, int TZ, int RY, int NT, bool PREV, bool STREAM = false, typename TI = T, bool DOT = false>
struct StepKernel {
    static constexpr int R = kMaxRadius;
    static constexpr int QL = 2 * R + 1;     // queue length: planes x-R .. x+R
    static constexpr int NYG = NT / TZ;
    static constexpr int TY = NYG * RY;
    static constexpr int SZ = TZ + 2 * R;
    static constexpr int SY = TY + 2 * R;
    static constexpr int NHALO = 2 * R * TZ + 2 * R * TY;
    static constexpr int NH = (NHALO + NT - 1) / NT;

    // values loaded for one plane t: its halo, the queue heads (plane t+R),
    // V_eff and yprev at the thread's own points
    struct Stage {
        T h[NH];
        T qh[RY];
        T v[RY];
        T p[RY];
    };

    const StepArgs<T, TI> &a;
    const TI *yk;
    const T *yp;
    T *out;
    long long P;
    int lz, lyg, xs, xe;
    unsigned pofs_i[RY];  // in-plane byte offsets of the own points in yk (TI), or kOutside
    unsigned pofs_t[RY];  // the same in the T arrays (V_eff, yprev, out)
    bool pok[RY];
    unsigned hofs[NH];    // in-plane byte offsets of the halo values in yk, or kOutside
    int hl[NH];
    T q[RY][QL];
    T dacc = T(0);

    __device__ StepKernel(const StepArgs<T, TI> &args) : a(args) {}

    __device__ __forceinline__ void load_stage(Stage &s, int t) const
    {
        const auto rk = plane_rsrc(yk, t, a.n1, P);
#pragma unroll
        for (int i = 0; i < NH; ++i) s.h[i] = (T)buf_load<TI, 0>(rk, hofs[i]);
        const auto rh = plane_rsrc(yk, t + R, a.n1, P);
#pragma unroll
        for (int r = 0; r < RY; ++r) s.qh[r] = (T)buf_load<TI, 0>(rh, pofs_i[r]);
        const auto rv = plane_rsrc(a.veff, t, a.n1, P);
#pragma unroll
        for (int r = 0; r < RY; ++r) s.v[r] = buf_load<T, 0>(rv, pofs_t[r]);
        if constexpr (PREV) {
            // read once: streamed past the caches when the block is large
            const auto rp = plane_rsrc(yp, t, a.n1, P);
#pragma unroll
            for (int r = 0; r < RY; ++r) s.p[r] = buf_load<T, STREAM ? kNonTemporal : 0>(rp, pofs_t[r]);
        }
    }

    // plane x, stage / LDS buffer S; the queue holds planes x-R .. x+R
    // queue slot of logical position d (planes x-R .. x+R) at rotation Q
    template <int Q>
    static constexpr int slot(int d) { return (Q + d) % QL; }

    template <int S, int Q>
    __device__ __forceinline__ void plane(int x, Stage (&st)[2], T (*lds)[SY * SZ])
    {
        Stage &s = st[S];
        T *L = lds[S];
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][slot<Q>(2 * R)] = s.qh[r];
        // publish the centre plane and its halo
#pragma unroll
        for (int r = 0; r < RY; ++r) L[(R + lyg * RY + r) * SZ + R + lz] = q[r][slot<Q>(R)];
#pragma unroll
        for (int i = 0; i < NH; ++i)
            if (hl[i] >= 0) L[hl[i]] = s.h[i];
        __syncthreads();

        T vcur[RY], pcur[RY];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            vcur[r] = s.v[r];
            pcur[r] = PREV ? s.p[r] : T(0);
        }
        // request plane x+2 into the stage just consumed
        load_stage(s, x + 2);

        const auto ro = plane_rsrc((const T *)out, x, a.n1, P);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int li = (R + lyg * RY + r) * SZ + R + lz;
            const T c = q[r][slot<Q>(R)];
            T acc = a.c0 * c;
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                const T ym = (r - p >= 0) ? q[r - p][slot<Q>(R)] : L[li - p * SZ];
                const T ypl = (r + p < RY) ? q[r + p][slot<Q>(R)] : L[li + p * SZ];
                const T six = (q[r][slot<Q>(R - p)] + q[r][slot<Q>(R + p)]) + (ym + ypl) + (L[li - p] + L[li + p]);
                acc += a.cp[p - 1] * six;
            }
            acc += (vcur[r] - a.shift) * c;
            T res = a.alpha * acc;
            if constexpr (PREV) res -= a.beta * pcur[r];
            if constexpr (DOT)
                if (pok[r]) dacc += c * res;
            // written once; points outside the grid are dropped by the range check
            buf_store<T, STREAM ? kNonTemporal : 0>(res, ro, pofs_t[r]);
        }
    }

    // planes x0 .. x0+2*QL-1 (stop at xe): the stage parity and the queue
    // rotation are compile-time per plane, so the queue never moves
    template <int U>
    __device__ __forceinline__ void run_block(int x0, int xe, Stage (&st)[2], T (*lds)[SY * SZ])
    {
        if constexpr (U < 2 * QL) {
            if (x0 + U >= xe) return;
            plane<U % 2, U % QL>(x0 + U, st, lds);
            run_block<U + 1>(x0, xe, st, lds);
        }
    }

    static constexpr size_t kLdsBytes = sizeof(T) * 2 * SY * SZ;

    // b: workgroup index within the launch (or work item within a batch)
    __device__ __forceinline__ void run(int b, T (*lds)[SY * SZ])
    {
        // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
        // contiguous range of patches so that neighbours share its L2.
        const int nb = a.nblocks;
        const int xcd = b & 7;
        int t = a.remap ? xcd * (nb >> 3) + min(xcd, nb & 7) + (b >> 3) : b;
        const int tzi = t % a.tiles_z;
        t /= a.tiles_z;
        const int tyi = t % a.tiles_y;
        t /= a.tiles_y;
        const int chunk = t % a.nchunks;
        const int col = t / a.nchunks;

        const int tid = threadIdx.x;
        lz = tid % TZ;
        lyg = tid / TZ;
        const int n2 = a.n2, n3 = a.n3;
        const int z0 = tzi * TZ, y0 = tyi * TY;
        const int z = z0 + lz;
        P = (long long)n2 * n3;
        yk = a.yk + (size_t)col * a.ldk;
        yp = PREV ? a.yprev + (size_t)col * a.ldp : nullptr;
        out = a.out + (size_t)col * a.ldo;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = y0 + lyg * RY + r;
            pok[r] = (z < n3) && (y < n2);
            const unsigned e = (unsigned)(y * n3 + z);
            pofs_i[r] = pok[r] ? e * (unsigned)sizeof(TI) : kOutside;
            pofs_t[r] = pok[r] ? e * (unsigned)sizeof(T) : kOutside;
        }
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const int e = tid + i * NT;
            int ly = -1, lzz = -1;
            if (e < 2 * R * TZ) {
                const int hy = e / TZ, hz = e % TZ;
                ly = hy < R ? hy : hy + TY;
                lzz = R + hz;
            } else if (e < NHALO) {
                const int e2 = e - 2 * R * TZ;
                const int zr = e2 / (2 * R), hz = e2 % (2 * R);
                ly = R + zr;
                lzz = hz < R ? hz : hz + TZ;
            }
            hl[i] = (ly >= 0) ? ly * SZ + lzz : -1;
            const int gy = y0 - R + ly, gz = z0 - R + lzz;
            const bool hok = ly >= 0 && gy >= 0 && gy < n2 && gz >= 0 && gz < n3;
            hofs[i] = hok ? (unsigned)(gy * n3 + gz) * (unsigned)sizeof(TI) : kOutside;
        }
        xs = chunk * a.chunk_x;
        xe = min(a.n1, xs + a.chunk_x);

        // queue: planes xs-R .. xs+R-1 (heads are filled from the stages)
#pragma unroll
        for (int d = 0; d < 2 * R; ++d) {
            const auto rq = plane_rsrc(yk, xs - R + d, a.n1, P);
#pragma unroll
            for (int r = 0; r < RY; ++r) q[r][d] = (T)buf_load<TI, 0>(rq, pofs_i[r]);
        }
        Stage st[2];
        load_stage(st[0], xs);
        load_stage(st[1], xs + 1);
        for (int x0 = xs; x0 < xe; x0 += 2 * QL) run_block<0>(x0, xe, st, lds);
    }
};

}  // namespace sparc
