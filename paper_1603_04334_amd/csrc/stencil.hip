// Fused stencil / local-potential / Chebyshev-recurrence kernel for gfx950.
//
// One launch computes, for every node x and every column c of an orbital
// block,
//     out(x,c) = alpha * ( -1/2 lap_h yk + (V_eff(x) - shift) yk )(x,c) - beta * yprev(x,c)
// i.e. the local part of one step of the three-term Chebyshev recurrence of
// Sec. 3.4 (alpha = 2 sigma_{k+1}/e, beta = sigma_k sigma_{k+1}, shift = c),
// of its first step (no yprev) or of a plain application of H (alpha = 1,
// shift = 0).  lap_h is the 2n_o-order stencil of Sec. 3.1 Eq. FD:Laplacian
// with f = 0 off the grid.  The nonlocal term alpha * V_nl yk is added by the
// projector scatter kernel that follows this launch.
//
// Data movement (the kernel is HBM-bound):
//  * A workgroup owns a TY x TZ patch of the (y, z) plane of one column and
//    streams it along x (the slowest axis), so every plane of yk, yprev and
//    out crosses HBM once.
//  * Lanes run along z (contiguous); each thread owns RY consecutive rows of
//    y.  It keeps a queue of the 2R+1 values of its points along x in
//    registers (x-neighbours never touch LDS), and the y-neighbours that fall
//    on its own rows are read from the queue centres as well.
//  * The current plane of the patch plus a cross-shaped halo (R rows in y, R
//    columns in z) is staged in LDS, double-buffered with one barrier per
//    plane; the remaining y- and z-neighbours come from there.  Halo values
//    belong to neighbouring patches and are served from L2 when neighbours
//    run on the same XCD, which the workgroup-index remap arranges.
//  * All global loads are unconditional (out-of-grid addresses are clamped
//    and the value replaced by zero) and are issued two planes ahead, so each
//    wait only covers loads issued one full plane earlier.
//  * yprev is read pointwise and out may alias it: a thread reads yprev(x)
//    one plane before it writes out(x), and no other thread touches x.
#include "internal.hpp"

namespace sparc {

const TileShape kShapes[kNumShapes] = {{32, 2, 256}, {32, 2, 512}, {32, 2, 768}, {64, 2, 256},
                                       {64, 2, 512}, {32, 4, 256}};

template <typename T>
struct StepArgs {
    const T *yk;
    const T *yprev;
    T *out;
    const T *veff;
    long long ldk, ldp, ldo;
    int n1, n2, n3;
    int tiles_y, tiles_z, nchunks, chunk_x;
    int nblocks;
    T c0;              // centre coefficient of -1/2 lap_h: -3 w_0
    T cp[kMaxRadius];  // -1/2 w_p, p = 1..kMaxRadius (zero beyond the op's radius)
    T alpha, beta, shift;
};

template <typename T, int TZ, int RY, int NT, bool PREV>
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

    const StepArgs<T> &a;
    const T *yk;
    const T *yp;
    T *out;
    long long P;
    int lz, lyg, xs, xe;
    int pofs[RY];    // in-plane offset of the own points
    bool pok[RY];
    int hofs[NH];    // in-plane offset of the halo values (0 when outside)
    bool hok[NH];
    int hl[NH];
    T q[RY][QL];

    __device__ StepKernel(const StepArgs<T> &args) : a(args) {}

    __device__ __forceinline__ void load_stage(Stage &s, int t) const
    {
        const bool tin = t < a.n1;
        const long long base = (long long)(tin ? t : 0) * P;
#pragma unroll
        for (int i = 0; i < NH; ++i) {
            const bool ok = tin && hok[i];
            const T v = yk[base + (ok ? hofs[i] : 0)];
            s.h[i] = ok ? v : T(0);
        }
        const int th = t + R;
        const bool hin = th < a.n1;
        const long long hbase = (long long)(hin ? th : 0) * P;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const bool ok = hin && pok[r];
            const T v = yk[hbase + (ok ? pofs[r] : 0)];
            s.qh[r] = ok ? v : T(0);
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const long long g = base + (pok[r] ? pofs[r] : 0);
            s.v[r] = a.veff[g];
            if constexpr (PREV) s.p[r] = yp[g];
        }
    }

    // plane x, stage / LDS buffer S; the queue holds planes x-R .. x+R
    template <int S>
    __device__ __forceinline__ void plane(int x, Stage (&st)[2], T (*lds)[SY * SZ])
    {
        Stage &s = st[S];
        T *L = lds[S];
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][2 * R] = s.qh[r];
        // publish the centre plane and its halo
#pragma unroll
        for (int r = 0; r < RY; ++r) L[(R + lyg * RY + r) * SZ + R + lz] = q[r][R];
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

        T *po = out;
        const long long pbase = (long long)x * P;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int li = (R + lyg * RY + r) * SZ + R + lz;
            const T c = q[r][R];
            T acc = a.c0 * c;
#pragma unroll
            for (int p = 1; p <= R; ++p) {
                const T ym = (r - p >= 0) ? q[r - p][R] : L[li - p * SZ];
                const T ypl = (r + p < RY) ? q[r + p][R] : L[li + p * SZ];
                const T six = (q[r][R - p] + q[r][R + p]) + (ym + ypl) + (L[li - p] + L[li + p]);
                acc += a.cp[p - 1] * six;
            }
            acc += (vcur[r] - a.shift) * c;
            T res = a.alpha * acc;
            if constexpr (PREV) res -= a.beta * pcur[r];
            if (pok[r]) po[pbase + pofs[r]] = res;
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int d = 0; d < 2 * R; ++d) q[r][d] = q[r][d + 1];
    }

    __device__ void run()
    {
        __shared__ T lds[2][SY * SZ];
        // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
        // contiguous range of patches so that neighbours share its L2.
        const int nb = a.nblocks;
        const int b = blockIdx.x;
        const int xcd = b & 7;
        int t = xcd * (nb >> 3) + min(xcd, nb & 7) + (b >> 3);
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
            pofs[r] = y * n3 + z;
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
            hok[i] = ly >= 0 && gy >= 0 && gy < n2 && gz >= 0 && gz < n3;
            hofs[i] = hok[i] ? gy * n3 + gz : 0;
        }
        xs = chunk * a.chunk_x;
        xe = min(a.n1, xs + a.chunk_x);

        // queue: planes xs-R .. xs+R-1 (heads are filled from the stages)
#pragma unroll
        for (int d = 0; d < 2 * R; ++d) {
            const int xx = xs - R + d;
            const bool in = xx >= 0 && xx < a.n1;
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const bool ok = in && pok[r];
                const T v = yk[(long long)(ok ? xx : 0) * P + (ok ? pofs[r] : 0)];
                q[r][d] = ok ? v : T(0);
            }
        }
        Stage st[2];
        load_stage(st[0], xs);
        load_stage(st[1], xs + 1);
        int x = xs;
        for (; x + 1 < xe; x += 2) {
            plane<0>(x, st, lds);
            plane<1>(x + 1, st, lds);
        }
        if (x < xe) plane<0>(x, st, lds);
    }
};

template <typename T, int TZ, int RY, int NT, bool PREV>
__global__ void __launch_bounds__(NT) step_kernel(const StepArgs<T> a)
{
    StepKernel<T, TZ, RY, NT, PREV> k(a);
    k.run();
}

StepLaunch choose_step_launch(const sparc_op *op, int dtype, int ns)
{
    StepLaunch L;
    // 32 x 16 patches of 256 threads measured fastest for both dtypes on the
    // 96^3 and larger grids (lowest register footprint, 4-5 waves per SIMD)
    L.shape = 0;
    if (op->tune_shape[dtype] >= 0) L.shape = op->tune_shape[dtype];
    const TileShape &s = kShapes[L.shape];
    const long long tiles = (long long)((op->n[1] + s.ty() - 1) / s.ty()) * ((op->n[2] + s.tz - 1) / s.tz);
    const long long waves = tiles * ns * (s.nt / 64);
    // split x so that about 8192 waves are in flight, keeping >= 4 planes per chunk
    long long nchunks = (8192 + waves - 1) / waves;
    nchunks = std::max<long long>(1, std::min<long long>(nchunks, op->n[0] / 4));
    L.chunk_x = (int)((op->n[0] + nchunks - 1) / nchunks);
    if (op->tune_chunk[dtype] > 0) L.chunk_x = std::min(op->n[0], op->tune_chunk[dtype]);
    return L;
}

template <typename T, int TZ, int RY, int NT>
static int launch_typed(const StepArgs<T> &a, bool prev, hipStream_t stream)
{
    if (prev)
        hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, true>), dim3(a.nblocks), dim3(NT), 0, stream, a);
    else
        hipLaunchKernelGGL((step_kernel<T, TZ, RY, NT, false>), dim3(a.nblocks), dim3(NT), 0, stream, a);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

template <typename T>
static int launch_step_t(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                         void *out, int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L,
                         hipStream_t stream, const T *veff)
{
    const TileShape &s = kShapes[L.shape];
    StepArgs<T> a;
    a.yk = (const T *)yk;
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
    a.c0 = (T)(-3.0 * op->w[0]);
    for (int p = 1; p <= kMaxRadius; ++p) a.cp[p - 1] = (T)(-0.5 * op->w[p]);
    a.alpha = (T)c.alpha;
    a.beta = (T)c.beta;
    a.shift = (T)c.shift;
    ProfScope prof(prev ? 0 : 3, stream);
    switch (L.shape) {
        case 0: return launch_typed<T, 32, 2, 256>(a, prev, stream);
        case 1: return launch_typed<T, 32, 2, 512>(a, prev, stream);
        case 2: return launch_typed<T, 32, 2, 768>(a, prev, stream);
        case 3: return launch_typed<T, 64, 2, 256>(a, prev, stream);
        case 4: return launch_typed<T, 64, 2, 512>(a, prev, stream);
        case 5: return launch_typed<T, 32, 4, 256>(a, prev, stream);
    }
    return fail(SPARC_E_ARG, "unknown tile shape");
}

int launch_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                void *out, int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream)
{
    if (dtype == SPARC_F64)
        return launch_step_t<double>(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, op->d_veff64);
    return launch_step_t<float>(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, op->d_veff32);
}

}  // namespace sparc
