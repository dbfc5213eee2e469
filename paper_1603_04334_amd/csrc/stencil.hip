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
//    on its own rows are read from the queue centres as well.  The plane loop
//    is unrolled over 2(2R+1) planes so that the queue rotates by renaming
//    registers instead of moving values.
//  * The current plane of the patch plus a cross-shaped halo (R rows in y, R
//    columns in z) is staged in LDS, double-buffered with one barrier per
//    plane; the remaining y- and z-neighbours come from there.  Halo values
//    belong to neighbouring patches and are served from L2 when neighbours
//    run on the same XCD, which the workgroup-index remap arranges.
//  * All global accesses are unconditional raw buffer loads and stores
//    through per-plane descriptors: a point or plane outside the grid falls
//    outside the descriptor's range, so it loads zero and its store is
//    dropped, without selects or 64-bit address arithmetic.  Loads are issued
//    two planes ahead, so each wait only covers loads issued one full plane
//    earlier.
//  * Patch shapes: 32 x 16 with 256 threads (FP64), 32 x 48 with 768 threads
//    (FP32 filter: fewer halo re-reads), 32 x 32 with 512 threads (FP64 H on
//    an FP32 block); sparc_autotune may override the filter's choice.
//  * yprev is read pointwise and out may alias it: a thread reads yprev(x)
//    one plane before it writes out(x), and no other thread touches x.
//  * When the three blocks of a step exceed the last-level (Infinity) cache,
//    yprev and out are streamed with non-temporal loads and stores, so the
//    L2 keeps the values that are reused (halos of Y_k, V_eff) instead;
//    smaller blocks stay cached from one step to the next.
#include "step_launch.hpp"

namespace sparc {

// scalar step kernels: 32 x 16 patches of 256 threads (filters and H X that
// the vector kernels cannot take), 32 x 32 patches of 512 threads (FP64 H on
// FP32 blocks)
const TileShape kShapes[kNumShapes] = {{32, 2, 256}, {32, 2, 512}};

// H v for one FP64 vector in one launch: the first ngather workgroups gather
// the projections of v (atom i % natoms, split i / natoms, as the standalone
// gather), the rest run the DOT step on 32 x 16 patches.  ngather is a
// multiple of 8, so the step's XCD-aware index remap still sees the hardware
// round-robin.
__global__ void __launch_bounds__(256) lanczos_h_kernel(const StepArgs<double, double> a,
                                                        const GatherArgs<double, double> g, int natoms, int ngather)
{
    if ((int)blockIdx.x < ngather) {
        __shared__ double tile[4][16][16];
        gather_item<double, double>(g, blockIdx.x % natoms, 0, blockIdx.x / natoms, tile, threadIdx.x);
        return;
    }
    using K = StepKernel<double, 32, 2, 256, false, false, double, true>;
    __shared__ double lds[2][K::SY * K::SZ];
    const int b = blockIdx.x - ngather;
    K k(a);
    k.run(b, lds);
    store_dot<double, 256>(k.dacc, a.dot, b);
}

// split x so that about 8192 waves are in flight, keeping >= 4 planes per chunk
static int default_chunk(const sparc_op *op, int shape, int ns)
{
    const TileShape &s = kShapes[shape];
    const long long tiles = (long long)((op->n[1] + s.ty() - 1) / s.ty()) * ((op->n[2] + s.tz - 1) / s.tz);
    const long long waves = tiles * ns * (s.nt / 64);
    long long nchunks = (8192 + waves - 1) / waves;
    nchunks = std::max<long long>(1, std::min<long long>(nchunks, op->n[0] / 4));
    return (int)((op->n[0] + nchunks - 1) / nchunks);
}

// taller patches cut the halo re-reads but pad n[1] up to a multiple of their
// height: take the taller one (shape) when its measured per-point time
// (speed, relative to 32 x 16) outweighs the padding
static int pick_taller(const sparc_op *op, int shape, double speed)
{
    const int ty = kShapes[shape].ty();
    const long long pad16 = (op->n[1] + 15) / 16 * 16, padt = (op->n[1] + ty - 1) / ty * ty;
    return speed * padt < pad16 ? shape : 0;
}

StepLaunch choose_step_launch(const sparc_op *op, int dtype, int ns)
{
    (void)dtype;
    StepLaunch L;
    L.shape = 0;
    L.chunk_x = default_chunk(op, L.shape, ns);
    return L;
}

// FP64 application of H to an FP32 block (Rayleigh-Ritz): 32 x 32 patches of
// 512 threads measured 19% faster per point than 32 x 16 on the 96^3 grid;
// launch overrides, which are tuned for the filter, do not apply
StepLaunch choose_mixed_launch(const sparc_op *op, int ns)
{
    StepLaunch L;
    L.shape = pick_taller(op, 1, 0.81);
    L.chunk_x = default_chunk(op, L.shape, ns);
    return L;
}

// per-type launches (step_f32.hip, step_f64.hip, step_mixed.hip)
int launch_step_f32(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp, void *out,
                    int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream, void *part);
int launch_step_f64(const sparc_op *op, const void *yk, int64_t ldk, const void *yprev, int64_t ldp, void *out,
                    int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream, void *part);
int launch_step_mixed(const sparc_op *op, const float *yk, int64_t ldk, double *out, int64_t ldo, int ns,
                      const StepCoef &c, const StepLaunch &L, hipStream_t stream);

int launch_step_f32_to_f64(const sparc_op *op, const float *yk, int64_t ldk, double *out, int64_t ldo, int ns,
                           const StepCoef &c, const StepLaunch &L, hipStream_t stream)
{
    if (c.has_prev) return fail(SPARC_E_ARG, "mixed-precision step has no Y_{k-1} term");
    return launch_step_mixed(op, yk, ldk, out, ldo, ns, c, L, stream);
}

int launch_step_gather(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                       void *out, int64_t ldo, int ns, void *part, const StepCoef &c, const StepLaunch &L,
                       hipStream_t stream)
{
    if (dtype == SPARC_F64) return launch_step_f64(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, part);
    return launch_step_f32(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, part);
}

int launch_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                void *out, int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream)
{
    if (dtype == SPARC_F64) return launch_step_f64(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, nullptr);
    return launch_step_f32(op, yk, ldk, yprev, ldp, out, ldo, ns, c, L, stream, nullptr);
}

// The single-vector FP64 step of the Lanczos iteration: 32 x 16 patches and
// the default x split, independent of any launch override, so that the
// workgroup count (one partial each) is fixed by the grid alone.
static StepLaunch dot_launch(const sparc_op *op)
{
    StepLaunch L;
    L.shape = 0;
    L.chunk_x = default_chunk(op, 0, 1);
    return L;
}

long long step_dot_blocks(const sparc_op *op)
{
    const TileShape &s = kShapes[0];
    const StepLaunch L = dot_launch(op);
    return (long long)((op->n[0] + L.chunk_x - 1) / L.chunk_x) * ((op->n[1] + s.ty() - 1) / s.ty()) *
           ((op->n[2] + s.tz - 1) / s.tz);
}

int launch_lanczos_h_f64(const sparc_op *op, const double *v, double *out, double *dot, double *part,
                         hipStream_t stream)
{
    const TileShape &s = kShapes[0];
    const StepLaunch L = dot_launch(op);
    StepArgs<double, double> a;
    a.yk = v;
    a.yprev = nullptr;
    a.out = out;
    a.veff = op->d_veff64;
    a.ldk = a.ldp = a.ldo = op->nd;
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.n3 = op->n[2];
    a.tiles_y = (op->n[1] + s.ty() - 1) / s.ty();
    a.tiles_z = (op->n[2] + s.tz - 1) / s.tz;
    a.chunk_x = L.chunk_x;
    a.nchunks = (op->n[0] + L.chunk_x - 1) / L.chunk_x;
    const long long nb = step_dot_blocks(op);
    if (nb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
    a.nblocks = (int)nb;
    a.remap = 1;
    a.dot = dot;
    a.c0 = -3.0 * op->w[0];
    for (int p = 1; p <= kMaxRadius; ++p) a.cp[p - 1] = -0.5 * op->w[p];
    a.alpha = 1.0;
    a.beta = 0.0;
    a.shift = 0.0;
    GatherArgs<double, double> g;
    g.Y = v;
    g.ldy = op->nd;
    g.ns = 1;
    g.nproj_total = op->nproj_total;
    g.atoms = op->d_atoms;
    g.box_off = op->d_box_off;
    g.chi = op->d_chi64;
    g.part = part;
    const int ngather = op->natoms * kGatherSplit;
    ProfScope prof(3, stream);
    hipLaunchKernelGGL(lanczos_h_kernel, dim3(ngather + a.nblocks), dim3(256), 0, stream, a, g, op->natoms, ngather);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

}  // namespace sparc
