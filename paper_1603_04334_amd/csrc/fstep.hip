// Vector step: one pass over an orbital block computes, for every node x and
// column c,
//     out(x,c) = alpha * ( -1/2 lap_h yk + (V_eff(x) - shift) yk )(x,c) - beta * yprev(x,c)
// the local part of one step of the three-term Chebyshev recurrence of Sec.
// 3.4 (its first step without yprev, or a plain application of H), with the
// stencil of Sec. 3.1 Eq. FD:Laplacian and f = 0 off the grid.  The same
// launch gathers the projections chi_Jp^T yk of the input on the matrix cores
// (its last workgroups); the projector scatter that follows adds
// alpha V_nl yk (Sec. 3.1 Eq. non-localPS:FD).
//
// Data movement (HBM-bound):
//  * A workgroup owns a TY x TZ patch (TZ = 32, 64, 80 or 160 nodes) of the
//    (y, z) plane of one column and streams it along x (wider patches cut the
//    share of the z halo, whose two partial lines per row are fetched whole;
//    a patch as wide as the grid has none).  Each lane owns one unit of consecutive z nodes of one
//    y row: 4 FP32 or 2 FP64 values, 16 bytes, so every global access is a
//    16-byte raw buffer load or store (a plain copy with 4-byte accesses per
//    lane reaches about 60% of the bandwidth of 16-byte accesses on this
//    chip).  A lane keeps the 13 x-planes of its unit in registers, one vector
//    per plane (x neighbours never touch LDS); the plane loop is unrolled over
//    26 planes so the queue rotates by register renaming.
//  * The current plane of the patch plus its halo (6 rows in y; 8 FP32 / 6
//    FP64 nodes in z, whole units) is staged in LDS, double-buffered with one
//    barrier per plane; y and z neighbours are read there as 16-byte units.
//  * Loads are issued two planes ahead; points and planes outside the grid
//    fall outside the per-plane buffer descriptor's range (load zero, store
//    dropped).  The grid's z extent and every leading dimension must be
//    multiples of the unit, so a unit is either inside the grid or outside;
//    other grids take the scalar kernels (stencil.hip).
//  * Per point the sums run in the same order as in the scalar kernels.
//  * Workgroup indices are remapped so consecutive patches of one column run
//    on the same XCD and share halos in its L2 (optionally, col_group columns
//    of one patch run back to back and share V_eff); yprev and out are streamed
//    non-temporally when a step's blocks exceed the last-level cache.
//  * Orbital blocking (col_block = 2): one workgroup steps two columns of the
//    same patch, loading V_eff once for both and sharing the halo offsets and
//    the plane loop; each column keeps its own register queue and LDS plane.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "fstep_launch.hpp"

namespace sparc {

static int vec_width(int dtype) { return dtype == SPARC_F64 ? 2 : 4; }

// patches offered per dtype (TY x TZ): FP64 8, 16, 32 x 32 and 8, 16, 24 x 64;
// FP32 16, 32, 64 x 32, 16, 32 x 64, 32 x 80 and 24 x 160 (128 to 960
// threads).  The wide ones cut the halo: a 24 x 160 patch spans a whole
// 160-node row, so it has no z halo at all and a y halo of 12 rows per 24.
static int vec_default_plan(int dtype) { return dtype == SPARC_F64 ? 1 : 2; }  // 16 x 32 FP64, 32 x 32 FP32

static int vec_nt(int dtype, int plan) { return (kPlanTZ[plan] / vec_width(dtype)) * kPlanTY[plan]; }

bool vec_plan_valid(int dtype, int plan)
{
    static const bool f64[kNumPlans] = {true, true, true, false, true, true, false, false, false, true};
    static const bool f32[kNumPlans] = {false, true, true, true, false, true, true, true, true, false};
    if (plan < 0 || plan >= kNumPlans) return false;
    return dtype == SPARC_F64 ? f64[plan] : f32[plan];
}

// two columns per workgroup double the register queues: only patches of at
// most 512 threads (whose waves may use 256 registers) take them
int vec_max_cblk(int dtype, int plan) { return vec_nt(dtype, plan) <= 512 ? 2 : 1; }

// split x so that about 8192 waves are in flight (at most kMaxChunks chunks,
// at least 4 planes each)
static int vec_default_chunks(const sparc_op *op, int dtype, int plan, int ns)
{
    const int ty = kPlanTY[plan], tz = kPlanTZ[plan];
    const long long tiles = (long long)((op->n[1] + ty - 1) / ty) * ((op->n[2] + tz - 1) / tz);
    const long long waves = tiles * ns * (vec_nt(dtype, plan) / 64);
    long long nch = (8192 + waves - 1) / waves;
    nch = std::max<long long>(1, std::min<long long>({nch, (long long)kMaxChunks, (long long)op->n[0] / 4}));
    return (int)nch;
}

static void set_chunks(const sparc_op *op, int nch, FLaunch &L)
{
    nch = std::max(1, std::min(nch, std::min(kMaxChunks, op->n[0])));
    L.chunk_x = (op->n[0] + nch - 1) / nch;
    L.nchunks = (op->n[0] + L.chunk_x - 1) / L.chunk_x;
}

FLaunch choose_vec_launch(const sparc_op *op, int dtype, int ns, std::initializer_list<int64_t> lds)
{
    FLaunch L;
    const int vz = vec_width(dtype);
    if (op->n[2] % vz != 0) return L;
    for (int64_t ld : lds)
        if (ld % vz != 0) return L;
    int plan = vec_default_plan(dtype);
    const bool tuned = tune_applies(op, dtype, ns);
    if (tuned && op->tune_shape[dtype] >= 0 && vec_plan_valid(dtype, op->tune_shape[dtype]))
        plan = op->tune_shape[dtype];
    int nch = vec_default_chunks(op, dtype, plan, ns);
    if (tuned && op->tune_chunk[dtype] > 0) nch = (op->n[0] + op->tune_chunk[dtype] - 1) / op->tune_chunk[dtype];
    L.plan = plan;
    set_chunks(op, nch, L);
    L.cgroup = (tuned && op->tune_group[dtype] > 0) ? op->tune_group[dtype] : 1;
    L.cblk = (tuned && op->tune_cblk[dtype] == 2 && vec_max_cblk(dtype, plan) == 2) ? 2 : 1;
    return L;
}

FLaunch vec_launch_plan(const sparc_op *op, int dtype, int ns, int plan)
{
    FLaunch L;
    L.plan = plan;
    set_chunks(op, vec_default_chunks(op, dtype, plan, ns), L);
    return L;
}

template <typename T>
static int launch_fstep_t(const sparc_op *op, const FLaunch &L, const void *yk, int64_t ldk, const void *yprev,
                          int64_t ldp, void *out, int64_t ldo, int ns, void *part, const StepCoef &c,
                          hipStream_t stream)
{
    const int ty = kPlanTY[L.plan], tz = kPlanTZ[L.plan];
    const int nt = (tz / VecTraits<T>::N) * ty;
    FStepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.yk = (const T *)yk;
    a.yprev = (const T *)yprev;
    a.out = (T *)out;
    a.veff = std::is_same<T, double>::value ? (const T *)op->d_veff64 : (const T *)op->d_veff32;
    a.ldk = ldk;
    a.ldp = ldp;
    a.ldo = ldo;
    a.n1 = op->n[0];
    a.n2 = op->n[1];
    a.n3 = op->n[2];
    a.tiles_y = (op->n[1] + ty - 1) / ty;
    a.tiles_z = (op->n[2] + tz - 1) / tz;
    a.chunk_x = L.chunk_x;
    a.nchunks = L.nchunks;
    const int cb = L.cblk == 2 ? 2 : 1;
    const int ngroups = (ns + cb - 1) / cb;  // column blocks
    const int G = std::max(1, std::min(L.cgroup, ngroups));
    const long long nb = (long long)(ngroups + G - 1) / G * G * L.nchunks * a.tiles_y * a.tiles_z;
    if (nb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
    a.nblocks = (int)nb;
    a.remap = 1;
    a.ns = ns;
    a.cgroup = G;
    a.c0 = (T)(-3.0 * op->w[0]);
    for (int p = 1; p <= kMaxRadius; ++p) a.cp[p - 1] = (T)(-0.5 * op->w[p]);
    a.alpha = (T)c.alpha;
    a.beta = (T)c.beta;
    a.shift = (T)c.shift;
    const bool prev = c.has_prev && yprev != nullptr;
    // blocks the last-level cache cannot keep between steps are streamed
    const bool strm = (double)op->nd * ns * 3 * sizeof(T) > kStreamBytes;
    GatherArgs<T, T> g;
    std::memset(&g, 0, sizeof(g));
    int ncb = 0, nitems = 0, ngb = 0;
    if (part && op->natoms > 0) {
        if ((long long)(ns + 15) / 16 > 65535) return fail(SPARC_E_SHAPE, "too many columns for one gather launch");
        if (nt < 256) {
            // the patch is too small to host gather items: a launch of its own
            int st;
            if ((st = launch_gather(op, std::is_same<T, double>::value ? SPARC_F64 : SPARC_F32, yk, ldk, ns, part,
                                    stream)))
                return st;
        } else {
            g.Y = (const T *)yk;
            g.ldy = ldk;
            g.ns = ns;
            g.nproj_total = op->nproj_total;
            g.atoms = op->d_atoms;
            g.box_off = op->d_box_off;
            g.chi = std::is_same<T, double>::value ? (const T *)op->d_chi64 : (const T *)op->d_chi32;
            g.part = (T *)part;
            ncb = (ns + 15) / 16;
            nitems = op->natoms * ncb * kGatherSplit;
            const int per = nt / 256;
            ngb = (nitems + per - 1) / per;
            if ((long long)a.nblocks + ngb > 0x7fffffffLL) return fail(SPARC_E_SHAPE, "too many workgroups for one launch");
        }
    }
    ProfScope prof(prev ? 0 : 3, stream);
    const int natoms = std::max(op->natoms, 1);
    if constexpr (std::is_same<T, float>::value) {
        if (tz == 160) {
            if (ty == 24) return fstep_f32_ty24_tz160(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
        } else if (tz == 80) {
            if (ty == 32) return fstep_f32_ty32_tz80(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
        } else if (tz == 64) {
            switch (ty) {
                case 16: return fstep_f32_ty16_tz64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 32: return fstep_f32_ty32_tz64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
            }
        } else {
            switch (ty) {
                case 16: return fstep_f32_ty16(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 32: return fstep_f32_ty32(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 64: return fstep_f32_ty64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
            }
        }
    } else {
        if (tz == 64) {
            switch (ty) {
                case 8: return fstep_f64_ty8_tz64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 16: return fstep_f64_ty16_tz64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 24: return fstep_f64_ty24_tz64(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
            }
        } else {
            switch (ty) {
                case 8: return fstep_f64_ty8(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 16: return fstep_f64_ty16(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
                case 32: return fstep_f64_ty32(a, g, natoms, ncb, nitems, ngb, prev, strm, cb, stream);
            }
        }
    }
    return fail(SPARC_E_ARG, "patch height not available for this dtype");
}

int launch_fstep(const sparc_op *op, int dtype, const FLaunch &L, const void *yk, int64_t ldk, const void *yprev,
                 int64_t ldp, void *out, int64_t ldo, int ns, void *part, const StepCoef &c, hipStream_t stream)
{
    if (L.plan < 0) return fail(SPARC_E_ARG, "vector step not available");
    if (dtype == SPARC_F64)
        return launch_fstep_t<double>(op, L, yk, ldk, yprev, ldp, out, ldo, ns, part, c, stream);
    return launch_fstep_t<float>(op, L, yk, ldk, yprev, ldp, out, ldo, ns, part, c, stream);
}

}  // namespace sparc
