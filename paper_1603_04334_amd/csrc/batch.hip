// Batched Chebyshev filters of uneven clusters in one persistent launch.
//
// Every filter of the batch is cut into work items of the same three kinds a
// standalone filter launches per degree step k (Sec. 3.4, Alg. 2):
//   A(k): projector-gather items (atom, split; all column blocks) and vector
//         stencil items (patch, x-chunk, group of 8 columns) of step k;
//   B(k): projector-scatter items (node block; all column groups) of step k.
// Dependencies per cluster: A(k) needs B(k-1) complete (A(k-1) when the cluster
// has no atoms), B(k) needs A(k) complete.  Items are numbered in level order
// (level 2k = A(k) of every cluster, level 2k+1 = B(k) of every cluster), and
// the persistent workgroups take them from one atomic ticket counter in that
// order, so an item only ever waits for items with smaller tickets, which are
// already held by running workgroups: the schedule cannot deadlock, whatever
// the grid size.  Each wait is additionally bounded; on timeout the batch
// raises an abort flag, every workgroup drains, and the host reports an error.
//
// Completion is published with a device-scope release (barrier, then one
// release increment of the counter) and observed with a device-scope acquire, so
// data written on one XCD is read correctly on another.  Each item runs exactly
// the arithmetic of the corresponding standalone kernel (the stencil items use
// the 256-thread vector patch of their dtype: 32 x 32 FP32, 16 x 32 FP64, whose
// per-point sums equal those of every other patch), so a cluster's result is
// bit-identical alone and in the batch.  Batched modes need grids and leading
// dimensions the vector kernels take.
//
// Modes: 0 = persistent kernel captured with the counter reset in a HIP graph
// (replayed on later runs); 1 = the same two launches without a graph;
// 2 = one grouped launch per level (kernel boundaries as barriers, no waits);
// 3 = the plain per-cluster filters one after another (reference);
// 4 = mode 2 captured in a HIP graph; 5 = the plain per-cluster filters
// (their tuned launches) on kBatchLanes streams of the batch, jobs dealt
// longest first to the least loaded stream, joined to the caller's stream
// by events: one cluster's launch tails and the gaps between its dependent
// launches overlap another's work.  Each job runs on one stream with its own
// workspace, so its result does not depend on the interleaving.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "fstep_kernel.hpp"
#include "nonlocal_kernel.hpp"

namespace sparc {

struct BatchClusterDev {
    // operator
    const void *veff;
    const void *chi;
    const void *hg;
    const AtomDev *atoms;
    const int *box_off;
    const int *blk_pt, *blk_at, *blk_atoms, *pts, *ent_off;
    const int4 *ent;
    int natoms, nproj_total, nl_nblk;
    int n1, n2, n3;
    int dtype;
    int ns, m;
    // buffers
    const void *X;
    void *P, *Q;  // Y_j lands in P for odd j, in Q for even j
    void *G;      // gather partials
    long long ldx, ldp, ldq;
    // stencil geometry (256-thread vector patches)
    int tiles_y, tiles_z, nchunks, chunk_x;
    // items per step
    int nG, nS, nC, ncb, ncg;
    double c0, cp[kMaxRadius];
    const double *coef;  // per step: alpha, beta, shift
    int *cntA, *cntB;    // per-step completion counters
};

constexpr int kBatchLanes = 4;  // streams of the concurrent mode (the process's default hardware queues)

struct BatchSegment {
    long long start;
    int cluster, kind, step, count;
};

struct BatchArgs {
    const BatchClusterDev *cl;
    const BatchSegment *seg;
    int nseg;
    long long total;
    unsigned int *ticket;
    int *abort;
    long long spin_limit;
    long long base;  // levelled mode: first item of the launch
    int waits;       // persistent mode: 1
};

constexpr int kBatchNT = 256;
constexpr int kBatchPlan[2] = {1, 2};  // per dtype (F64, F32): the 256-thread patch heights

template <typename T>
struct BatchTY;
template <>
struct BatchTY<float> {
    static constexpr int TY = 32;
};
template <>
struct BatchTY<double> {
    static constexpr int TY = 16;
};
template <typename T, bool PREV>
using BStep = FStep<T, BatchTY<T>::TY, PREV, false>;

constexpr int kBatchColGroup = 8;  // columns per stencil item

struct StepSel {
    const void *yk, *yprev;
    void *out;
    long long ldk, ldp, ldo;
};

__device__ inline StepSel select_buffers(const BatchClusterDev &c, int k)
{
    StepSel s;
    const bool odd_next = ((k + 1) & 1) != 0;
    s.out = odd_next ? c.P : c.Q;
    s.ldo = odd_next ? c.ldp : c.ldq;
    s.yk = k == 0 ? c.X : ((k & 1) ? c.P : c.Q);
    s.ldk = k == 0 ? c.ldx : ((k & 1) ? c.ldp : c.ldq);
    s.yprev = k == 1 ? c.X : s.out;  // Y_{k-1}, overwritten in place from k = 2 on
    s.ldp = k == 1 ? c.ldx : s.ldo;
    return s;
}

// projector gather of step k: item = (atom, split), all column blocks
template <typename T>
__device__ __forceinline__ void do_gather(const BatchClusterDev &c, int k, int local, char *smem)
{
    const StepSel sel = select_buffers(c, k);
    GatherArgs<T> g;
    g.Y = (const T *)sel.yk;
    g.ldy = sel.ldk;
    g.ns = c.ns;
    g.nproj_total = c.nproj_total;
    g.atoms = c.atoms;
    g.box_off = c.box_off;
    g.chi = (const T *)c.chi;
    g.part = (T *)c.G;
    const int atom = local / kGatherSplit, ks = local % kGatherSplit;
#pragma unroll 1
    for (int cb = 0; cb < c.ncb; ++cb) {
        gather_item<T>(g, atom, cb, ks, (T(*)[16][16])smem, threadIdx.x);
        __syncthreads();
    }
}

// stencil of step k: item = (patch, x-chunk, group of kBatchColGroup columns)
template <typename T, bool PREV>
__device__ __forceinline__ void do_step(const BatchClusterDev &c, int k, int local, char *smem)
{
    using K = BStep<T, PREV>;
    const StepSel sel = select_buffers(c, k);
    FStepArgs<T> a;
    a.yk = (const T *)sel.yk;
    a.yprev = (const T *)sel.yprev;
    a.out = (T *)sel.out;
    a.veff = (const T *)c.veff;
    a.ldk = sel.ldk;
    a.ldp = sel.ldp;
    a.ldo = sel.ldo;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.n3 = c.n3;
    a.tiles_y = c.tiles_y;
    a.tiles_z = c.tiles_z;
    a.nchunks = c.nchunks;
    a.chunk_x = c.chunk_x;
    a.nblocks = c.nS;
    a.remap = 0;
    a.ns = c.ns;
    a.cgroup = 1;
    a.c0 = (T)c.c0;
    for (int p = 0; p < kMaxRadius; ++p) a.cp[p] = (T)c.cp[p];
    const double *cf = c.coef + 3 * k;
    a.alpha = (T)cf[0];
    a.beta = (T)cf[1];
    a.shift = (T)cf[2];
    const int per_col = c.tiles_y * c.tiles_z * c.nchunks;
    const int tc = local % per_col, g = local / per_col;
    const int c1 = min(c.ns, (g + 1) * kBatchColGroup);
#pragma unroll 1
    for (int col = g * kBatchColGroup; col < c1; ++col) {
        K s(a);
        s.run(col * per_col + tc, *(typename K::Shared *)smem);
        __syncthreads();
    }
}

// projector scatter of step k: item = node block, all column groups
template <typename T>
__device__ __forceinline__ void do_scatter(const BatchClusterDev &c, int k, int local, char *smem)
{
    const StepSel sel = select_buffers(c, k);
    ScatterArgs<T> sa;
    sa.out = (T *)sel.out;
    sa.ldo = sel.ldo;
    sa.ns = c.ns;
    sa.nproj_total = c.nproj_total;
    sa.blk_pt = c.blk_pt;
    sa.blk_at = c.blk_at;
    sa.blk_atoms = c.blk_atoms;
    sa.pts = c.pts;
    sa.ent_off = c.ent_off;
    sa.ent = c.ent;
    sa.atoms = c.atoms;
    sa.chi = (const T *)c.chi;
    sa.hg = (const T *)c.hg;
    sa.part = (const T *)c.G;
    sa.alpha = (T)c.coef[3 * k];
#pragma unroll 1
    for (int cg = 0; cg < c.ncg; ++cg) {
        scatter_item<T, kScatterCols>(sa, local, cg, (T *)smem, kMaxProj);
        __syncthreads();
    }
}

template <typename T>
__device__ __forceinline__ void run_item(const BatchClusterDev &c, int kind, int k, int local, char *smem)
{
    if (kind == 1)
        do_scatter<T>(c, k, local, smem);
    else if (local < c.nG)
        do_gather<T>(c, k, local, smem);
    else if (k == 0)
        do_step<T, false>(c, k, local - c.nG, smem);
    else
        do_step<T, true>(c, k, local - c.nG, smem);
}

__device__ inline int find_segment(const BatchSegment *seg, int nseg, int t)
{
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg[mid].start <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

constexpr size_t cmax(size_t x, size_t y) { return x > y ? x : y; }
constexpr size_t kBatchLds = cmax(sizeof(BStep<float, true>::Shared), sizeof(BStep<double, true>::Shared));

template <bool F32, bool F64>
__global__ void __launch_bounds__(kBatchNT) batch_kernel(const BatchArgs args)
{
    // the stencil planes, the gather tile or the scatter table
    __shared__ __align__(16) char smem[cmax(cmax(kBatchLds, sizeof(double) * 4 * 16 * 16),
                                            sizeof(double) * kScatterSlots * kMaxProj * kScatterCols)];
    __shared__ int s_t;
    __shared__ int s_go;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            if (args.waits)
                s_t = __hip_atomic_load(args.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          ? (int)args.total
                          : (int)atomicAdd(args.ticket, 1u);
            else
                s_t = (int)args.base + (int)blockIdx.x;
        }
        __syncthreads();
        // the ticket is the same for the whole workgroup: make that explicit so
        // the schedule and cluster descriptor are read with scalar loads
        const int t = __builtin_amdgcn_readfirstlane(s_t);
        if (t >= args.total) break;
        const BatchSegment sg = args.seg[find_segment(args.seg, args.nseg, t)];
        const BatchClusterDev &c = args.cl[sg.cluster];
        const int local = t - (int)sg.start;
        if (args.waits) {
            if (tid == 0) {
                const int *cnt = nullptr;
                int target = 0;
                if (sg.kind == 0 && sg.step > 0) {
                    if (c.natoms > 0) {
                        cnt = c.cntB + (sg.step - 1);
                        target = c.nC;
                    } else {
                        cnt = c.cntA + (sg.step - 1);
                        target = c.nS;
                    }
                } else if (sg.kind == 1) {
                    cnt = c.cntA + sg.step;
                    target = c.nG + c.nS;
                }
                int go = 1;
                if (cnt) {
                    long long it = 0;
                    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                        if (__hip_atomic_load(args.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            go = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                        if (++it > args.spin_limit) {
                            __hip_atomic_store(args.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            go = 0;
                            break;
                        }
                    }
                }
                s_go = go;
            }
            __syncthreads();
            if (!s_go) {
                __syncthreads();
                continue;
            }
        }
        if (F32 && c.dtype == SPARC_F32) run_item<float>(c, sg.kind, sg.step, local, smem);
        if (F64 && c.dtype == SPARC_F64) run_item<double>(c, sg.kind, sg.step, local, smem);
        if (!args.waits) break;  // grouped launch: one item per workgroup
        {
            // every wave's stores have completed to L2 at the barrier; one
            // device-scope release then publishes them with the count
            __syncthreads();
            if (tid == 0) {
                int *cnt = (sg.kind == 0 ? c.cntA : c.cntB) + sg.step;
                __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __syncthreads();
    }
}

__global__ void zero_ints(int *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

}  // namespace sparc

using namespace sparc;

struct sparc_batch {
    int device = 0;
    int mode = 0;
    int njobs = 0;
    bool f32 = false, f64 = false;
    std::vector<sparc_batch_job> jobs;
    std::vector<BatchClusterDev> host_cl;
    std::vector<BatchSegment> segs;
    std::vector<long long> level_start;  // first item of each level (levelled mode), plus the end
    long long total = 0;
    BatchClusterDev *d_cl = nullptr;
    BatchSegment *d_seg = nullptr;
    int *d_ints = nullptr;  // ticket, abort, then all counters
    long long nints = 0;
    double *d_coef = nullptr;
    void *d_work = nullptr;  // per-cluster W and gather partials
    int grid = 0;
    hipStream_t cap = nullptr;  // capture stream (the null stream cannot be captured)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // mode 5: the batch's streams, one join event each plus the start event,
    // and the stream of every job
    hipStream_t lane[kBatchLanes] = {};
    hipEvent_t lane_ev[kBatchLanes + 1] = {};
    std::vector<int> lane_of;
};

namespace {

int batch_enqueue(sparc_batch *b, hipStream_t s)
{
    BatchArgs a;
    a.cl = b->d_cl;
    a.seg = b->d_seg;
    a.nseg = (int)b->segs.size();
    a.total = b->total;
    a.ticket = (unsigned int *)b->d_ints;
    a.abort = b->d_ints + 1;
    a.spin_limit = 1LL << 22;
    hipLaunchKernelGGL(zero_ints, dim3((unsigned)std::min<long long>(1024, (b->nints + 255) / 256)), dim3(256), 0, s,
                       b->d_ints, b->nints);
    if (b->mode == 2 || b->mode == 4) {
        a.waits = 0;
        for (size_t L = 0; L + 1 < b->level_start.size(); ++L) {
            const long long n = b->level_start[L + 1] - b->level_start[L];
            if (n <= 0) continue;
            a.base = b->level_start[L];
            a.total = b->level_start[L + 1];
            if (b->f32 && b->f64)
                hipLaunchKernelGGL((batch_kernel<true, true>), dim3((unsigned)n), dim3(kBatchNT), 0, s, a);
            else if (b->f64)
                hipLaunchKernelGGL((batch_kernel<false, true>), dim3((unsigned)n), dim3(kBatchNT), 0, s, a);
            else
                hipLaunchKernelGGL((batch_kernel<true, false>), dim3((unsigned)n), dim3(kBatchNT), 0, s, a);
        }
    } else {
        a.waits = 1;
        a.base = 0;
        if (b->f32 && b->f64)
            hipLaunchKernelGGL((batch_kernel<true, true>), dim3(b->grid), dim3(kBatchNT), 0, s, a);
        else if (b->f64)
            hipLaunchKernelGGL((batch_kernel<false, true>), dim3(b->grid), dim3(kBatchNT), 0, s, a);
        else
            hipLaunchKernelGGL((batch_kernel<true, false>), dim3(b->grid), dim3(kBatchNT), 0, s, a);
    }
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

}  // namespace

extern "C" {

int sparc_batch_create(const sparc_batch_job *jobs, int32_t njobs, int32_t mode, sparc_batch **out)
{
    if (!jobs || njobs < 1 || !out || mode < 0 || mode > 5) return fail(SPARC_E_ARG, "bad batch arguments");
    *out = nullptr;
    sparc_batch *b = new (std::nothrow) sparc_batch();
    if (!b) return fail(SPARC_E_NOMEM, "host allocation failed");
    auto cleanup = [&](int st) {
        sparc_batch_destroy(b);
        return st;
    };
    (void)hipGetDevice(&b->device);
    b->mode = mode;
    b->njobs = njobs;
    b->jobs.assign(jobs, jobs + njobs);
    // validate and size the per-cluster workspaces
    size_t work = 0;
    std::vector<size_t> woff(njobs), goff(njobs);
    int maxm = 0;
    for (int i = 0; i < njobs; ++i) {
        const sparc_batch_job &j = jobs[i];
        if (!j.op || !j.X || !j.Y || j.ns < 1 || (j.dtype != SPARC_F64 && j.dtype != SPARC_F32))
            return cleanup(fail(SPARC_E_ARG, "job " + std::to_string(i) + ": bad arguments"));
        if (j.m < 1 || !(j.a0 < j.a && j.a < j.b))
            return cleanup(fail(SPARC_E_BOUNDS, "job " + std::to_string(i) + ": bad degree or bounds"));
        if (j.ldx < j.op->nd || j.ldy < j.op->nd)
            return cleanup(fail(SPARC_E_SHAPE, "job " + std::to_string(i) + ": leading dimension below N_d"));
        if (j.op->device != b->device) return cleanup(fail(SPARC_E_ARG, "ops of a batch must live on one device"));
        // per job: gather partials then the extra block, the layout sparc_cheb_filter expects
        const size_t es = elem_size(j.dtype);
        goff[i] = work;
        work += gather_bytes(j.op, j.dtype, j.ns);
        woff[i] = work;
        work += align_up((size_t)j.op->nd * j.ns * es);
        maxm = std::max(maxm, j.m);
        (j.dtype == SPARC_F32 ? b->f32 : b->f64) = true;
    }
    if (hipMalloc(&b->d_work, std::max<size_t>(work, 256)) != hipSuccess)
        return cleanup(fail(SPARC_E_NOMEM, "device allocation of batch workspaces failed"));
    // counters: ticket, abort, then cntA and cntB per cluster and step
    b->nints = 2;
    std::vector<long long> cnt_off(njobs);
    for (int i = 0; i < njobs; ++i) {
        cnt_off[i] = b->nints;
        b->nints += 2LL * jobs[i].m;
    }
    long long ncoef = 0;
    for (int i = 0; i < njobs; ++i) ncoef += 3LL * jobs[i].m;
    if (hipMalloc(&b->d_ints, b->nints * sizeof(int)) != hipSuccess ||
        hipMalloc(&b->d_coef, ncoef * sizeof(double)) != hipSuccess)
        return cleanup(fail(SPARC_E_NOMEM, "device allocation of batch counters failed"));
    // the abort flag reads zero also in the modes that never reset it
    if (hipMemset(b->d_ints, 0, b->nints * sizeof(int)) != hipSuccess)
        return cleanup(fail(SPARC_E_HIP, "clearing the batch counters failed"));
    std::vector<double> coef(ncoef);
    long long cpos = 0;
    b->host_cl.resize(njobs);
    for (int i = 0; i < njobs; ++i) {
        const sparc_batch_job &j = jobs[i];
        const sparc_op *op = j.op;
        BatchClusterDev &c = b->host_cl[i];
        std::memset(&c, 0, sizeof(c));
        const bool f64 = j.dtype == SPARC_F64;
        c.veff = f64 ? (const void *)op->d_veff64 : (const void *)op->d_veff32;
        c.chi = f64 ? (const void *)op->d_chi64 : (const void *)op->d_chi32;
        c.hg = f64 ? (const void *)op->d_hg64 : (const void *)op->d_hg32;
        c.atoms = op->d_atoms;
        c.box_off = op->d_box_off;
        c.blk_pt = op->d_nl_blk_pt;
        c.blk_at = op->d_nl_blk_at;
        c.blk_atoms = op->d_nl_blk_atoms;
        c.pts = op->d_nl_pts;
        c.ent_off = op->d_nl_off;
        c.ent = (const int4 *)op->d_nl_ent;
        c.natoms = op->natoms;
        c.nproj_total = op->nproj_total;
        c.nl_nblk = op->nl_nblk;
        c.n1 = op->n[0];
        c.n2 = op->n[1];
        c.n3 = op->n[2];
        c.dtype = j.dtype;
        c.ns = j.ns;
        c.m = j.m;
        char *W = (char *)b->d_work + woff[i];
        c.X = j.X;
        c.ldx = j.ldx;
        const bool odd = (j.m & 1) != 0;
        c.P = odd ? j.Y : (void *)W;
        c.Q = odd ? (void *)W : j.Y;
        c.ldp = odd ? j.ldy : op->nd;
        c.ldq = odd ? op->nd : j.ldy;
        c.G = (char *)b->d_work + goff[i];
        // stencil geometry: the dtype's 256-thread vector patch and the
        // standalone filter's x split for it
        if (mode != 3 && mode != 5) {
            const FLaunch V = choose_vec_launch(op, j.dtype, j.ns, {j.ldx, j.ldy, op->nd});
            if (V.plan < 0)
                return cleanup(fail(SPARC_E_SHAPE, "job " + std::to_string(i) +
                                                       ": batched modes need the vector step kernels (z extent and "
                                                       "leading dimensions multiples of 4 FP32 / 2 FP64 values)"));
            const FLaunch B = V.plan == kBatchPlan[j.dtype] ? V : vec_launch_plan(op, j.dtype, j.ns, kBatchPlan[j.dtype]);
            const int ty = kPlanTY[B.plan];
            c.tiles_y = (c.n2 + ty - 1) / ty;
            c.tiles_z = (c.n3 + 31) / 32;
            c.chunk_x = B.chunk_x;
            c.nchunks = B.nchunks;
        } else {
            c.tiles_y = c.tiles_z = c.chunk_x = c.nchunks = 1;
        }
        c.ncb = (j.ns + 15) / 16;
        c.ncg = (j.ns + kScatterCols - 1) / kScatterCols;
        const long long nS = (long long)c.tiles_y * c.tiles_z * c.nchunks * ((j.ns + kBatchColGroup - 1) / kBatchColGroup);
        const long long nG = op->natoms > 0 ? (long long)op->natoms * kGatherSplit : 0;
        const long long nC = op->natoms > 0 ? (long long)op->nl_nblk : 0;
        if (nS > 0x7fffffffLL || nG > 0x7fffffffLL || nC > 0x7fffffffLL)
            return cleanup(fail(SPARC_E_SHAPE, "job " + std::to_string(i) + ": too many work items"));
        c.nS = (int)nS;
        c.nG = (int)nG;
        c.nC = (int)nC;
        c.c0 = -3.0 * op->w[0];
        for (int p = 1; p <= kMaxRadius; ++p) c.cp[p - 1] = -0.5 * op->w[p];
        // recurrence coefficients (FP64)
        const double e = 0.5 * (j.b - j.a), cc = 0.5 * (j.b + j.a);
        const double sigma1 = e / (j.a0 - cc), tau = 2.0 / sigma1;
        double sigma = sigma1;
        c.coef = b->d_coef + cpos;
        for (int k = 0; k < j.m; ++k) {
            double al, be;
            if (k == 0) {
                al = sigma1 / e;
                be = 0.0;
            } else {
                const double sn = 1.0 / (tau - sigma);
                al = 2.0 * sn / e;
                be = sigma * sn;
                sigma = sn;
            }
            coef[cpos + 3 * k] = al;
            coef[cpos + 3 * k + 1] = be;
            coef[cpos + 3 * k + 2] = cc;
        }
        cpos += 3LL * j.m;
        c.cntA = b->d_ints + cnt_off[i];
        c.cntB = c.cntA + j.m;
    }
    // level-ordered segments
    b->total = 0;
    for (int L = 0; L < 2 * maxm; ++L) {
        b->level_start.push_back(b->total);
        const int k = L / 2, kind = L % 2;
        for (int i = 0; i < njobs; ++i) {
            const BatchClusterDev &c = b->host_cl[i];
            if (k >= c.m) continue;
            const long long cnt = kind == 0 ? (long long)c.nG + c.nS : c.nC;
            if (cnt == 0) continue;
            b->segs.push_back({b->total, i, kind, k, (int)cnt});
            b->total += cnt;
        }
    }
    b->level_start.push_back(b->total);
    if (hipMalloc(&b->d_cl, njobs * sizeof(BatchClusterDev)) != hipSuccess ||
        hipMalloc(&b->d_seg, std::max<size_t>(1, b->segs.size()) * sizeof(BatchSegment)) != hipSuccess)
        return cleanup(fail(SPARC_E_NOMEM, "device allocation of the batch schedule failed"));
    if (hipMemcpy(b->d_cl, b->host_cl.data(), njobs * sizeof(BatchClusterDev), hipMemcpyHostToDevice) ||
        hipMemcpy(b->d_seg, b->segs.data(), b->segs.size() * sizeof(BatchSegment), hipMemcpyHostToDevice) ||
        hipMemcpy(b->d_coef, coef.data(), ncoef * sizeof(double), hipMemcpyHostToDevice))
        return cleanup(fail(SPARC_E_HIP, "copy of the batch schedule failed"));
    // persistent grid: the resident workgroups of the whole device
    int cus = 0, per_cu = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    hipError_t oe;
    if (b->total > 0x7fffffffLL) return cleanup(fail(SPARC_E_SHAPE, "batch has too many work items"));
    if (b->f32 && b->f64)
        oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<true, true>, kBatchNT, 0);
    else if (b->f64)
        oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<false, true>, kBatchNT, 0);
    else
        oe = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel<true, false>, kBatchNT, 0);
    if (oe != hipSuccess || per_cu < 1) per_cu = 1;
    b->grid = std::max(1, cus * per_cu);
    if (mode == 5) {
        for (int l = 0; l < kBatchLanes; ++l)
            if (hipStreamCreateWithFlags(&b->lane[l], hipStreamNonBlocking) != hipSuccess)
                return cleanup(fail(SPARC_E_HIP, "stream creation failed"));
        for (int l = 0; l <= kBatchLanes; ++l)
            if (hipEventCreateWithFlags(&b->lane_ev[l], hipEventDisableTiming) != hipSuccess)
                return cleanup(fail(SPARC_E_HIP, "event creation failed"));
        // longest first to the least loaded stream (work ~ N_d N_s m bytes)
        std::vector<int> order(njobs);
        for (int i = 0; i < njobs; ++i) order[i] = i;
        auto cost = [&](int i) {
            return (double)jobs[i].op->nd * jobs[i].ns * jobs[i].m * elem_size(jobs[i].dtype);
        };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
        double load[kBatchLanes] = {};
        b->lane_of.assign(njobs, 0);
        for (int i : order) {
            int l = 0;
            for (int q = 1; q < kBatchLanes; ++q)
                if (load[q] < load[l]) l = q;
            b->lane_of[i] = l;
            load[l] += cost(i);
        }
    }
    *out = b;
    return SPARC_OK;
}

int sparc_batch_run(sparc_batch *b, void *stream)
{
    if (!b) return fail(SPARC_E_ARG, "batch is NULL");
    TraceRange trace("sparc_batch_run");
    hipStream_t s = (hipStream_t)stream;
    if (b->mode == 5) {
        // the batch's streams start after the caller's stream's earlier work
        // and the caller's stream waits for all of them
        SPARC_HIP(hipEventRecord(b->lane_ev[kBatchLanes], s));
        for (int l = 0; l < kBatchLanes; ++l) SPARC_HIP(hipStreamWaitEvent(b->lane[l], b->lane_ev[kBatchLanes], 0));
        int st = SPARC_OK;
        for (int i = 0; i < b->njobs && !st; ++i) {
            const sparc_batch_job &j = b->jobs[i];
            const size_t need = sparc_workspace_bytes(j.op, j.dtype, j.ns, 1);
            st = sparc_cheb_filter(j.op, j.dtype, j.X, j.ldx, j.Y, j.ldy, j.ns, j.m, j.a0, j.a, j.b, b->host_cl[i].G,
                                   need, b->lane[b->lane_of[i]]);
        }
        // join every stream, also after a failed submission
        for (int l = 0; l < kBatchLanes; ++l) {
            if (hipEventRecord(b->lane_ev[l], b->lane[l]) != hipSuccess ||
                hipStreamWaitEvent(s, b->lane_ev[l], 0) != hipSuccess)
                if (!st) st = fail(SPARC_E_HIP, "joining the batch streams failed");
        }
        return st;
    }
    if (b->mode == 3) {
        // reference: the plain filters one after another on the stream
        for (int i = 0; i < b->njobs; ++i) {
            const sparc_batch_job &j = b->jobs[i];
            const size_t need = sparc_workspace_bytes(j.op, j.dtype, j.ns, 1);
            const int st = sparc_cheb_filter(j.op, j.dtype, j.X, j.ldx, j.Y, j.ldy, j.ns, j.m, j.a0, j.a, j.b,
                                             b->host_cl[i].G, need, stream);
            if (st) return st;
        }
        return SPARC_OK;
    }
    if (b->mode == 0 || b->mode == 4) {
        if (!b->exec) {
            // capture once on the batch's own stream; the graph holds the
            // counter reset (a kernel, no memset node) and the persistent kernel
            if (!b->cap) SPARC_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
            SPARC_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
            int st = batch_enqueue(b, b->cap);
            hipGraph_t g = nullptr;
            hipError_t ce = hipStreamEndCapture(b->cap, &g);
            if (st) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (ce != hipSuccess) return fail(SPARC_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(ce));
            b->graph = g;
            SPARC_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
        }
        SPARC_HIP(hipGraphLaunch(b->exec, s));
        return SPARC_OK;
    }
    return batch_enqueue(b, s);
}

int sparc_batch_check(sparc_batch *b, void *stream, int32_t *aborted)
{
    if (!b || !aborted) return fail(SPARC_E_ARG, "null argument");
    int v = 0;
    SPARC_HIP(hipMemcpyAsync(&v, b->d_ints + 1, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream));
    SPARC_HIP(hipStreamSynchronize((hipStream_t)stream));
    *aborted = v;
    if (v) return fail(SPARC_E_JOB, "batch aborted: a dependency wait exceeded its bound");
    return SPARC_OK;
}

int sparc_batch_info(const sparc_batch *b, int64_t *items, int32_t *levels, int32_t *grid)
{
    if (!b) return fail(SPARC_E_ARG, "batch is NULL");
    if (items) *items = b->total;
    if (levels) *levels = (int32_t)b->level_start.size() - 1;
    if (grid) *grid = b->grid;
    return SPARC_OK;
}

int sparc_batch_destroy(sparc_batch *b)
{
    if (!b) return SPARC_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int l = 0; l < kBatchLanes; ++l) {
        if (b->lane[l]) {
            (void)hipStreamSynchronize(b->lane[l]);
            (void)hipStreamDestroy(b->lane[l]);
        }
    }
    for (int l = 0; l <= kBatchLanes; ++l)
        if (b->lane_ev[l]) (void)hipEventDestroy(b->lane_ev[l]);
    (void)hipFree(b->d_cl);
    (void)hipFree(b->d_seg);
    (void)hipFree(b->d_ints);
    (void)hipFree(b->d_coef);
    (void)hipFree(b->d_work);
    delete b;
    return SPARC_OK;
}

}  // extern "C"
