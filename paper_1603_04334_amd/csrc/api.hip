// C ABI of the Chebyshev-filter library: operator construction, H application,
// the filter driver, status strings and per-kernel event timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "internal.hpp"

namespace sparc {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int status, const std::string &msg)
{
    set_error(msg);
    return status;
}

size_t elem_size(int dtype) { return dtype == SPARC_F64 ? sizeof(double) : sizeof(float); }

// ---------------------------------------------------------------- profiling

namespace {
struct ProfRec {
    int kernel;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
constexpr int kProfKernels = 8;
int64_t g_prof_count[kProfKernels] = {};
double g_prof_ms[kProfKernels] = {};
}  // namespace

TraceRange::TraceRange(const char *name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

ProfScope::ProfScope(int k, hipStream_t s) : kernel(k), stream(s)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, stream);
    ev0 = e;
}

ProfScope::~ProfScope()
{
    if (!ev0) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipEventDestroy((hipEvent_t)ev0);
        return;
    }
    (void)hipEventRecord(e, stream);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({kernel, (hipEvent_t)ev0, e});
}

// ---------------------------------------------------------------- weights

// Laplacian weights of Sec. 3.1 Eq. weightsLap.  The factorial ratio
// (n_o!)^2 / ((n_o-p)!(n_o+p)!) is accumulated as a product of p factors
// (n_o-p+i)/(n_o+i), i = 1..p.
static void laplacian_weights(int no, double h, double *w)
{
    double inv_h2 = 1.0 / (h * h);
    double s = 0.0;
    for (int q = no; q >= 1; --q) s += 1.0 / (double(q) * q);
    w[0] = -s * inv_h2;
    for (int p = 1; p <= no; ++p) {
        double ratio = 1.0;
        for (int i = 1; i <= p; ++i) ratio *= double(no - p + i) / double(no + i);
        double sign = (p & 1) ? 1.0 : -1.0;
        w[p] = 2.0 * sign * ratio / (double(p) * p) * inv_h2;
    }
    for (int p = no + 1; p <= kMaxRadius; ++p) w[p] = 0.0;
}

static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

static size_t block_bytes(int64_t nd, int64_t ld, int ns, int dtype)
{
    return (size_t)((int64_t)(ns - 1) * ld + nd) * elem_size(dtype);
}

static int check_block(const sparc_op *op, const void *p, int64_t ld, int ns, const char *name)
{
    if (!p) return fail(SPARC_E_ARG, std::string(name) + " is NULL");
    if (ns < 1) return fail(SPARC_E_SHAPE, "ns must be >= 1");
    if (ld < op->nd) return fail(SPARC_E_SHAPE, std::string("leading dimension of ") + name + " is below N_d");
    return SPARC_OK;
}

int launch_h_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                  void *out, int64_t ldo, int ns, void *part, const StepCoef &c, const StepLaunch &L,
                  hipStream_t stream, const FLaunch *V)
{
    int st;
    if (V && V->plan >= 0)
        st = launch_fstep(op, dtype, *V, yk, ldk, yprev, ldp, out, ldo, ns, part, c, stream);
    else
        st = launch_step_gather(op, dtype, yk, ldk, yprev, ldp, out, ldo, ns, part, c, L, stream);
    if (st) return st;
    return launch_scatter(op, dtype, out, ldo, ns, part, c.alpha, stream);
}

}  // namespace sparc

using namespace sparc;

extern "C" {

const char *sparc_status_str(int s)
{
    switch (s) {
        case SPARC_OK: return "ok";
        case SPARC_PENDING: return "pending";
        case SPARC_E_ARG: return "invalid argument";
        case SPARC_E_SHAPE: return "inconsistent shape";
        case SPARC_E_BOUNDS: return "invalid filter bounds or degree";
        case SPARC_E_NOMEM: return "out of device memory";
        case SPARC_E_HIP: return "HIP runtime error";
        case SPARC_E_BUSY: return "reserved";
        case SPARC_E_TICKET: return "unknown ticket";
        case SPARC_E_JOB: return "job failed";
        case SPARC_E_WORKSPACE: return "workspace missing or too small";
        case SPARC_E_BREAKDOWN: return "numerical breakdown (Lanczos invariant subspace or singular M_s)";
        case SPARC_E_ALIAS: return "overlapping buffers";
    }
    return "unknown status";
}

const char *sparc_last_error(void) { return g_last_error.c_str(); }

int sparc_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return SPARC_OK;
}

int sparc_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_pending) {
        (void)hipEventSynchronize(r.b);
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    for (int k = 0; k < kProfKernels; ++k) {
        g_prof_count[k] = 0;
        g_prof_ms[k] = 0;
    }
    return SPARC_OK;
}

int sparc_profile_read(int32_t kernel, int64_t *launches, double *total_ms)
{
    if (kernel < 0 || kernel >= kProfKernels) return fail(SPARC_E_ARG, "kernel id must be 0..7");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof_pending) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(SPARC_E_HIP, "event synchronisation failed");
        float ms = 0;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        g_prof_count[r.kernel] += 1;
        g_prof_ms[r.kernel] += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
    if (launches) *launches = g_prof_count[kernel];
    if (total_ms) *total_ms = g_prof_ms[kernel];
    return SPARC_OK;
}

int sparc_op_create(const sparc_grid *grid, const double *veff, int32_t natoms, const sparc_atom *atoms,
                    sparc_op **out)
{
    if (!grid || !veff || !out || natoms < 0 || (natoms > 0 && !atoms))
        return fail(SPARC_E_ARG, "null argument or negative atom count");
    *out = nullptr;
    for (int d = 0; d < 3; ++d)
        if (grid->n[d] < 1) return fail(SPARC_E_SHAPE, "grid extents must be >= 1");
    if (!(grid->h > 0)) return fail(SPARC_E_SHAPE, "grid spacing must be > 0");
    if (grid->radius < 1 || grid->radius > kMaxRadius) return fail(SPARC_E_SHAPE, "radius must be in 1..6");
    // one FP64 plane must stay below 2 GiB (32-bit in-plane byte offsets in the kernels)
    const int64_t plane = (int64_t)grid->n[1] * grid->n[2];
    if (plane >= (1LL << 28)) return fail(SPARC_E_SHAPE, "n[1]*n[2] must be below 2^28");
    const int64_t nd_all = (int64_t)grid->n[0] * plane;

    sparc_op *op = new (std::nothrow) sparc_op();
    if (!op) return fail(SPARC_E_NOMEM, "host allocation failed");
    auto cleanup = [&](int st) {
        sparc_op_destroy(op);
        return st;
    };
    (void)hipGetDevice(&op->device);
    for (int d = 0; d < 3; ++d) op->n[d] = grid->n[d];
    op->h = grid->h;
    op->radius = grid->radius;
    op->nd = nd_all;
    laplacian_weights(op->radius, op->h, op->w);

    const int64_t nd = op->nd;
    op->vmax = -INFINITY;
    std::vector<float> v32(nd);
    for (int64_t i = 0; i < nd; ++i) {
        op->vmax = std::max(op->vmax, veff[i]);
        v32[i] = (float)veff[i];
    }
    if (hipMalloc(&op->d_veff64, nd * sizeof(double)) != hipSuccess ||
        hipMalloc(&op->d_veff32, nd * sizeof(float)) != hipSuccess)
        return cleanup(fail(SPARC_E_NOMEM, "device allocation of V_eff failed"));
    if (hipMemcpy(op->d_veff64, veff, nd * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(op->d_veff32, v32.data(), nd * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(SPARC_E_HIP, "copy of V_eff failed"));

    // atoms
    op->natoms = natoms;
    int64_t chi_total = 0, box_total = 0;
    for (int J = 0; J < natoms; ++J) {
        const sparc_atom &A = atoms[J];
        if (A.nproj < 1 || A.nproj > kMaxProj || !A.chi || !A.gamma)
            return cleanup(fail(SPARC_E_ARG, "atom " + std::to_string(J) + ": nproj outside 1..16 or null data"));
        for (int d = 0; d < 3; ++d)
            if (A.ext[d] < 1 || A.lo[d] < 0 || A.lo[d] + A.ext[d] > grid->n[d])
                return cleanup(fail(SPARC_E_SHAPE, "atom " + std::to_string(J) + ": projector cube outside the grid"));
        AtomDev a;
        for (int d = 0; d < 3; ++d) {
            a.lo[d] = A.lo[d];
            a.ext[d] = A.ext[d];
        }
        a.nproj = A.nproj;
        a.proj0 = op->nproj_total;
        a.chi0 = chi_total;
        const int64_t nbox = (int64_t)A.ext[0] * A.ext[1] * A.ext[2];
        a.box0 = (int)box_total;
        box_total += nbox;
        chi_total += nbox * A.nproj;
        op->nproj_total += A.nproj;
        op->max_nproj = std::max(op->max_nproj, A.nproj);
        op->atoms.push_back(a);
        double tr = 0, gmax = -INFINITY;
        for (int64_t i = 0; i < nbox * A.nproj; ++i) tr += A.chi[i] * A.chi[i];
        for (int p = 0; p < A.nproj; ++p) {
            op->gamma.push_back(A.gamma[p]);
            gmax = std::max(gmax, A.gamma[p]);
        }
        op->chi_trace.push_back(tr);
        op->atom_gmax.push_back(gmax);
    }
    if (natoms > 0) {
        std::vector<double> chi64(chi_total);
        std::vector<float> chi32(chi_total);
        for (int J = 0; J < natoms; ++J) {
            const sparc_atom &A = atoms[J];
            const int64_t cnt = (int64_t)A.ext[0] * A.ext[1] * A.ext[2] * A.nproj;
            std::memcpy(&chi64[op->atoms[J].chi0], A.chi, cnt * sizeof(double));
            for (int64_t i = 0; i < cnt; ++i) chi32[op->atoms[J].chi0 + i] = (float)A.chi[i];
        }
        const double h3 = op->h * op->h * op->h;
        std::vector<double> hg64(op->nproj_total);
        std::vector<float> hg32(op->nproj_total);
        for (int p = 0; p < op->nproj_total; ++p) {
            hg64[p] = h3 * op->gamma[p];
            hg32[p] = (float)hg64[p];
        }
        if (hipMalloc(&op->d_atoms, natoms * sizeof(AtomDev)) != hipSuccess ||
            hipMalloc(&op->d_chi64, chi_total * sizeof(double)) != hipSuccess ||
            hipMalloc(&op->d_chi32, chi_total * sizeof(float)) != hipSuccess ||
            hipMalloc(&op->d_hg64, op->nproj_total * sizeof(double)) != hipSuccess ||
            hipMalloc(&op->d_hg32, op->nproj_total * sizeof(float)) != hipSuccess)
            return cleanup(fail(SPARC_E_NOMEM, "device allocation of projector data failed"));
        if (hipMemcpy(op->d_atoms, op->atoms.data(), natoms * sizeof(AtomDev), hipMemcpyHostToDevice) ||
            hipMemcpy(op->d_chi64, chi64.data(), chi_total * sizeof(double), hipMemcpyHostToDevice) ||
            hipMemcpy(op->d_chi32, chi32.data(), chi_total * sizeof(float), hipMemcpyHostToDevice) ||
            hipMemcpy(op->d_hg64, hg64.data(), op->nproj_total * sizeof(double), hipMemcpyHostToDevice) ||
            hipMemcpy(op->d_hg32, hg32.data(), op->nproj_total * sizeof(float), hipMemcpyHostToDevice))
            return cleanup(fail(SPARC_E_HIP, "copy of projector data failed"));
    }

    // cube-point grid offsets and the unique covered nodes with their (atom, cube index) entries
    if (natoms > 0) {
        if (box_total > 0x7fffffffLL) return cleanup(fail(SPARC_E_SHAPE, "projector cubes too large"));
        std::vector<int> boff(box_total);
        std::vector<std::pair<int64_t, std::pair<int, int>>> cover;
        cover.reserve(box_total);
        for (int J = 0; J < natoms; ++J) {
            const AtomDev &a = op->atoms[J];
            int loc = 0;
            for (int i = 0; i < a.ext[0]; ++i)
                for (int j = 0; j < a.ext[1]; ++j)
                    for (int k = 0; k < a.ext[2]; ++k, ++loc) {
                        const int64_t g = (int64_t)(a.lo[2] + k) + (int64_t)op->n[2] * ((a.lo[1] + j) + (int64_t)op->n[1] * (a.lo[0] + i));
                        boff[a.box0 + loc] = (int)g;
                        cover.push_back({g, {J, loc}});
                    }
        }
        std::stable_sort(cover.begin(), cover.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        // unique nodes and their (atom, cube index) entries
        std::vector<int> pts, off;
        std::vector<std::pair<int, int>> raw;
        for (size_t e = 0; e < cover.size(); ++e) {
            if (e == 0 || cover[e].first != cover[e - 1].first) {
                pts.push_back((int)cover[e].first);
                off.push_back((int)e);
            }
            raw.push_back(cover[e].second);
        }
        off.push_back((int)cover.size());
        // scatter blocks: at most kBlock nodes touching at most kScatterSlots atoms
        std::vector<int> blk_pt{0}, blk_at{0}, blk_atoms, ent(4 * raw.size());
        std::vector<int> slot_of(natoms, -1);
        std::vector<int> cur;
        auto close_block = [&](int end_pt) {
            blk_pt.push_back(end_pt);
            op->nl_max_slots = std::max(op->nl_max_slots, (int)cur.size());
            for (int J : cur) {
                blk_atoms.push_back(J);
                slot_of[J] = -1;
            }
            blk_at.push_back((int)blk_atoms.size());
            cur.clear();
        };
        for (size_t pi = 0; pi < pts.size(); ++pi)
            if (off[pi + 1] - off[pi] > kScatterSlots)
                return cleanup(fail(SPARC_E_SHAPE, "more than 32 projector cubes overlap at one node"));
        for (size_t pi = 0; pi < pts.size(); ++pi) {
            int fresh = 0;
            for (int e = off[pi]; e < off[pi + 1]; ++e)
                if (slot_of[raw[e].first] < 0) ++fresh;
            const int in_block = (int)pi - blk_pt.back();
            if (in_block == kBlock || (int)cur.size() + fresh > kScatterSlots) close_block((int)pi);
            for (int e = off[pi]; e < off[pi + 1]; ++e) {
                const int J = raw[e].first;
                if (slot_of[J] < 0) {
                    slot_of[J] = (int)cur.size();
                    cur.push_back(J);
                }
                const AtomDev &a = op->atoms[J];
                const int nbox = a.ext[0] * a.ext[1] * a.ext[2];
                ent[4 * e + 0] = (int)(a.chi0 + raw[e].second);
                ent[4 * e + 1] = nbox;
                ent[4 * e + 2] = slot_of[J];
                ent[4 * e + 3] = a.nproj;
            }
        }
        close_block((int)pts.size());
        if (chi_total > 0x7fffffffLL) return cleanup(fail(SPARC_E_SHAPE, "projector data too large"));
        op->nl_npts = (int)pts.size();
        op->nl_nblk = (int)blk_pt.size() - 1;
        auto up = [&](int **dst, const std::vector<int> &v) {
            if (hipMalloc(dst, std::max<size_t>(1, v.size()) * sizeof(int)) != hipSuccess) return false;
            return v.empty() || hipMemcpy(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
        };
        if (!up(&op->d_box_off, boff) || !up(&op->d_nl_pts, pts) || !up(&op->d_nl_off, off) || !up(&op->d_nl_ent, ent) ||
            !up(&op->d_nl_blk_pt, blk_pt) || !up(&op->d_nl_blk_at, blk_at) || !up(&op->d_nl_blk_atoms, blk_atoms))
            return cleanup(fail(SPARC_E_NOMEM, "device allocation of projector tables failed"));
    }
    *out = op;
    return SPARC_OK;
}

int sparc_op_destroy(sparc_op *op)
{
    if (!op) return SPARC_OK;
    (void)hipFree(op->d_veff64);
    (void)hipFree(op->d_veff32);
    (void)hipFree(op->d_atoms);
    (void)hipFree(op->d_chi64);
    (void)hipFree(op->d_chi32);
    (void)hipFree(op->d_hg64);
    (void)hipFree(op->d_hg32);
    (void)hipFree(op->d_box_off);
    (void)hipFree(op->d_nl_pts);
    (void)hipFree(op->d_nl_off);
    (void)hipFree(op->d_nl_ent);
    (void)hipFree(op->d_nl_blk_pt);
    (void)hipFree(op->d_nl_blk_at);
    (void)hipFree(op->d_nl_blk_atoms);
    (void)hipFree(op->d_fatoms);
    (void)hipFree(op->d_fbox_off);
    (void)hipFree(op->d_ffun);
    (void)hipFree(op->d_fgamma);
    delete op;
    return SPARC_OK;
}

int64_t sparc_op_nd(const sparc_op *op) { return op ? op->nd : 0; }
int32_t sparc_op_nproj(const sparc_op *op) { return op ? op->nproj_total : 0; }

size_t sparc_workspace_bytes(const sparc_op *op, int32_t dtype, int32_t ns, int32_t which)
{
    if (!op || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32)) return 0;
    const size_t g = gather_bytes(op, dtype, ns);
    if (which == 0) return g;
    return g + align_up((size_t)op->nd * ns * elem_size(dtype));
}

int sparc_op_set_launch(sparc_op *op, int32_t dtype, int32_t tile_z, int32_t tile_y, int32_t chunk_x,
                        int32_t col_group, int32_t col_block)
{
    if (!op || (dtype != SPARC_F64 && dtype != SPARC_F32)) return fail(SPARC_E_ARG, "null op or bad dtype");
    if (col_block < 0 || col_block > 2) return fail(SPARC_E_ARG, "col_block must be 0, 1 or 2");
    if (tile_z <= 0 && tile_y <= 0) {
        op->tune_shape[dtype] = -1;
    } else {
        // patches of TY x TZ nodes offered for the dtype
        int found = -1;
        for (int p = 0; p < kNumPlans; ++p)
            if (kPlanTZ[p] == tile_z && kPlanTY[p] == tile_y && vec_plan_valid(dtype, p)) found = p;
        if (found < 0) return fail(SPARC_E_ARG, "unsupported tile shape");
        if (col_block == 2 && vec_max_cblk(dtype, found) < 2)
            return fail(SPARC_E_ARG, "this tile shape takes one column per workgroup");
        op->tune_shape[dtype] = found;
    }
    op->tune_chunk[dtype] = chunk_x > 0 ? chunk_x : 0;
    op->tune_group[dtype] = col_group > 0 ? col_group : 0;
    op->tune_cblk[dtype] = col_block;
    op->tune_ns[dtype] = -1;
    return SPARC_OK;
}

int sparc_step_config(const sparc_op *op, int32_t dtype, int32_t ns, int32_t *tile_z, int32_t *tile_y,
                      int32_t *chunk_x, int32_t *col_group, int32_t *col_block)
{
    if (!op || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32)) return fail(SPARC_E_ARG, "null op, ns < 1 or bad dtype");
    const FLaunch V = choose_vec_launch(op, dtype, ns, {});
    if (V.plan >= 0) {
        if (tile_z) *tile_z = kPlanTZ[V.plan];
        if (tile_y) *tile_y = kPlanTY[V.plan];
        if (chunk_x) *chunk_x = V.chunk_x;
        if (col_group) *col_group = std::min(V.cgroup, (ns + V.cblk - 1) / V.cblk);
        if (col_block) *col_block = V.cblk;
        return SPARC_OK;
    }
    StepLaunch L = choose_step_launch(op, dtype, ns);
    if (tile_z) *tile_z = kShapes[L.shape].tz;
    if (tile_y) *tile_y = kShapes[L.shape].ty();
    if (chunk_x) *chunk_x = L.chunk_x;
    if (col_group) *col_group = 1;
    if (col_block) *col_block = 1;
    return SPARC_OK;
}

int sparc_h_apply(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y, int64_t ldy, int32_t ns,
                  void *ws, size_t ws_bytes, void *stream)
{
    if (!op) return fail(SPARC_E_ARG, "op is NULL");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "dtype must be SPARC_F64 or SPARC_F32");
    int st;
    if ((st = check_block(op, X, ldx, ns, "X")) || (st = check_block(op, Y, ldy, ns, "Y"))) return st;
    const size_t need = sparc_workspace_bytes(op, dtype, ns, 0);
    if (op->natoms > 0 && (!ws || ws_bytes < need)) return fail(SPARC_E_WORKSPACE, "workspace too small");
    const size_t bx = block_bytes(op->nd, ldx, ns, dtype), by = block_bytes(op->nd, ldy, ns, dtype);
    if (overlaps(X, bx, Y, by) || overlaps(X, bx, ws, need) || overlaps(Y, by, ws, need))
        return fail(SPARC_E_ALIAS, "X, Y and the workspace must not overlap");
    hipStream_t s = (hipStream_t)stream;
    StepCoef c{1.0, 0.0, 0.0, 0};
    const FLaunch V = choose_vec_launch(op, dtype, ns, {ldx, ldy});
    StepLaunch L = choose_step_launch(op, dtype, ns);
    TraceRange trace("sparc_h_apply");
    return launch_h_step(op, dtype, X, ldx, nullptr, 0, Y, ldy, ns, ws, c, L, s, &V);
}

int sparc_cheb_filter(const sparc_op *op, int32_t dtype, const void *X, int64_t ldx, void *Y, int64_t ldy,
                      int32_t ns, int32_t m, double a0, double a, double b, void *ws, size_t ws_bytes, void *stream)
{
    if (!op) return fail(SPARC_E_ARG, "op is NULL");
    if (dtype != SPARC_F64 && dtype != SPARC_F32) return fail(SPARC_E_ARG, "dtype must be SPARC_F64 or SPARC_F32");
    if (m < 1) return fail(SPARC_E_BOUNDS, "degree m must be >= 1");
    if (!(a0 < a && a < b) || !std::isfinite(a0) || !std::isfinite(b))
        return fail(SPARC_E_BOUNDS, "filter bounds must satisfy a0 < a < b");
    int st;
    if ((st = check_block(op, X, ldx, ns, "X")) || (st = check_block(op, Y, ldy, ns, "Y"))) return st;
    const size_t need = sparc_workspace_bytes(op, dtype, ns, 1);
    if (!ws || ws_bytes < need) return fail(SPARC_E_WORKSPACE, "workspace too small");
    const size_t bx = block_bytes(op->nd, ldx, ns, dtype), by = block_bytes(op->nd, ldy, ns, dtype);
    if (overlaps(X, bx, Y, by) || overlaps(X, bx, ws, need) || overlaps(Y, by, ws, need))
        return fail(SPARC_E_ALIAS, "X, Y and the workspace must not overlap");

    TraceRange trace("sparc_cheb_filter");
    hipStream_t s = (hipStream_t)stream;
    char *G = (char *)ws;
    char *W = G + gather_bytes(op, dtype, ns);
    const int64_t ldw = op->nd;

    // Y_k is written to buffer P for odd k and Q for even k, so that Y_m
    // lands in Y; Y_{k+1} overwrites Y_{k-1} in place.
    void *P = (m & 1) ? Y : (void *)W;
    void *Q = (m & 1) ? (void *)W : Y;
    const int64_t ldP = (m & 1) ? ldy : ldw;
    const int64_t ldQ = (m & 1) ? ldw : ldy;

    const double e = 0.5 * (b - a);
    const double c = 0.5 * (b + a);
    const double sigma1 = e / (a0 - c);
    const double tau = 2.0 / sigma1;
    // one kernel family for every step of the filter
    const FLaunch V = choose_vec_launch(op, dtype, ns, {ldx, ldy, ldw});
    StepLaunch L = choose_step_launch(op, dtype, ns);

    // Y_1 = (sigma_1/e)(H - cI) X
    StepCoef c1{sigma1 / e, 0.0, c, 0};
    {
        TraceRange step("filter step");
        if ((st = launch_h_step(op, dtype, X, ldx, nullptr, 0, P, ldP, ns, G, c1, L, s, &V))) return st;
    }

    double sigma = sigma1;
    for (int k = 1; k < m; ++k) {
        const double sigma_next = 1.0 / (tau - sigma);
        const void *yk = (k & 1) ? P : Q;
        const int64_t ldk = (k & 1) ? ldP : ldQ;
        const void *yprev = (k == 1) ? X : ((k & 1) ? Q : P);
        const int64_t ldp = (k == 1) ? ldx : ((k & 1) ? ldQ : ldP);
        void *out = ((k + 1) & 1) ? P : Q;
        const int64_t ldo = ((k + 1) & 1) ? ldP : ldQ;
        StepCoef ck{2.0 * sigma_next / e, sigma * sigma_next, c, 1};
        TraceRange step("filter step");
        if ((st = launch_h_step(op, dtype, yk, ldk, yprev, ldp, out, ldo, ns, G, ck, L, s, &V))) return st;
        sigma = sigma_next;
    }
    return SPARC_OK;
}

int sparc_upper_bound(const sparc_op *op, double *ub)
{
    if (!op || !ub) return fail(SPARC_E_ARG, "null argument");
    // 1D symbol of -1/2 lap_h: s(t) = -w_0 - sum_p w_p cos(p t); maximise on a
    // fine grid and add the Lipschitz bound times the grid step.
    const int N = 20000;
    double smax = -INFINITY, lip = 0;
    for (int p = 1; p <= op->radius; ++p) lip += std::fabs(op->w[p]) * p;
    for (int i = 0; i <= N; ++i) {
        const double t = M_PI * i / N;
        double s = -op->w[0];
        for (int p = 1; p <= op->radius; ++p) s -= op->w[p] * std::cos(p * t);
        smax = std::max(smax, s);
    }
    smax += lip * (M_PI / N);
    double bound = 3.0 * smax + op->vmax;
    const double h3 = op->h * op->h * op->h;
    for (int J = 0; J < op->natoms; ++J)
        if (op->atom_gmax[J] > 0) bound += h3 * op->atom_gmax[J] * op->chi_trace[J];
    *ub = bound;
    return SPARC_OK;
}

int sparc_select_bounds(const double *theta, int32_t k, int32_t nwant, double shift, double bfactor, double ubound,
                        double *a0, double *a, double *b)
{
    if (!theta || k < 1 || nwant < 1 || !a0 || !a || !b) return fail(SPARC_E_ARG, "bad arguments");
    const int iw = std::min(nwant, k) - 1;
    double A0 = theta[0], A = theta[iw] + shift, B = bfactor * theta[k - 1];
    if (ubound > 0 && ubound < B) B = ubound;
    if (!(A0 < A && A < B)) return fail(SPARC_E_BOUNDS, "Ritz values give degenerate filter bounds");
    *a0 = A0;
    *a = A;
    *b = B;
    return SPARC_OK;
}

}  // extern "C"
