// Internal declarations of the Chebyshev-filter library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sparc_filter.h"

namespace sparc {

constexpr int kMaxRadius = 6;    // largest stencil half-width n_o supported
constexpr int kMaxProj = 16;     // largest projector count per atom
constexpr int kBlock = 256;      // threads per workgroup of the stencil kernels
constexpr int kGatherSplit = 8;  // workgroups sharing one atom's cube points in the gather
constexpr int kScatterSlots = 32;  // most atoms one scatter block may touch
constexpr double kStreamBytes = 256.0 * 1024 * 1024;  // last-level cache of the chip

// Per-atom record used by the device kernels.
struct AtomDev {
    int lo[3];
    int ext[3];
    int nproj;
    int proj0;        // index of the atom's first projector in the global projector list
    int box0;         // offset of the atom's cube in the cube-point offset table
    long long chi0;   // offset of the atom's chi block (nproj * nbox values)
};

// Patches of the vector step kernels: TY x TZ nodes in (y, z) per plan
constexpr int kNumPlans = 10;
constexpr int kPlanTY[kNumPlans] = {8, 16, 32, 64, 8, 16, 32, 24, 32, 24};
constexpr int kPlanTZ[kNumPlans] = {32, 32, 32, 32, 64, 64, 64, 160, 80, 64};

// Tile shapes of the fused step kernel: a workgroup of nt threads owns a
// TY x TZ patch of the (y, z) plane and streams it along x.  TZ lanes run
// along z; each thread owns RY consecutive rows of y.
struct TileShape {
    int tz, ry, nt;
    int ty() const { return ry * (nt / tz); }
};
constexpr int kNumShapes = 2;
extern const TileShape kShapes[kNumShapes];

}  // namespace sparc

struct sparc_op {
    int device = 0;
    int n[3] = {0, 0, 0};
    double h = 0;
    int radius = 0;
    int64_t nd = 0;
    double w[sparc::kMaxRadius + 1] = {0};  // Laplacian weights w_0..w_radius (zero beyond)
    double vmax = 0;
    double *d_veff64 = nullptr;
    float *d_veff32 = nullptr;
    int natoms = 0;
    int nproj_total = 0;
    int max_nproj = 0;
    std::vector<sparc::AtomDev> atoms;
    std::vector<double> gamma;      // per global projector
    std::vector<double> chi_trace;  // per atom: trace(chi^T chi)
    std::vector<double> atom_gmax;  // per atom: max gamma
    sparc::AtomDev *d_atoms = nullptr;
    double *d_chi64 = nullptr;
    float *d_chi32 = nullptr;
    double *d_hg64 = nullptr;  // h^3 gamma per global projector
    float *d_hg32 = nullptr;
    int *d_box_off = nullptr;  // grid index of every cube point (atoms back to back)
    // unique nodes covered by at least one projector cube, their entries
    // (chi index of projector 0, cube size, block slot, nproj) and the
    // scatter blocks (node ranges and the atoms each touches)
    int nl_npts = 0;
    int nl_nblk = 0;
    int nl_max_slots = 0;  // most atoms one scatter block touches
    int *d_nl_pts = nullptr;
    int *d_nl_off = nullptr;
    int *d_nl_ent = nullptr;  // int4 records
    int *d_nl_blk_pt = nullptr;
    int *d_nl_blk_at = nullptr;
    int *d_nl_blk_atoms = nullptr;
    // launch overrides (set by sparc_op_set_launch; -1 / 0 = library choice)
    int tune_shape[2] = {-1, -1};
    int tune_chunk[2] = {0, 0};
    int tune_ns[2] = {-1, -1};  // block width the launch choice was tuned for; -1: every width
    int tune_group[2] = {0, 0};  // column group of the vector step (0 = library choice)
    int tune_cblk[2] = {0, 0};   // columns per workgroup of the vector step (0 = library choice)
    // nonlocal-force tables, built on the first sparc_nonlocal_force call:
    // per atom four gather records (the cube with chi, and for each axis d
    // the cube widened by the stencil radius along d with -grad_d chi), their
    // grid offsets and function values (FP64), and gamma per projector
    mutable std::mutex force_mu;
    mutable bool force_ready = false;
    mutable sparc::AtomDev *d_fatoms = nullptr;
    mutable int *d_fbox_off = nullptr;
    mutable double *d_ffun = nullptr;
    mutable double *d_fgamma = nullptr;
};

namespace sparc {

// thread-local error message
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define SPARC_HIP(call)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::sparc::fail(SPARC_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_size(int dtype);
inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// Launch parameters of one fused step: out = alpha*((H - shift) yk) - beta*yprev
struct StepCoef {
    double alpha, beta, shift;
    int has_prev;
};

// launch override of the op for a block of ns columns of the given dtype
inline bool tune_applies(const sparc_op *op, int dtype, int ns) { return op->tune_ns[dtype] < 0 || op->tune_ns[dtype] == ns; }

struct StepLaunch {
    int shape;     // index into kShapes
    int chunk_x;   // planes per workgroup along x (>= 1)
};

StepLaunch choose_step_launch(const sparc_op *op, int dtype, int ns);
// launch of the FP64 step on an FP32 block (launch_step_f32_to_f64)
StepLaunch choose_mixed_launch(const sparc_op *op, int ns);

// bytes of the gather's partial projections for ns columns
inline size_t gather_bytes(const sparc_op *op, int dtype, int ns)
{
    return align_up((size_t)kGatherSplit * (op->nproj_total > 0 ? op->nproj_total : 1) * ns *
                    (dtype == SPARC_F64 ? 8 : 4));
}

// Launch of the vector step kernels (fstep.hip): patch height TY =
// kPlanTY[plan], x split and column group.  plan < 0: the grid or a leading
// dimension rules the vector kernels out.
struct FLaunch {
    int plan = -1;
    int chunk_x = 0, nchunks = 0;
    int cgroup = 1;  // column blocks of one patch on consecutive workgroups
    int cblk = 1;    // columns per workgroup (1 or 2: orbital blocking)
};
constexpr int kMaxChunks = 16;  // most x-chunks of a vector step launch

// is plan a patch height offered for dtype
bool vec_plan_valid(int dtype, int plan);
int vec_max_cblk(int dtype, int plan);  // columns per workgroup the plan's patch can hold (1 or 2)
// vector launch for a block of ns columns whose leading dimensions are lds
FLaunch choose_vec_launch(const sparc_op *op, int dtype, int ns, std::initializer_list<int64_t> lds);
// the default x split of patch height `plan` (no tuning applied)
FLaunch vec_launch_plan(const sparc_op *op, int dtype, int ns, int plan);
// enqueue a vector step; with part (and atoms) the same launch gathers the
// projections of yk into part (the standalone gather's layout)
int launch_fstep(const sparc_op *op, int dtype, const FLaunch &L, const void *yk, int64_t ldk, const void *yprev,
                 int64_t ldp, void *out, int64_t ldo, int ns, void *part, const StepCoef &c, hipStream_t stream);

// enqueue the projector gather: split partial sums of chi_Jp^T Y(:,c) per atom
int launch_gather(const sparc_op *op, int dtype, const void *Y, int64_t ldy, int ns, void *part,
                  hipStream_t stream);

// enqueue the projector scatter: out += alpha * V_nl Y from the gathered partials
int launch_scatter(const sparc_op *op, int dtype, void *out, int64_t ldo, int ns, const void *part, double alpha,
                   hipStream_t stream);

// enqueue one fused stencil / potential / recurrence step (local part of H)
int launch_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                void *out, int64_t ldo, int ns, const StepCoef &c, const StepLaunch &L, hipStream_t stream);

// H applied in FP64 to an FP32 block (values widened on load): the
// projector gather and the local step of the Rayleigh-Ritz product H Y
int launch_gather_f32_to_f64(const sparc_op *op, const float *Y, int64_t ldy, int ns, double *part,
                             hipStream_t stream);
int launch_step_f32_to_f64(const sparc_op *op, const float *yk, int64_t ldk, double *out, int64_t ldo, int ns,
                           const StepCoef &c, const StepLaunch &L, hipStream_t stream);

// One launch for one FP64 vector v (N_d values, contiguous): out = H_loc v,
// dot[b] = sum over workgroup b's points of v(x) (H_loc v)(x) for
// b < step_dot_blocks(op), and the projector gather of v into part (as
// launch_gather with ns = 1); the scatter follows separately
long long step_dot_blocks(const sparc_op *op);
int launch_lanczos_h_f64(const sparc_op *op, const double *v, double *out, double *dot, double *part,
                         hipStream_t stream);

// the projector gather of yk into part and the local step in one launch
int launch_step_gather(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                       void *out, int64_t ldo, int ns, void *part, const StepCoef &c, const StepLaunch &L,
                       hipStream_t stream);

// the full operator step: gather(yk) and the local step in one launch (the
// vector kernels when V is given and usable, else the scalar ones), then the
// scatter(alpha)
int launch_h_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                  void *out, int64_t ldo, int ns, void *part, const StepCoef &c, const StepLaunch &L,
                  hipStream_t stream, const FLaunch *V = nullptr);

// small generalized eigensolver (n <= 64) in one workgroup: theta ascending,
// evec column-major and M-orthonormal; info = 0 or the failing Cholesky column
int launch_small_sygv(const double *Hs, const double *Ms, int n, double *theta, double *evec, int *info,
                      hipStream_t stream);

// true when the last sparc_rayleigh_ritz of this thread failed because the
// Cholesky factorisation of M_s broke down (rank-deficient filtered block)
extern thread_local bool g_rr_rank_deficient;

// buffers of the CheFSI passes: the filtered block Y (ldy), the filter's
// workspace, the Rayleigh-Ritz workspace, the ns x ns eigenvectors, the
// rotation's workspace and ns device doubles for the occupations
struct ChefsiBuffers {
    void *Y;
    int64_t ldy;
    void *fws;
    size_t fws_bytes;
    void *rr;
    size_t rr_bytes;
    double *evec;
    void *rot;
    size_t rot_bytes;
    double *occ;
};

// `passes` CheFSI passes on X in place (filter, Rayleigh-Ritz, Fermi level,
// rotation); the cutoff of every pass after the first is the previous Fermi
// level + 0.1 Ha; a pass whose block turns out rank deficient is redone at
// half the degree.  a0: in, the lambda_1 estimate; out, lowered to a pass's
// lowest Ritz value where a cutoff fell at or below it.  theta (passes x ns),
// lambda_f, degrees: host outputs (may be null); rho: device density of the
// final block (may be null); halvings: number of degree halvings (may be
// null).  Synchronous.
int chefsi_run(const sparc_op *op, int dtype, void *X, int64_t ldx, int ns, int m, int passes, double ne, double kT,
               double &a0, double a, double b, const ChefsiBuffers &B, double *theta, double *lambda_f,
               int32_t *degrees, double *rho, hipStream_t s, int *halvings);

// roctx range over the host side of an entry point or a step of it, for
// timelines that show the library's phases beside its kernels (rocprofv3
// --marker-trace); without a tool that records markers it costs a call
struct TraceRange {
    explicit TraceRange(const char *name);
    ~TraceRange();
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// profiling hooks (no-ops unless enabled)
struct ProfScope {
    int kernel;
    hipStream_t stream;
    void *ev0 = nullptr;
    ProfScope(int kernel, hipStream_t s);
    ~ProfScope();
};

}  // namespace sparc
