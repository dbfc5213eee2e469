// Internal declarations of the Chebyshev-filter library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sparc_filter.h"

namespace sparc {

constexpr int kMaxRadius = 6;    // largest stencil half-width n_o supported
constexpr int kMaxProj = 16;     // largest projector count per atom
constexpr int kBlock = 256;      // threads per workgroup of the stencil kernels

// Per-atom record used by the device kernels.
struct AtomDev {
    int lo[3];
    int ext[3];
    int nproj;
    int proj0;        // index of the atom's first projector in the global projector list
    long long chi0;   // offset of the atom's chi block (nproj * nbox values)
};

// Tile shapes of the fused step kernel: a workgroup owns a TY x TZ patch of
// the (y, z) plane and streams it along x.  TZ lanes run along z; each thread
// owns RY rows of y spaced 256/TZ apart.
struct TileShape {
    int tz, ry;
    int ty() const { return ry * (kBlock / tz); }
};
constexpr int kNumShapes = 4;
extern const TileShape kShapes[kNumShapes];

struct TileLists {
    int tiles_y = 0, tiles_z = 0;
    int *d_off = nullptr;   // tiles_y*tiles_z + 1 offsets into d_list
    int *d_list = nullptr;  // atom indices whose cube meets the tile's (y,z) footprint
};

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
    sparc::TileLists lists[sparc::kNumShapes];
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

struct StepLaunch {
    int shape;     // index into kShapes
    int chunk_x;   // planes per workgroup along x (>= 1)
};

StepLaunch choose_step_launch(const sparc_op *op, int dtype, int ns);

// enqueue the projector gather G[p][c] = h^3 gamma_p sum_x chi_p(x) Y(x,c)
int launch_gather(const sparc_op *op, int dtype, const void *Y, int64_t ldy, int ns, void *G,
                  hipStream_t stream);

// enqueue one fused step
int launch_step(const sparc_op *op, int dtype, const void *yk, int64_t ldk, const void *yprev, int64_t ldp,
                void *out, int64_t ldo, int ns, const void *G, const StepCoef &c, const StepLaunch &L,
                hipStream_t stream);

// profiling hooks (no-ops unless enabled)
struct ProfScope {
    int kernel;
    hipStream_t stream;
    void *ev0 = nullptr;
    ProfScope(int kernel, hipStream_t s);
    ~ProfScope();
};

}  // namespace sparc
