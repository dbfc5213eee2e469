// Autotuner of the vector step launch: for one operator, dtype and column
// count it times every patch height, a few x splits, column groups and one or
// two columns per workgroup (orbital blocking) of what a filter step enqueues
// (the fused stencil / potential / recurrence pass with the projector gather
// of its input in the same launch, then the projector scatter) on
// pseudo-random scratch blocks, with HIP events around repeated steps, and
// keeps the fastest.  Choices are cached per
// (grid, atoms, projectors, columns, dtype) in the process and, when
// SPARC_TUNE_CACHE names a file, in that text file (one line per entry:
// n1 n2 n3 natoms nproj ns dtype plan chunk group block microseconds).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <tuple>

#include "internal.hpp"

namespace sparc {
namespace {

using Key = std::tuple<int, int, int, int, int, int, int>;
struct Choice {
    int plan, chunk, group, cblk;
    double us;
};
std::mutex g_tune_mu;
std::map<Key, Choice> g_tune;
bool g_tune_loaded = false;

void load_cache()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("SPARC_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int n1, n2, n3, na, np, ns, dt, pl, ch, gr, cb;
    double us;
    while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %d %d %lf", &n1, &n2, &n3, &na, &np, &ns, &dt, &pl, &ch, &gr, &cb,
                       &us) == 12)
        if (pl >= 0 && pl < kNumPlans && ch > 0 && gr > 0 && (cb == 1 || cb == 2))
            g_tune[Key(n1, n2, n3, na, np, ns, dt)] = {pl, ch, gr, cb, us};
    std::fclose(f);
}

void store_cache(const Key &k, const Choice &c)
{
    const char *path = std::getenv("SPARC_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), c.plan, c.chunk, c.group, c.cblk,
                 c.us);
    std::fclose(f);
}

// scratch blocks of pseudo-random values in [-1, 1) (a multiplicative hash of
// the index): all-zero blocks run measurably faster than orbital data on this
// chip, which would bias the choice
template <typename T>
__global__ void __launch_bounds__(256) fill_hash(T *__restrict__ x, long long n, unsigned salt)
{
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const unsigned h = ((unsigned)i ^ salt) * 2654435761u;
        x[i] = (T)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
    }
}

void fill_scratch(int dtype, void *p, size_t bytes, unsigned salt, hipStream_t s)
{
    if (dtype == SPARC_F64)
        hipLaunchKernelGGL(fill_hash<double>, dim3(4096), dim3(256), 0, s, (double *)p, (long long)(bytes / 8), salt);
    else
        hipLaunchKernelGGL(fill_hash<float>, dim3(4096), dim3(256), 0, s, (float *)p, (long long)(bytes / 4), salt);
}

}  // namespace
}  // namespace sparc

using namespace sparc;

extern "C" int sparc_autotune(sparc_op *op, int32_t dtype, int32_t ns, void *stream, int32_t *tile_z, int32_t *tile_y,
                              int32_t *chunk_x, int32_t *col_group, int32_t *col_block, double *best_us)
{
    if (!op || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32)) return fail(SPARC_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    if (choose_vec_launch(op, dtype, ns, {}).plan < 0)
        return fail(SPARC_E_SHAPE, "the vector step kernels cannot take this grid (nothing to tune)");
    const Key key(op->n[0], op->n[1], op->n[2], op->natoms, op->nproj_total, ns, dtype);
    Choice best{-1, 0, 1, 1, 1e30};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) best = it->second;
    }
    if (best.plan < 0) {
        const size_t es = elem_size(dtype);
        const size_t blk = (size_t)op->nd * ns * es;
        const int saved_shape = op->tune_shape[dtype], saved_chunk = op->tune_chunk[dtype];
        const int saved_ns = op->tune_ns[dtype], saved_group = op->tune_group[dtype];
        const int saved_cblk = op->tune_cblk[dtype];
        const int n1 = op->n[0];
        const int chunks[] = {0, n1, (n1 + 1) / 2, (n1 + 3) / 4, (n1 + 7) / 8};
        const size_t pb = std::max<size_t>(gather_bytes(op, dtype, ns), 256);
        void *X = nullptr, *Y = nullptr, *Pv = nullptr, *G = nullptr;
        if (hipMalloc(&X, blk) != hipSuccess || hipMalloc(&Y, blk) != hipSuccess || hipMalloc(&Pv, blk) != hipSuccess ||
            hipMalloc(&G, pb) != hipSuccess) {
            (void)hipFree(X);
            (void)hipFree(Y);
            (void)hipFree(Pv);
            (void)hipFree(G);
            return fail(SPARC_E_NOMEM, "autotune scratch allocation failed");
        }
        op->tune_ns[dtype] = ns;
        fill_scratch(dtype, X, blk, 0x9e3779b9u, s);
        fill_scratch(dtype, Pv, blk, 0x7f4a7c15u, s);
        (void)hipMemsetAsync(G, 0, pb, s);
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        StepCoef cf{1.0, 0.5, 0.0, 1};
        const StepLaunch Ls = choose_step_launch(op, dtype, ns);
        int st = SPARC_OK;
        const int groups[] = {1, 4, 8, 16};
        for (int p = 0; p < kNumPlans && st == SPARC_OK; ++p) {
            if (!vec_plan_valid(dtype, p)) continue;
            for (int ci = 0; ci < 5 && st == SPARC_OK; ++ci) {
                if (chunks[ci] > 0 && chunks[ci] < 4) continue;
                for (int cb = 1; cb <= 2 && st == SPARC_OK; ++cb) {
                for (int gi = 0; gi < 4 && st == SPARC_OK; ++gi) {
                    if (groups[gi] * cb > ns && gi > 0) continue;
                    if (cb == 2 && (ns < 2 || vec_max_cblk(dtype, p) < 2)) continue;
                    op->tune_shape[dtype] = p;
                    op->tune_chunk[dtype] = chunks[ci];
                    op->tune_group[dtype] = groups[gi];
                    op->tune_cblk[dtype] = cb;
                    const FLaunch L = choose_vec_launch(op, dtype, ns, {});
                    if (L.plan != p) continue;
                    // a filter step as the filter runs it: the step with the
                    // gather of its input in one launch, then the scatter
                    if ((st = launch_h_step(op, dtype, X, op->nd, Pv, op->nd, Y, op->nd, ns, G, cf, Ls, s, &L))) break;
                    (void)hipEventRecord(e0, s);
                    const int reps = 3;
                    for (int r = 0; r < reps && st == SPARC_OK; ++r)
                        st = launch_h_step(op, dtype, X, op->nd, Pv, op->nd, Y, op->nd, ns, G, cf, Ls, s, &L);
                    (void)hipEventRecord(e1, s);
                    if (hipEventSynchronize(e1) != hipSuccess) st = fail(SPARC_E_HIP, "autotune timing failed");
                    float ms = 0;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    const double us = ms * 1e3 / reps;
                    if (st == SPARC_OK && us < best.us) best = {p, L.chunk_x, L.cgroup, L.cblk, us};
                }
                }
            }
        }
        op->tune_shape[dtype] = saved_shape;
        op->tune_chunk[dtype] = saved_chunk;
        op->tune_ns[dtype] = saved_ns;
        op->tune_group[dtype] = saved_group;
        op->tune_cblk[dtype] = saved_cblk;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(X);
        (void)hipFree(Y);
        (void)hipFree(Pv);
        (void)hipFree(G);
        if (st) return st;
        if (best.plan < 0) return fail(SPARC_E_SHAPE, "no usable patch height");
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
        store_cache(key, best);
    }
    op->tune_shape[dtype] = best.plan;
    op->tune_chunk[dtype] = best.chunk;
    op->tune_group[dtype] = best.group;
    op->tune_cblk[dtype] = best.cblk;
    op->tune_ns[dtype] = ns;  // the choice holds for this block width only
    if (tile_z) *tile_z = kPlanTZ[best.plan];
    if (tile_y) *tile_y = kPlanTY[best.plan];
    if (chunk_x) *chunk_x = best.chunk;
    if (col_group) *col_group = best.group;
    if (col_block) *col_block = best.cblk;
    if (best_us) *best_us = best.us;
    return SPARC_OK;
}
