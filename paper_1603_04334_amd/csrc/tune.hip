// Autotuner of the fused step kernel's launch: for one operator, dtype and
// column count it times every tile shape and a few x-chunk lengths on scratch
// blocks (HIP events around repeated recurrence-step launches) and keeps the
// fastest.  Choices are cached per (grid, columns, dtype) in the process and,
// when SPARC_TUNE_CACHE names a file, in that text file (one line per entry:
// n1 n2 n3 ns dtype shape chunk microseconds).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <tuple>

#include "internal.hpp"

namespace sparc {
namespace {

using Key = std::tuple<int, int, int, int, int>;
struct Choice {
    int shape, chunk;
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
    int n1, n2, n3, ns, dt, sh, ch;
    double us;
    while (std::fscanf(f, "%d %d %d %d %d %d %d %lf", &n1, &n2, &n3, &ns, &dt, &sh, &ch, &us) == 8)
        if (sh >= 0 && sh < kNumShapes && ch > 0) g_tune[Key(n1, n2, n3, ns, dt)] = {sh, ch, us};
    std::fclose(f);
}

void store_cache(const Key &k, const Choice &c)
{
    const char *path = std::getenv("SPARC_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), c.shape, c.chunk, c.us);
    std::fclose(f);
}

}  // namespace
}  // namespace sparc

using namespace sparc;

extern "C" int sparc_autotune(sparc_op *op, int32_t dtype, int32_t ns, void *stream, int32_t *tile_z, int32_t *tile_y,
                              int32_t *chunk_x, double *best_us)
{
    if (!op || ns < 1 || (dtype != SPARC_F64 && dtype != SPARC_F32)) return fail(SPARC_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const Key key(op->n[0], op->n[1], op->n[2], ns, dtype);
    Choice best{-1, 0, 1e30};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) best = it->second;
    }
    if (best.shape < 0) {
        const size_t es = elem_size(dtype);
        const size_t blk = (size_t)op->nd * ns * es;
        void *X = nullptr, *Y = nullptr, *P = nullptr;
        if (hipMalloc(&X, blk) != hipSuccess || hipMalloc(&Y, blk) != hipSuccess || hipMalloc(&P, blk) != hipSuccess) {
            (void)hipFree(X);
            (void)hipFree(Y);
            (void)hipFree(P);
            return fail(SPARC_E_NOMEM, "autotune scratch allocation failed");
        }
        (void)hipMemsetAsync(X, 0, blk, s);
        (void)hipMemsetAsync(P, 0, blk, s);
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        const int saved_shape = op->tune_shape[dtype], saved_chunk = op->tune_chunk[dtype];
        const int saved_ns = op->tune_ns[dtype];
        op->tune_ns[dtype] = ns;
        const int n1 = op->n[0];
        const int chunks[] = {0, n1, (n1 + 1) / 2, (n1 + 3) / 4, (n1 + 7) / 8};
        StepCoef cf{1.0, 0.5, 0.0, 1};
        int st = SPARC_OK;
        for (int sh = 0; sh < kNumShapes && st == SPARC_OK; ++sh) {
            for (int ci = 0; ci < 5 && st == SPARC_OK; ++ci) {
                if (chunks[ci] > 0 && chunks[ci] < 4) continue;
                op->tune_shape[dtype] = sh;
                op->tune_chunk[dtype] = chunks[ci];
                const StepLaunch L = choose_step_launch(op, dtype, ns);
                if ((st = launch_step(op, dtype, X, op->nd, P, op->nd, Y, op->nd, ns, cf, L, s))) break;
                (void)hipEventRecord(e0, s);
                const int reps = 3;
                for (int r = 0; r < reps && st == SPARC_OK; ++r)
                    st = launch_step(op, dtype, X, op->nd, P, op->nd, Y, op->nd, ns, cf, L, s);
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) st = fail(SPARC_E_HIP, "autotune timing failed");
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                const double us = ms * 1e3 / reps;
                if (st == SPARC_OK && us < best.us) best = {sh, L.chunk_x, us};
            }
        }
        op->tune_shape[dtype] = saved_shape;
        op->tune_chunk[dtype] = saved_chunk;
        op->tune_ns[dtype] = saved_ns;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(X);
        (void)hipFree(Y);
        (void)hipFree(P);
        if (st) return st;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
        store_cache(key, best);
    }
    op->tune_shape[dtype] = best.shape;
    op->tune_chunk[dtype] = best.chunk;
    op->tune_ns[dtype] = ns;  // the choice holds for this block width only
    if (tile_z) *tile_z = kShapes[best.shape].tz;
    if (tile_y) *tile_y = kShapes[best.shape].ty();
    if (chunk_x) *chunk_x = best.chunk;
    if (best_us) *best_us = best.us;
    return SPARC_OK;
}
