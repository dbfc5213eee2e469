// Request server for CheFSI passes (Sec. 3.4) on resident clusters.
//
// A request asks for one SCF iteration's eigensolve on a cluster.  On the
// cluster's first request its operator is built, its orbitals are copied into
// a resident block, the filter bounds come from the device Lanczos (Sec. 4)
// and the first-SCF rule runs: several CheFSI passes (filter, FP64
// Rayleigh-Ritz, Fermi level, rotation) from the caller's random block
// without a density update in between (Sec. 3.4, last paragraph).  Every
// later request runs one pass on the resident rotated orbitals.  The cutoff
// of each pass after the first is the previous pass's Fermi level + 0.1 Ha
// (Sec. 4), carried from request to request.  Every pass runs in the
// cluster's own dtype.  Requests of one cluster run in submission order;
// requests of different clusters run concurrently on the workers' own
// streams, so work admitted while other requests are on the device overlaps
// with them (continuous batching).  A cluster is admitted only when its
// device footprint fits the budget next to the resident clusters; its memory
// is returned after the request that carries `release`.  Every step is
// deterministic and per-cluster buffers are private, so a cluster's results
// do not depend on what else runs.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>

#include "internal.hpp"

namespace sparc {
namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct AtomCopy {
    sparc_atom a;
    std::vector<double> chi, gamma;
};

struct Cluster {
    uint64_t id = 0;
    sparc_grid grid{};
    std::vector<double> veff;
    std::vector<AtomCopy> atoms;
    int dtype = 0, ns = 0, m = 0;
    double ne = 0, lambda_f = 0;  // electron count; Fermi level of the last pass
    double theta0 = 0;            // lowest Ritz value of the last pass
    const void *X0 = nullptr;
    int64_t ldx0 = 0;
    const double *v0 = nullptr;
    int64_t nd = 0;
    size_t footprint = 0;
    bool resident = false, busy = false;
    int next_step = 0, submitted = 0;
    bool released = false;
    // device state
    sparc_op *op = nullptr;
    void *X = nullptr, *Y = nullptr, *ws = nullptr, *rr = nullptr, *evec = nullptr, *rot = nullptr;
    size_t ws_bytes = 0, rr_bytes = 0, rot_bytes = 0;
    double a0 = 0, a = 0, b = 0;
};

struct Request {
    uint64_t ticket;
    uint64_t cluster;
    int step;
    int release;
    double *ritz;
    double t_submit;
};

}  // namespace
}  // namespace sparc

using namespace sparc;

struct sparc_server {
    int device = 0;
    size_t budget = 0;
    int lanczos_k = 40;
    int first_passes = 3;
    double kT = 1e-3;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::deque<Request> pending;
    std::unordered_map<uint64_t, Cluster *> clusters;
    std::unordered_set<uint64_t> retired;  // ids of released or failed clusters (their records are freed)
    std::map<uint64_t, sparc_job_result> done;
    std::map<uint64_t, int> open;  // tickets submitted and not yet polled as done
    uint64_t next_ticket = 1;
    size_t used = 0;
    int64_t n_done = 0, n_running = 0;
    std::vector<std::thread> workers;
};

namespace {

// dst(:, c) = src(:, c) for the ns columns of an nd-row block, converted to To
template <typename Ti, typename To>
__global__ void copy_block(const Ti *__restrict__ src, long long lds, To *__restrict__ dst, long long ldd,
                           long long nd, int ns)
{
    const long long total = nd * ns;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total;
         t += (long long)gridDim.x * blockDim.x) {
        const long long c = t / nd, x = t - c * nd;
        dst[c * ldd + x] = (To)src[c * lds + x];
    }
}

template <typename Ti, typename To>
int launch_copy(const void *src, long long lds, void *dst, long long ldd, long long nd, int ns, hipStream_t s)
{
    hipLaunchKernelGGL((copy_block<Ti, To>), dim3(4096), dim3(256), 0, s, (const Ti *)src, lds, (To *)dst, ldd, nd, ns);
    SPARC_HIP(hipGetLastError());
    return SPARC_OK;
}

size_t estimate_footprint(const Cluster &c, int lanczos_k)
{
    const size_t s = c.dtype == SPARC_F64 ? 8 : 4;
    size_t chi = 0, box = 0, nproj = 0;
    for (auto &a : c.atoms) {
        const size_t nb = (size_t)a.a.ext[0] * a.a.ext[1] * a.a.ext[2];
        chi += nb * a.a.nproj;
        box += nb;
        nproj += a.a.nproj;
    }
    const size_t nd = (size_t)c.nd, ns = (size_t)c.ns;
    size_t f = nd * 12 + chi * 12 + box * 28 + 4096;                 // operator
    f += 3 * nd * ns * s + 4 * std::max<size_t>(1, nproj) * ns * s;  // X, Y, filter workspace
    f += nd * ns * 8;                                                 // Rayleigh-Ritz H Y
    f += 4 * std::max<size_t>(1, nproj) * ns * 8 + 1024 * 2 * ns * ns * 8 + 4 * (ns + 64) * (ns + 64) * 8 + 4096;
    // first request only: the Lanczos basis and workspace
    return f + nd * (lanczos_k + 1) * 8 + 4096 * (lanczos_k + 2) * 8;
}

// Cluster blocks come from the stream-ordered allocator on the worker's
// stream, so allocating or returning them does not wait for other workers'
// work on the device.
void free_device(Cluster &c, hipStream_t s)
{
    for (void **p : {&c.X, &c.Y, &c.ws, &c.rr, &c.evec, &c.rot}) {
        if (*p) (void)hipFreeAsync(*p, s);
        *p = nullptr;
    }
    (void)hipStreamSynchronize(s);
    sparc_op_destroy(c.op);
    c.op = nullptr;
    c.resident = false;
}

// runs one request on stream s; returns a status
int execute(sparc_server *srv, Cluster &c, const Request &r, hipStream_t s, sparc_job_result &res)
{
    TraceRange trace("serve request");
    int st;
    int passes = 1;
    double cut = c.lambda_f + 0.1;  // Sec. 4: previous Fermi level + 0.1 Ha
    if (c.resident && cut <= c.a0) c.a0 = c.theta0;  // the lambda_1 estimate was too high (as between passes)
    if (!c.resident) {
        std::vector<sparc_atom> at(c.atoms.size());
        for (size_t i = 0; i < at.size(); ++i) at[i] = c.atoms[i].a;
        if ((st = sparc_op_create(&c.grid, c.veff.data(), (int)at.size(), at.data(), &c.op))) return st;
        c.ws_bytes = sparc_workspace_bytes(c.op, c.dtype, c.ns, 1);
        c.rr_bytes = sparc_rr_workspace_bytes(c.op, c.dtype, c.ns);
        c.rot_bytes = sparc_rotate_workspace_bytes(c.dtype, c.ns);
        const size_t blk = (size_t)c.nd * c.ns * elem_size(c.dtype);
        if (hipMallocAsync(&c.X, blk, s) != hipSuccess || hipMallocAsync(&c.Y, blk, s) != hipSuccess ||
            hipMallocAsync(&c.ws, c.ws_bytes, s) != hipSuccess || hipMallocAsync(&c.rr, c.rr_bytes, s) != hipSuccess ||
            hipMallocAsync(&c.evec, (size_t)c.ns * c.ns * sizeof(double), s) != hipSuccess ||
            hipMallocAsync(&c.rot, c.rot_bytes, s) != hipSuccess)
            return fail(SPARC_E_NOMEM, "cluster allocation failed");
        c.resident = true;
        // bounds from the device Lanczos; later requests keep a0 and b
        const size_t lb = sparc_lanczos_workspace_bytes(c.op, srv->lanczos_k);
        void *lw = nullptr;
        if (hipMallocAsync(&lw, lb, s) != hipSuccess) return fail(SPARC_E_NOMEM, "Lanczos workspace allocation failed");
        std::vector<double> lt(srv->lanczos_k);
        st = sparc_lanczos(c.op, srv->lanczos_k, c.v0, nullptr, nullptr, lt.data(), lw, lb, s);
        (void)hipFreeAsync(lw, s);
        if (st) return st;
        double ub = 0;
        sparc_upper_bound(c.op, &ub);
        if ((st = sparc_select_bounds(lt.data(), srv->lanczos_k, 8, 0.1, 1.01, ub, &c.a0, &c.a, &c.b))) return st;
        if (c.dtype == SPARC_F64)
            st = launch_copy<double, double>(c.X0, c.ldx0, c.X, c.nd, c.nd, c.ns, s);
        else
            st = launch_copy<float, float>(c.X0, c.ldx0, c.X, c.nd, c.nd, c.ns, s);
        if (st) return st;
        passes = srv->first_passes;  // the first SCF iteration (Sec. 3.4, last paragraph)
        cut = c.a;
    }
    std::vector<double> theta((size_t)passes * c.ns), lf(passes);
    std::vector<int32_t> deg(passes);
    ChefsiBuffers B{c.Y, c.nd, c.ws, c.ws_bytes, c.rr, c.rr_bytes, (double *)c.evec, c.rot, c.rot_bytes, nullptr};
    int halvings = 0;
    if ((st = chefsi_run(c.op, c.dtype, c.X, c.nd, c.ns, c.m, passes, c.ne, srv->kT, c.a0, cut, c.b, B, theta.data(),
                         lf.data(), deg.data(), nullptr, s, &halvings)))
        return st;
    const double *last = theta.data() + (size_t)(passes - 1) * c.ns;
    c.lambda_f = lf[passes - 1];
    c.theta0 = last[0];
    if (r.ritz) std::memcpy(r.ritz, last, (size_t)c.ns * sizeof(double));
    res.lambda_min = last[0];
    res.lambda_f = c.lambda_f;
    res.passes = passes;
    res.halvings = halvings;
    int64_t degsum = 0;
    for (int p = 0; p < passes; ++p) degsum += deg[p];
    res.updates = c.nd * (int64_t)c.ns * degsum;
    return SPARC_OK;
}

// first pending request that may start now (FIFO order, skipping blocked ones)
std::deque<Request>::iterator admissible(sparc_server *srv)
{
    for (auto it = srv->pending.begin(); it != srv->pending.end(); ++it) {
        auto ci = srv->clusters.find(it->cluster);
        if (ci == srv->clusters.end()) continue;
        Cluster &c = *ci->second;
        if (c.released || c.busy || it->step != c.next_step) continue;
        if (!c.resident && srv->used + c.footprint > srv->budget) continue;
        return it;
    }
    return srv->pending.end();
}

void worker_main(sparc_server *srv)
{
    (void)hipSetDevice(srv->device);
    hipStream_t s = nullptr;
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (;;) {
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->cv.wait(lk, [&] { return srv->stop || admissible(srv) != srv->pending.end(); });
        auto it = admissible(srv);
        if (it == srv->pending.end()) {
            if (srv->stop) break;
            continue;
        }
        const Request r = *it;
        srv->pending.erase(it);
        Cluster &c = *srv->clusters[r.cluster];
        c.busy = true;
        if (!c.resident) srv->used += c.footprint;
        ++srv->n_running;
        lk.unlock();

        sparc_job_result res{};
        res.step = r.step;
        res.t_submit = r.t_submit;
        res.t_start = now_s();
        res.status = execute(srv, c, r, s, res);
        if (res.status != SPARC_OK) {
            (void)hipStreamSynchronize(s);
            std::strncpy(res.error, sparc_last_error(), sizeof(res.error) - 1);
        }
        res.t_end = now_s();

        lk.lock();
        if (r.release || res.status != SPARC_OK) {
            // a released or failed cluster takes no further requests: its
            // queued ones fail below and later submissions are refused
            c.released = true;
            lk.unlock();
            free_device(c, s);
            lk.lock();
            srv->used -= c.footprint;
        }
        c.busy = false;
        c.next_step = r.step + 1;
        srv->done[r.ticket] = res;
        ++srv->n_done;
        --srv->n_running;
        // requests queued behind a failed or released cluster can never run
        for (auto p = srv->pending.begin(); p != srv->pending.end();) {
            auto ci = srv->clusters.find(p->cluster);
            if (ci != srv->clusters.end() && ci->second->released) {
                sparc_job_result fr{};
                fr.status = SPARC_E_JOB;
                std::strncpy(fr.error, "an earlier request of this cluster failed", sizeof(fr.error) - 1);
                fr.step = p->step;
                fr.t_submit = p->t_submit;
                fr.t_start = fr.t_end = now_s();
                srv->done[p->ticket] = fr;
                ++srv->n_done;
                p = srv->pending.erase(p);
            } else {
                ++p;
            }
        }
        if (c.released) {
            // no request refers to it any more: drop the record with its host
            // copies of V_eff and the projectors; the id stays refused
            srv->clusters.erase(r.cluster);
            srv->retired.insert(r.cluster);
            delete &c;
        }
        lk.unlock();
        srv->cv.notify_all();
    }
    (void)hipStreamDestroy(s);
}

}  // namespace

extern "C" {

double sparc_clock(void) { return now_s(); }

uint64_t sparc_cluster_footprint(const sparc_cluster_desc *d, int32_t lanczos_steps)
{
    if (!d) return 0;
    Cluster c;
    c.dtype = d->dtype;
    c.ns = d->ns;
    c.nd = (int64_t)d->grid.n[0] * d->grid.n[1] * d->grid.n[2];
    c.atoms.resize(d->natoms > 0 ? d->natoms : 0);
    for (int i = 0; i < d->natoms; ++i) c.atoms[i].a = d->atoms[i];
    return estimate_footprint(c, lanczos_steps > 0 ? lanczos_steps : 40);
}

int sparc_server_create(const sparc_server_cfg *cfg, sparc_server **out)
{
    if (!cfg || !out) return fail(SPARC_E_ARG, "null argument");
    *out = nullptr;
    if (cfg->workers < 1 || cfg->workers > 64) return fail(SPARC_E_ARG, "workers must be in 1..64");
    sparc_server *srv = new (std::nothrow) sparc_server();
    if (!srv) return fail(SPARC_E_NOMEM, "host allocation failed");
    (void)hipGetDevice(&srv->device);
    srv->budget = cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (size_t)250e9;
    srv->lanczos_k = cfg->lanczos_steps > 0 ? cfg->lanczos_steps : 40;
    if (cfg->first_passes < 0 || cfg->first_passes > 64) {
        delete srv;
        return fail(SPARC_E_ARG, "first_passes must be in 0..64");
    }
    if (cfg->kT < 0 || !(cfg->kT == cfg->kT)) {
        delete srv;
        return fail(SPARC_E_ARG, "kT must be >= 0");
    }
    srv->first_passes = cfg->first_passes > 0 ? cfg->first_passes : 3;
    srv->kT = cfg->kT > 0 ? cfg->kT : 1e-3;
    for (int i = 0; i < cfg->workers; ++i) srv->workers.emplace_back(worker_main, srv);
    *out = srv;
    return SPARC_OK;
}

int sparc_filter_submit(sparc_server *srv, const sparc_filter_job *job, uint64_t *ticket)
{
    if (!srv || !job || !ticket) return fail(SPARC_E_ARG, "null argument");
    const double t = now_s();
    // host copies of a new cluster's description are made outside the lock
    std::unique_ptr<Cluster> fresh;
    if (job->desc) {
        const sparc_cluster_desc &d = *job->desc;
        if (!d.veff || (d.natoms > 0 && !d.atoms) || d.natoms < 0 || !d.X0 || !d.v0)
            return fail(SPARC_E_ARG, "incomplete cluster description");
        if (d.dtype != SPARC_F64 && d.dtype != SPARC_F32) return fail(SPARC_E_ARG, "bad dtype");
        if (d.ns < 1 || d.m < 1) return fail(SPARC_E_BOUNDS, "ns and m must be >= 1");
        if (!(d.ne > 0.0 && d.ne < 2.0 * d.ns)) return fail(SPARC_E_ARG, "need 0 < ne < 2 ns");
        if (d.grid.n[0] < 1 || d.grid.n[1] < 1 || d.grid.n[2] < 1) return fail(SPARC_E_SHAPE, "bad grid");
        const int64_t nd = (int64_t)d.grid.n[0] * d.grid.n[1] * d.grid.n[2];
        if (d.ldx0 < nd) return fail(SPARC_E_SHAPE, "leading dimension of X0 is below N_d");
        fresh.reset(new (std::nothrow) Cluster());
        if (!fresh) return fail(SPARC_E_NOMEM, "host allocation failed");
        Cluster &c = *fresh;
        c.id = job->cluster;
        c.grid = d.grid;
        c.nd = nd;
        c.veff.assign(d.veff, d.veff + nd);
        c.atoms.resize(d.natoms);
        for (int i = 0; i < d.natoms; ++i) {
            const sparc_atom &a = d.atoms[i];
            AtomCopy &ac = c.atoms[i];
            ac.a = a;
            const size_t cnt = (size_t)a.ext[0] * a.ext[1] * a.ext[2] * (a.nproj > 0 ? a.nproj : 0);
            if (a.chi) ac.chi.assign(a.chi, a.chi + cnt);
            if (a.gamma) ac.gamma.assign(a.gamma, a.gamma + (a.nproj > 0 ? a.nproj : 0));
            ac.a.chi = a.chi ? ac.chi.data() : nullptr;
            ac.a.gamma = a.gamma ? ac.gamma.data() : nullptr;
        }
        c.dtype = d.dtype;
        c.ns = d.ns;
        c.m = d.m;
        c.ne = d.ne;
        c.X0 = d.X0;
        c.ldx0 = d.ldx0;
        c.v0 = d.v0;
        c.footprint = estimate_footprint(c, srv->lanczos_k);
        if (c.footprint > srv->budget) return fail(SPARC_E_NOMEM, "cluster footprint exceeds the device budget");
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->retired.count(job->cluster)) return fail(SPARC_E_JOB, "cluster already released or failed");
    auto ci = srv->clusters.find(job->cluster);
    Cluster *c = ci == srv->clusters.end() ? nullptr : ci->second;
    if (fresh) {
        if (c) return fail(SPARC_E_ARG, "cluster id already in use");
        c = fresh.release();
        srv->clusters[job->cluster] = c;
    } else if (!c) {
        return fail(SPARC_E_ARG, "unknown cluster (its first request must carry a description)");
    }
    if (c->released) return fail(SPARC_E_JOB, "cluster already released or failed");
    Request r{srv->next_ticket++, job->cluster, c->submitted++, job->release, job->ritz, t};
    srv->pending.push_back(r);
    srv->open[r.ticket] = 1;
    *ticket = r.ticket;
    srv->cv.notify_all();
    return SPARC_OK;
}

int sparc_filter_poll(sparc_server *srv, uint64_t ticket, sparc_job_result *res)
{
    if (!srv) return fail(SPARC_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto d = srv->done.find(ticket);
    if (d == srv->done.end()) {
        if (srv->open.count(ticket)) return SPARC_PENDING;
        return fail(SPARC_E_TICKET, "unknown ticket");
    }
    if (res) *res = d->second;
    srv->done.erase(d);
    srv->open.erase(ticket);
    return SPARC_OK;
}

int sparc_server_stats(sparc_server *srv, int64_t *done, int64_t *pending, int64_t *running, uint64_t *hbm_used)
{
    if (!srv) return fail(SPARC_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (done) *done = srv->n_done;
    if (pending) *pending = (int64_t)srv->pending.size();
    if (running) *running = srv->n_running;
    if (hbm_used) *hbm_used = srv->used;
    return SPARC_OK;
}

int sparc_server_clusters(sparc_server *srv, int64_t *records, int64_t *retired)
{
    if (!srv) return fail(SPARC_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (records) *records = (int64_t)srv->clusters.size();
    if (retired) *retired = (int64_t)srv->retired.size();
    return SPARC_OK;
}

int sparc_server_destroy(sparc_server *srv)
{
    if (!srv) return SPARC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // requests that have not started are dropped
        srv->pending.clear();
    }
    srv->cv.notify_all();
    for (auto &t : srv->workers) t.join();
    hipStream_t s = nullptr;
    (void)hipSetDevice(srv->device);
    (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    for (auto &kv : srv->clusters) {
        free_device(*kv.second, s);
        delete kv.second;
    }
    (void)hipStreamDestroy(s);
    delete srv;
    return SPARC_OK;
}

}  // extern "C"
