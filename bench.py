"""Benchmark of the Chebyshev-filter hot path on one MI355X.

Workload (default): the largest single-GPU cluster, a 160^3 grid with h = 0.35
bohr, 128 atoms with 9 Kleinman-Bylander projectors each (l = 0, 1, 2), 600
orbitals N(0,1), filter degree m = 30, stencil order 12.  One step is one
filtered-subspace pass over the resident orbital block: 40-step FP64 Lanczos
bounds on the device, the Chebyshev filter in the selected dtype (FP32 by
default, FP32 accumulation), FP64 Rayleigh-Ritz on the device and the
subspace rotation; each pass starts from the orbitals the previous one
rotated.  ``value`` is filtered orbital*gridpoint updates per second of the
whole step (N_d * N_s * m / step time).  The FP64 pass is measured beside it.

Prints ONE JSON line.  Defaults: 1 GPU, 5 timed steps, 1 warmup.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KSTEPS_LANCZOS = 40
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic_cluster160.txt")
# launch choices of the autotuner on MI355X for the benchmark clusters (read
# by the library through SPARC_TUNE_CACHE; a fresh tuning run appends to it),
# so that the benchmark runs the launch its committed counters were taken on
TUNE_CACHE = os.path.join(ROOT, "paper_1603_04334_amd", "tune_mi355x.txt")
STENCIL_SRCS = [os.path.join(ROOT, "paper_1603_04334_amd", "csrc", f)
                for f in ("fstep.hip", "fstep_kernel.hpp", "fstep_launch.hpp", "nonlocal_kernel.hpp")]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    p.add_argument("--workload", choices=["large", "medium", "small"], default="large")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64-compare", action="store_true")
    p.add_argument("--no-secondary", action="store_true", help="skip the medium-cluster and small-cluster lines")
    p.add_argument("--no-batch", action="store_true", help="skip the batched uneven-cluster measurement")
    p.add_argument("--no-next", action="store_true",
                   help="skip the first-SCF, density, force and electrostatic-potential measurements")
    p.add_argument("--batch-only", action="store_true", help="print only the batched measurement")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--serve-only", action="store_true", help="print only the serving measurement")
    p.add_argument("--serve-rates", default="50",
                   help="comma-separated Poisson arrival rates in requests/s (full sweep: 50,100,200,500,1000,2000)")
    p.add_argument("--serve-requests", type=int, default=500, help="requests per rate point (5 per cluster)")
    p.add_argument("--serve-workers", type=int, default=4)
    p.add_argument("--copy-calibration", action="store_true",
                   help="run only the library's reference copy kernel on 4 GiB (counter calibration)")
    p.add_argument("--filter-only", action="store_true",
                   help="run only the filter of the workload (warmup + steps launches; for counter runs)")
    return p.parse_args()


def source_hash() -> str:
    """Hash of the dominant launch's sources (vector step and gather)."""
    h = hashlib.sha256()
    for f in STENCIL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(dtype, config=None):
    """Calibrated HBM bytes per recurrence-step launch from committed counter
    runs, or None when absent, taken on a different kernel source, or on
    another launch configuration than ``config`` (tile_z tile_y chunk_x
    col_group col_block)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("stencil_sha256_16") != source_hash():
        return None
    if config is not None and kv.get(f"{dtype}_launch") != " ".join(str(int(v)) for v in config):
        return None
    try:
        return float(kv[f"{dtype}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_bandwidth(nbytes=4 << 30, reps=10):
    """GB/s (read + written) of the library's reference copy kernel."""
    import torch
    from paper_1603_04334_amd import binding
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    binding.stream_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        binding.stream_copy(b, a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def alg_bytes_per_step_launch(case, cl, s):
    """Algorithmic HBM bytes of one recurrence-step launch (the fused step with
    Y_{k-1} and the projector gather of the same Y_k): read Y_k and Y_{k-1},
    write Y_{k+1} (s bytes per orbital*gridpoint each), read V_eff once (s per
    gridpoint), read the projector values once (s per cube point and
    projector) and write the gather's 8 split partials (s per projector and
    orbital each).  The gather's second read of Y_k at the cube points is
    an implementation cost and is not counted."""
    chi = sum(int(np.prod(a.ext)) * a.nproj for a in cl.atoms)
    return 3 * s * cl.nd * case.ns + s * cl.nd + s * chi + s * 8 * cl.nproj_total * case.ns


class Pass:
    """Resident state of one workload and one dtype."""

    def __init__(self, case, cluster, op, dtype, tune=True):
        import torch
        from paper_1603_04334_amd import binding, inputs
        self.binding = binding
        self.case = case
        self.cl = cluster
        self.op = op
        self.dt = torch.float32 if dtype == "f32" else torch.float64
        self.code = binding.SPARC_F32 if dtype == "f32" else binding.SPARC_F64
        self.tuned = op.autotune(self.code, case.ns) if tune else None
        self.X = inputs.device_orbitals(cluster.nd, case.ns, case.seed, self.dt)
        self.Y = torch.empty_like(self.X)
        self.R = torch.empty_like(self.X)
        self.v0 = torch.from_numpy(inputs.lanczos_start(cluster.nd, case.seed)).cuda()
        self.ws = op.workspace(self.code, case.ns, 1)
        self.ub = op.upper_bound()
        self.bounds = None
        self.ritz = None
        self.first_ritz = None
        self.stage_ms = None

    def step(self, profile_filter=False, stages=False):
        import torch
        b = self.binding
        t = [time.perf_counter()]
        _, _, theta = self.op.lanczos(KSTEPS_LANCZOS, self.v0)
        a0, a, bb = b.select_bounds(theta, 8, ubound=self.ub)
        self.bounds = (a0, a, bb)
        t.append(time.perf_counter())
        if profile_filter:
            b.profile.enable(True)
        self.op.cheb_filter(self.X, self.case.m, a0, a, bb, Y=self.Y, ws=self.ws)
        if profile_filter:
            b.profile.enable(False)
        if stages:
            torch.cuda.synchronize()
        t.append(time.perf_counter())
        self.ritz, Qt = self.op.rayleigh_ritz(self.Y)
        if self.first_ritz is None:
            self.first_ritz = self.ritz.copy()
        t.append(time.perf_counter())
        b.rotate(self.Y, Qt, out=self.R)
        if stages:
            torch.cuda.synchronize()
        t.append(time.perf_counter())
        if stages:
            self.stage_ms = {k: (t[i + 1] - t[i]) * 1e3 for i, k in enumerate(("lanczos", "filter", "rayleigh_ritz",
                                                                                 "rotation"))}
        # the next pass continues from the rotated orbitals, as the SCF passes do
        self.X, self.R = self.R, self.X

    def filter_only(self):
        a0, a, bb = self.bounds
        self.op.cheb_filter(self.X, self.case.m, a0, a, bb, Y=self.Y, ws=self.ws)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def measure_pass(case, cl, op, dtype, steps, warmup, kernel_stats=False):
    """Whole-step and filter-only timing of one dtype; kernel statistics of the
    recurrence-step launches (HIP events on the launching stream) and a stage
    breakdown when asked."""
    import torch
    from paper_1603_04334_amd import binding
    p = Pass(case, cl, op, dtype)
    out = {}
    t_step = timed(p.step, steps, warmup)
    out["ms_per_step"] = t_step * 1e3
    out["first_ritz"] = p.first_ritz
    out["bounds"] = p.bounds
    out["tuned"] = p.tuned
    if kernel_stats:
        binding.profile.reset()
        torch.cuda.synchronize()
        for _ in range(steps):
            p.step(profile_filter=True)
        torch.cuda.synchronize()
        out["kernels"] = {k: binding.profile.read(k) for k in range(4)}
        binding.profile.reset()
        p.step(stages=True)
        out["stages_ms"] = p.stage_ms
    out["filter_ms"] = timed(p.filter_only, steps, 1) * 1e3
    del p
    torch.cuda.empty_cache()
    return out


def batch_measure(reps=5, nclusters=64):
    """Batched uneven clusters (grid edge in {32..96}, h = 0.45, 2-24 atoms,
    16-128 orbitals, degree 16-28), FP32 with FP64 coefficients.  Bounds come
    from the device Lanczos (setup, untimed); orbitals are seeded N(0,1) drawn
    on the device.  Returns throughput of each execution mode and of the plain
    unbatched FP64 filters on the same clusters."""
    import torch
    from paper_1603_04334_amd import binding, inputs
    recipe = inputs.batch_recipe(nclusters=nclusters)
    jobs32, jobs64, ops, work = [], [], [], 0
    for r in recipe:
        cl = inputs.make_cluster(r["n"], r["h"], r["natoms"], r["zmax"], r["lmax"], r["seed"])
        op = binding.Operator(cl)
        _, _, theta = op.lanczos(KSTEPS_LANCZOS, torch.from_numpy(inputs.lanczos_start(cl.nd, r["seed"])).cuda())
        a0, a, b = binding.select_bounds(theta, 8, ubound=op.upper_bound())
        X = inputs.device_orbitals(cl.nd, r["ns"], r["seed"])
        jobs32.append((op, X, torch.empty_like(X), r["m"], a0, a, b))
        X64 = X.double()
        jobs64.append((op, X64, torch.empty_like(X64), r["m"], a0, a, b))
        ops.append(op)
        work += cl.nd * r["ns"] * r["m"]
    out = {"workload": f"{nclusters} uneven clusters, grid edge 32-96, h=0.45, 16-128 orbitals, degree 16-28",
           "updates_per_run": work}
    for name, jobs, mode in (("persistent_graph_f32", jobs32, 0), ("grouped_levels_graph_f32", jobs32, 4),
                             ("concurrent_streams_f32", jobs32, 5), ("sequential_f32", jobs32, 3),
                             ("sequential_f64", jobs64, 3)):
        bt = binding.Batch(jobs, mode=mode)
        bt.run()
        if bt.check():
            raise RuntimeError("batch aborted")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            bt.run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if bt.check():
            raise RuntimeError("batch aborted")
        out[name] = {"ms": dt * 1e3, "value": work / dt}
        if mode == 0:
            out["items"], out["levels"], out["grid"] = bt.info()
        bt.close()
    for k in ("persistent_graph_f32", "grouped_levels_graph_f32", "concurrent_streams_f32", "sequential_f32"):
        out[k]["vs_sequential_f64"] = out[k]["value"] / out["sequential_f64"]["value"]
    for k in ("persistent_graph_f32", "grouped_levels_graph_f32", "concurrent_streams_f32"):
        out[k]["vs_sequential_f32"] = out[k]["value"] / out["sequential_f32"]["value"]
    return out


SERVE_STEPS = 5
SERVE_BUDGET = 250e9


class ServeSetup:
    """Clusters of the serving stream (grid edge log-uniform in [24,128], h =
    0.45, 1-64 atoms, N_s = N_e/2 + 30, degree 20-30, FP32:FP64 = 80:20),
    built once.  Synthetic orbitals and Lanczos starts are prefixes of one
    seeded N(0,1) device buffer per dtype, which the server copies at
    admission."""

    def __init__(self, nclusters):
        import torch
        from paper_1603_04334_amd import binding, inputs
        sessions = inputs.serving_recipe(seed=5, nclusters=nclusters, rate=1.0, steps_per_cluster=SERVE_STEPS)
        self.specs = {r["cluster"]["seed"]: r["cluster"] for r in sessions}
        specs = self.specs
        maxnd = max(c["n"] ** 3 for c in specs.values())
        maxns = max(c["ns"] for c in specs.values())
        self.X64 = inputs.device_orbitals(maxnd * maxns, 1, 5, torch.float64).view(-1)
        self.X32 = self.X64.float() if any(c["fp32"] for c in specs.values()) else None
        self.v0 = inputs.device_orbitals(maxnd, 1, 6, torch.float64).view(-1)
        torch.cuda.synchronize()
        self.descs = {}
        for i, (sd, c) in enumerate(specs.items()):
            if i % 50 == 0:
                print(f"serving setup: cluster {i} of {len(specs)}", file=sys.stderr, flush=True)
            cl = inputs.make_cluster(c["n"], c["h"], c["natoms"], c["zmax"], c["lmax"], sd)
            src = self.X32 if c["fp32"] else self.X64
            X0 = src[: cl.nd * c["ns"]].view(c["ns"], cl.nd)
            # electrons of the cluster's atoms; where the 256-orbital cap cuts
            # ns below N_e/2 + 30, the count the capped block is sized for
            ne = min(c["ne"], 2 * (c["ns"] - 30))
            self.descs[sd] = binding.cluster_desc(cl, X0, self.v0[: cl.nd], c["m"], ne=ne)


def serve_point(setup, rate, nclusters, workers):
    """Open loop over sessions: a cluster's session arrives at its Poisson time
    and submits its first pass; each later pass is submitted as soon as the
    previous one is done (an SCF client waits for its orbitals).  Request
    latency = completion - submission of the pass; session latency =
    completion of the last pass - arrival."""
    from paper_1603_04334_amd import binding, inputs
    sessions = inputs.serving_recipe(seed=5, nclusters=nclusters, rate=rate, steps_per_cluster=SERVE_STEPS)
    srv = binding.Server(workers=workers, budget=int(SERVE_BUDGET), lanczos_steps=KSTEPS_LANCZOS)
    done = []          # (session index, pass, result)
    open_t = {}        # ticket -> (session index, pass)
    lag = 0.0
    nxt = 0
    try:
        t0 = binding.clock() + 0.01
        deadline = time.time() + 900
        while nxt < len(sessions) or open_t:
            now = binding.clock()
            while nxt < len(sessions) and t0 + sessions[nxt]["t_arrive"] <= now:
                c = sessions[nxt]["cluster"]
                tk = srv.submit(c["seed"], setup.descs[c["seed"]], release=SERVE_STEPS == 1)
                lag = max(lag, binding.clock() - (t0 + sessions[nxt]["t_arrive"]))
                open_t[tk] = (nxt, 0)
                nxt += 1
            for tk in list(open_t):
                r = srv.poll(tk)
                if r is None:
                    continue
                i, k = open_t.pop(tk)
                done.append((i, k, r))
                if r["status"] == 0 and k + 1 < SERVE_STEPS:
                    c = sessions[i]["cluster"]
                    open_t[srv.submit(c["seed"], release=k + 2 == SERVE_STEPS)] = (i, k + 1)
            if time.time() > deadline:
                raise RuntimeError("serving run did not finish")
            wait = (t0 + sessions[nxt]["t_arrive"] - binding.clock()) if nxt < len(sessions) else 1e-3
            time.sleep(min(max(wait, 0.0), 5e-4))
        records = srv.clusters()
    finally:
        srv.close()
    ok = [(i, k, r) for i, k, r in done if r["status"] == 0]
    failed = {}
    failures = []
    for i, k, r in done:
        if r["status"] != 0:
            failed[binding.status_name(r["status"])] = failed.get(binding.status_name(r["status"]), 0) + 1
            c = sessions[i]["cluster"]
            failures.append({"n": c["n"], "ns": c["ns"], "m": c["m"], "natoms": c["natoms"], "fp32": c["fp32"],
                             "seed": c["seed"], "pass": k, "status": binding.status_name(r["status"]),
                             "error": r.get("error", "")})
    lat = np.array([r["t_end"] - r["t_submit"] for _, _, r in ok])
    is32 = np.array([sessions[i]["cluster"]["fp32"] for i, _, _ in ok])
    last = {}
    for i, k, r in ok:
        if k == SERVE_STEPS - 1:
            last[i] = r["t_end"] - (t0 + sessions[i]["t_arrive"])
    sess = np.array(list(last.values()))
    span = max(r["t_end"] for _, _, r in done) - t0
    upd = sum(r["updates"] for _, _, r in ok)
    q = lambda a, p: float(np.percentile(a, p) * 1e3) if len(a) else None
    return {"rate": rate, "sessions": len(sessions), "requests": len(sessions) * SERVE_STEPS,
            "completed": len(ok), "failed": failed, "failures": failures[:8],
            "p50_ms": q(lat, 50), "p99_ms": q(lat, 99), "mean_ms": float(lat.mean() * 1e3) if len(lat) else None,
            "p50_ms_f32": q(lat[is32], 50), "p99_ms_f32": q(lat[is32], 99),
            "p50_ms_f64": q(lat[~is32], 50), "p99_ms_f64": q(lat[~is32], 99),
            "session_p50_ms": q(sess, 50), "session_p99_ms": q(sess, 99),
            "throughput_req_s": len(ok) / span, "updates_per_s": upd / span, "span_s": span,
            "max_arrival_lag_ms": lag * 1e3, "host_cluster_records_left": records[0],
            "passes": int(sum(r["passes"] for _, _, r in ok)),
            "degree_halvings": int(sum(r["halvings"] for _, _, r in ok))}


def serve_sequential_f64(setup):
    """The same sessions' work without the server: every cluster in FP64,
    one after another on one stream through the plain library calls
    (operator, Lanczos bounds, three CheFSI passes, then one pass per later
    request).  The comparison point for the served throughput."""
    import torch
    from paper_1603_04334_amd import binding, inputs
    torch.cuda.synchronize()
    upd = 0
    t0 = time.perf_counter()
    for i, (sd, c) in enumerate(setup.specs.items()):
        if i % 50 == 0:
            print(f"serving reference: cluster {i} of {len(setup.specs)}", file=sys.stderr, flush=True)
        cl = inputs.make_cluster(c["n"], c["h"], c["natoms"], c["zmax"], c["lmax"], sd)
        op = binding.Operator(cl)
        X = setup.X64[: cl.nd * c["ns"]].view(c["ns"], cl.nd).clone()
        _, _, theta = op.lanczos(KSTEPS_LANCZOS, setup.v0[: cl.nd])
        a0, a, bb = binding.select_bounds(theta, 8, ubound=op.upper_bound())
        ne = min(c["ne"], 2 * (c["ns"] - 30))
        cut = a
        for k in range(SERVE_STEPS):
            th, lf, deg = op.chefsi(X, c["m"], 3 if k == 0 else 1, ne, a0, cut, bb)
            # the library's rule between passes: a cutoff at or below a0 lowers
            # a0 to the last pass's lowest Ritz value
            for p in range(th.shape[0] - 1):
                if lf[p] + 0.1 <= a0:
                    a0 = float(th[p][0])
            cut = float(lf[-1]) + 0.1
            if cut <= a0:
                a0 = float(th[-1][0])
            upd += cl.nd * c["ns"] * int(deg.sum())
        del X, op
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"what": "the same sessions in FP64, one cluster after another through the library calls, no server",
            "seconds": dt, "updates_per_s": upd / dt, "requests_per_s": len(setup.specs) * SERVE_STEPS / dt}


def serve_measure(rates, nrequests, workers):
    import torch
    from paper_1603_04334_amd import binding
    nclusters = max(1, nrequests // SERVE_STEPS)
    setup = ServeSetup(nclusters)
    # warm-up: kernels, library handles, allocator pools
    serve_point(setup, 1e6, min(nclusters, 8), workers)
    points = []
    for r in rates:
        points.append(serve_point(setup, r, nclusters, workers))
        print(f"serving point done: {json.dumps(points[-1])}", file=sys.stderr, flush=True)
    out = {"workload": f"{nclusters} cluster sessions x {SERVE_STEPS} SCF-iteration requests (the first: Lanczos "
                       f"bounds and 3 CheFSI passes from a random block; later: one pass, cutoff = last Fermi level "
                       f"+ 0.1 Ha), grid edge log-uniform 24-128, h=0.45, 1-64 atoms, N_s = N_e/2+30, degree 20-30, "
                       f"FP32:FP64 = 80:20, Poisson session arrivals at rate/{SERVE_STEPS}, requests chained",
           "workers": workers, "budget_bytes": SERVE_BUDGET, "points": points,
           "cleared_hip_errors": int(binding.lib().sparc_cleared_hip_errors())}
    print("bench: serving reference (sequential FP64)", file=sys.stderr, flush=True)
    out["sequential_f64"] = serve_sequential_f64(setup)
    del setup
    torch.cuda.empty_cache()
    return out


def secondary(args):
    """Filter throughput of the medium cluster (96^3, 64 orbitals, m = 24) in
    FP32 and FP64 and the latency of one whole pass and of one filter on the
    small cluster (24^3, 8 orbitals, m = 20), which is latency-bound."""
    import torch
    from paper_1603_04334_amd import binding, inputs
    out = {}
    c = inputs.MEDIUM
    cl = inputs.case_cluster(c.name)
    op = binding.Operator(cl)
    med = {"workload": c.name}
    for dt in ("f32", "f64"):
        p = Pass(c, cl, op, dt)
        p.step()
        ms = timed(p.filter_only, 20, 2) * 1e3
        med[f"filter_{dt}"] = {"ms": ms, "value": cl.nd * c.ns * c.m / (ms * 1e-3)}
        if dt == "f64":
            out["_full_medium"] = (c, cl, op, p.bounds)
        del p
    out["medium"] = med
    c = inputs.SMALL
    cl = inputs.case_cluster(c.name)
    op = binding.Operator(cl)
    p = Pass(c, cl, op, "f64", tune=False)
    p.step()
    out["_full_small"] = (c, cl, op, p.bounds)
    step_ms = timed(p.step, 20, 3) * 1e3
    filt_ms = timed(p.filter_only, 50, 3) * 1e3
    out["small_latency"] = {"workload": c.name, "pass_ms": step_ms, "filter_ms": filt_ms,
                            "pass": "lanczos40_fp64+cheb_filter_fp64+rayleigh_ritz_fp64+rotation"}
    del p
    torch.cuda.empty_cache()
    return out


def _event_ms(fn, reps):
    """Average device time of fn over reps runs, HIP events on the current stream."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def next_rows(case, cl, op, dtype):
    """The rows after the filtered-subspace pass, on the same cluster: the
    first SCF iteration (three CheFSI passes from the random block, cutoff =
    last Fermi level + 0.1 Ha), one later pass, the Fermi level, the density
    of the rotated block, the nonlocal forces and the electrostatic potential
    of a neutral synthetic charge on the same grid."""
    import torch
    from paper_1603_04334_amd import binding, inputs
    dt = torch.float32 if dtype == "f32" else torch.float64
    s = 4 if dtype == "f32" else 8
    nd, ns, m = cl.nd, case.ns, case.m
    ne = 2.0 * (ns - 30)  # N_s = N_e / 2 + 30 (Sec. 4)
    out = {"electrons": ne}
    X = inputs.device_orbitals(nd, ns, case.seed, dt)
    v0 = torch.from_numpy(inputs.lanczos_start(nd, case.seed)).cuda()
    _, _, theta = op.lanczos(KSTEPS_LANCZOS, v0)
    a0, a, bb = binding.select_bounds(theta, 8, ubound=op.upper_bound())
    code = binding.SPARC_F32 if dtype == "f32" else binding.SPARC_F64
    ws = torch.empty(int(binding.lib().sparc_chefsi_workspace_bytes(op.handle, code, ns)), dtype=torch.uint8,
                     device="cuda")
    rho = torch.empty(nd, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, lf, deg = op.chefsi(X, m, 3, ne, a0, a, bb, rho=rho, ws=ws)
    t1 = time.perf_counter()
    th2, lf2, deg2 = op.chefsi(X, m, 1, ne, a0, float(lf[-1]) + 0.1, bb, ws=ws)
    t2 = time.perf_counter()
    out["first_scf"] = {"passes": 3, "ms": (t1 - t0) * 1e3, "degrees": [int(d) for d in deg],
                        "cutoffs": [a] + [float(v) + 0.1 for v in lf[:-1]], "lambda_f": [float(v) for v in lf],
                        "lowest_ritz": [float(t[0]) for t in th],
                        "density_integral": float(rho.sum().item()) * cl.h ** 3}
    out["later_pass"] = {"ms": (t2 - t1) * 1e3, "cutoff": float(lf[-1]) + 0.1, "lambda_f": float(lf2[0]),
                         "degree": int(deg2[0])}
    del ws
    # Fermi level (host)
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        lfv, occ = binding.fermi_level(th2[0], ne)
    out["fermi_level"] = {"us": (time.perf_counter() - t0) / reps * 1e6, "lambda_f": lfv, "states": ns}
    # density of the rotated block
    g = torch.from_numpy(occ).cuda()
    ms = _event_ms(lambda: binding.density(X, g, cl.h, rho=rho), 5)
    byt = s * nd * ns + 8 * nd
    out["density"] = {"ms": ms, "alg_bytes": byt, "gbs": byt / (ms * 1e-3) / 1e9,
                      "frac_of_peak": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "bytes": "s N_d N_s read + 8 N_d written"}
    # nonlocal forces
    fws = torch.empty(int(binding.lib().sparc_force_workspace_bytes(op.handle, ns)), dtype=torch.uint8,
                      device="cuda")
    f = torch.empty(len(cl.atoms), 3, dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    op.nonlocal_force(X, g, force=f, ws=fws)
    torch.cuda.synchronize()
    first = (time.perf_counter() - t0) * 1e3
    ms = _event_ms(lambda: op.nonlocal_force(X, g, force=f, ws=fws), 5)
    R = cl.radius
    pts = 0
    for at in cl.atoms:
        e = list(at.ext)
        pts += int(np.prod(e))
        for d in range(3):
            lo = max(0, at.lo[d] - R)
            hi = min(cl.n[d], at.lo[d] + at.ext[d] + R)
            ee = list(e)
            ee[d] = hi - lo
            pts += int(np.prod(ee))
    byt = s * pts * ns
    out["nonlocal_force"] = {"ms": ms, "first_call_ms_with_tables": first, "orbital_bytes_read": byt,
                             "gbs": byt / (ms * 1e-3) / 1e9, "atoms": len(cl.atoms),
                             "bytes": "s N_s per point of each atom's cube and its three widened gradient boxes"}
    del fws, X, rho
    torch.cuda.empty_cache()
    # electrostatic potential of a neutral synthetic charge on the same grid
    n = (case.n,) * 3
    h = case.h
    ax = [(torch.arange(1, case.n + 1, device="cuda", dtype=torch.float64) - 0.5 * (case.n + 1)) * h] * 3
    Xg, Yg, Zg = torch.meshgrid(*ax, indexing="ij")
    charge = torch.zeros(n, dtype=torch.float64, device="cuda")
    cen = 0.5 * (case.n + 1) * h
    for at in cl.atoms:
        r2 = (Xg - (at.pos[0] - cen)) ** 2 + (Yg - (at.pos[1] - cen)) ** 2 + (Zg - (at.pos[2] - cen)) ** 2
        for sig, q in ((0.6, -at.Z), (1.1, at.Z)):
            charge += q * torch.exp(-r2 / (2 * sig * sig)) / (2 * np.pi * sig * sig) ** 1.5
    charge = charge.reshape(-1).contiguous()
    del Xg, Yg, Zg
    P = binding.Poisson(n, h)
    pws = torch.empty(int(binding.lib().sparc_poisson_workspace_bytes(P.handle)), dtype=torch.uint8, device="cuda")
    phi = torch.zeros(nd, dtype=torch.float64, device="cuda")
    P.solve(charge, phi=phi, tol=1e-10, ws=pws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, it, res, _ = P.solve(charge, phi=phi, tol=1e-10, ws=pws)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    per_it = 14 * 8 * nd  # matvec 2, p.q 2, x/r/z update 7, p update 3 vector passes
    out["poisson"] = {"grid": list(n), "tol": 1e-10, "iterations": it, "rel_resid": res, "ms": ms,
                      "ms_per_iteration": ms / max(it, 1), "bytes_per_iteration": per_it,
                      "gbs": per_it * it / (ms * 1e-3) / 1e9, "lmax": 6, "block": [4, 4, 4]}
    del P, pws, phi, charge
    torch.cuda.empty_cache()
    return out


def cpu_baseline(case, cl, op, bounds, ncols=16):
    """The C oracle's FP64 filter on the host's OpenMP threads, on a seeded
    subset of the workload's orbitals (the first ncols columns of the same
    device-drawn block), with the bounds the GPU passes used; the metric is
    per orbital*gridpoint, so the subset's rate is the rate of the whole
    block.  The same columns are filtered on the GPU in FP64 and FP32 and
    compared with the oracle (per-orbital relative error)."""
    import torch
    import oracle
    from paper_1603_04334_amd import inputs
    a0, a, b = bounds
    X32 = inputs.device_orbitals(cl.nd, case.ns, case.seed)[:ncols].contiguous()
    Xh = X32.double().cpu().numpy()
    t0 = time.perf_counter()
    ref = oracle.cheb_filter(cl, Xh, case.m, a0, a, b)
    dt = time.perf_counter() - t0
    out = {"value": ncols * cl.nd * case.m / dt, "unit": "orbital*gridpts/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": f"FP64 C oracle Chebyshev filter (degree {case.m}) of {ncols} of the {case.ns} orbitals of "
                     f"the same cluster and bounds, {dt:.1f} s on the host; the rate of the whole block is "
                     f"extrapolated from this subset (columns are independent)"}

    def rel(g, r):
        return float((np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)).max())

    y64 = op.cheb_filter(X32.double(), case.m, a0, a, b).cpu().numpy()
    n32 = min(4, ncols)
    ref32 = oracle.cheb_filter(inputs.round_cluster_f32(cl), Xh[:n32], case.m, a0, a, b)
    y32 = op.cheb_filter(X32[:n32].contiguous(), case.m, a0, a, b).double().cpu().numpy()
    out["parity"] = {"columns_f64": ncols, "columns_f32": n32, "max_rel_err_f64": rel(y64, ref),
                     "max_rel_err_f32": rel(y32, ref32), "tolerance_f64": 1e-12, "tolerance_f32": 5e-5}
    torch.cuda.empty_cache()
    return out


def cpu_full_run(case, cl, op, bounds):
    """The C oracle's FP64 filter of a whole (small) workload on the host's
    threads, with the FP64 filter of the same block on the GPU compared
    column by column."""
    import torch
    import oracle
    from paper_1603_04334_amd import inputs
    a0, a, b = bounds
    X = inputs.device_orbitals(cl.nd, case.ns, case.seed, torch.float64)
    Xh = X.cpu().numpy()
    t0 = time.perf_counter()
    ref = oracle.cheb_filter(cl, Xh, case.m, a0, a, b)
    dt = time.perf_counter() - t0
    y = op.cheb_filter(X, case.m, a0, a, b).cpu().numpy()
    err = float((np.linalg.norm(y - ref, axis=1) / np.linalg.norm(ref, axis=1)).max())
    return {"workload": case.name, "updates": cl.nd * case.ns * case.m, "seconds": dt,
            "value": cl.nd * case.ns * case.m / dt, "gpu_fp64_max_rel_err": err}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    os.environ.setdefault("SPARC_TUNE_CACHE", TUNE_CACHE)
    import torch
    from paper_1603_04334_amd import binding, inputs
    binding.lib()
    if args.copy_calibration:
        n = 4 << 30
        a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        for _ in range(5):
            binding.stream_copy(bb, a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}))
        return
    if args.batch_only:
        print(json.dumps(batch_measure()), flush=True)
        return
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    if args.serve_only:
        print(json.dumps(serve_measure(rates, args.serve_requests, args.serve_workers)), flush=True)
        return
    case = {"large": inputs.LARGE, "medium": inputs.MEDIUM, "small": inputs.SMALL}[args.workload]
    cl = inputs.case_cluster(case.name)
    op = binding.Operator(cl)
    if args.filter_only:
        p = Pass(case, cl, op, args.dtype)
        p.step()
        for _ in range(args.warmup + args.steps):
            p.filter_only()
        torch.cuda.synchronize()
        print(json.dumps({"filter_only_runs": args.warmup + args.steps, "workload": case.name, "dtype": args.dtype}))
        return
    s = 4 if args.dtype == "f32" else 8
    updates = cl.nd * case.ns * case.m
    print(f"bench: {case.name} {args.dtype}: timing {args.steps} steps", file=sys.stderr, flush=True)
    main_res = measure_pass(case, cl, op, args.dtype, args.steps, args.warmup, kernel_stats=True)
    t_step = main_res["ms_per_step"] * 1e-3
    n_launch, ms = main_res["kernels"][0]
    n_sc, ms_sc = main_res["kernels"][2]
    n_f, ms_f = main_res["kernels"][3]
    avg_s = ms / 1e3 / max(n_launch, 1)
    alg = alg_bytes_per_step_launch(case, cl, s)
    achieved = alg / avg_s / 1e9
    copy_gbs = copy_bandwidth()
    tz, ty, cx, cg, cb = op.step_config(binding.SPARC_F32 if args.dtype == "f32" else binding.SPARC_F64, case.ns)

    out = {
        "metric": "filtered orbital*gridpts/s",
        "value": updates / t_step,
        "unit": "orbital*gridpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": case.name, "grid": [case.n] * 3, "h": case.h, "atoms": case.natoms,
                   "projectors_per_atom": (case.lmax + 1) ** 2, "orbitals": case.ns, "degree": case.m,
                   "stencil_radius": 6, "step": "lanczos40_fp64+cheb_filter+rayleigh_ritz_fp64+rotation",
                   "parallelism": "single_gpu", "tile": {"z": tz, "y": ty, "chunk_x": cx, "col_group": cg, "col_block": cb}},
        "filter_only": {"value": updates / (main_res["filter_ms"] * 1e-3), "ms": main_res["filter_ms"]},
        "stages_ms": main_res["stages_ms"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": read_traffic(args.dtype, (tz, ty, cx, cg, cb)),
                     "kernel": "fstep_kernel (vector stencil + local potential + recurrence with Y_{k-1}, with the "
                               "projector gather of Y_k in its last workgroups)",
                     "launches": n_launch, "avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg,
                     "copy_kernel_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "scatter_kernel": {"launches": n_sc, "avg_launch_us": ms_sc / max(n_sc, 1) * 1e3},
        "first_step_kernel": {"launches": n_f, "avg_launch_us": ms_f / max(n_f, 1) * 1e3},
        "bounds": list(main_res["bounds"]),
    }
    if not args.no_fp64_compare and args.dtype == "f32":
        print("bench: FP64 pass", file=sys.stderr, flush=True)
        r64 = measure_pass(case, cl, op, "f64", args.steps, args.warmup)
        out["fp64"] = {"value": updates / (r64["ms_per_step"] * 1e-3), "ms_per_step": r64["ms_per_step"],
                       "filter_only": updates / (r64["filter_ms"] * 1e-3), "filter_ms": r64["filter_ms"]}
        # the first pass of both runs starts from the same block with the same
        # (FP64 Lanczos) bounds: FP32 filter + FP64 Rayleigh-Ritz against the
        # FP64 filter + FP64 Rayleigh-Ritz
        d = np.abs(main_res["first_ritz"] - r64["first_ritz"])
        out["ritz_f32_vs_f64"] = {"max_abs_diff_ha": float(d.max()), "tolerance_ha": 1e-6,
                                  "lowest": float(main_res["first_ritz"][0])}
    if not args.no_next:
        print("bench: first SCF iteration, density, forces, electrostatic potential", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["next_rows"] = next_rows(case, cl, op, args.dtype)
    full = []
    if not args.no_secondary and args.workload == "large":
        print("bench: medium and small clusters", file=sys.stderr, flush=True)
        sec = secondary(args)
        full = [sec.pop("_full_small"), sec.pop("_full_medium")]
        out.update(sec)
    if not args.no_batch:
        print("bench: batched clusters", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["batched"] = batch_measure()
    if not args.no_serve:
        print("bench: serving", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        out["serving"] = serve_measure(rates, args.serve_requests, args.serve_workers)
    if not args.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case, cl, op, main_res["bounds"],
                                           ncols=16 if args.workload == "large" else min(case.ns, 16))
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        out["cpu_baseline"]["host_cpus"] = os.cpu_count()
        # the small and medium clusters in full (same bounds as their GPU passes)
        out["cpu_baseline"]["full_runs"] = [cpu_full_run(*f) for f in full]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
