"""Benchmark of the Chebyshev-filter hot path on one MI355X.

Workload: the medium synthetic cluster (96^3 grid, h = 0.4 bohr, 16 atoms with
4 Kleinman-Bylander projectors each, 64 orbitals N(0,1), degree m = 24,
stencil order 12).  One step is one filtered-subspace pass over the resident
orbital block: 40-step FP64 Lanczos bounds on the device, the Chebyshev filter
in the selected dtype, FP64 Rayleigh-Ritz on the device and the subspace
rotation; each pass starts from the orbitals the previous one rotated.  ``value`` is filtered orbital*gridpoint updates per second of the
whole step (N_d * N_s * m / step time).

Prints ONE JSON line (rank 0).  Defaults: 1 GPU, 10 timed steps, 3 warmup.
Modes: --dtype f32 (default; FP64 also measured and reported beside it) or f64.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic_cluster96.txt")
STENCIL_SRCS = [os.path.join(ROOT, "paper_1603_04334_amd", "csrc", f) for f in ("stencil.hip", "step_kernel.hpp")]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--dtype", choices=["f32", "f64"], default="f32")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-fp64-compare", action="store_true")
    p.add_argument("--no-batch", action="store_true", help="skip the batched uneven-cluster measurement")
    p.add_argument("--batch-only", action="store_true", help="print only the batched measurement")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--serve-only", action="store_true", help="print only the serving measurement")
    p.add_argument("--serve-rates", default="50",
                   help="comma-separated Poisson arrival rates in requests/s (full sweep: 50,100,200,500,1000,2000)")
    p.add_argument("--serve-requests", type=int, default=500, help="requests per rate point (5 per cluster)")
    p.add_argument("--serve-workers", type=int, default=4)
    p.add_argument("--copy-calibration", action="store_true",
                   help="run only a plain device copy of known size (for counter calibration)")
    return p.parse_args()


def source_hash() -> str:
    """Hash of the step kernel's sources (launch code and kernel body)."""
    h = hashlib.sha256()
    for f in STENCIL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(dtype):
    """HBM bytes per recurrence-step launch from committed counter runs, or
    None when absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("stencil_sha256_16") != source_hash():
        return None
    try:
        return float(kv[f"{dtype}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    import torch
    n = 1 << 28  # 256 Mi floats = 1 GiB read + 1 GiB written
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}))


class Pass:
    """Resident state of one workload and one dtype."""

    def __init__(self, case, cluster, dtype):
        import torch
        from paper_1603_04334_amd import binding, inputs
        self.binding = binding
        self.case = case
        self.cl = cluster
        self.dt = torch.float32 if dtype == "f32" else torch.float64
        self.code = binding.SPARC_F32 if dtype == "f32" else binding.SPARC_F64
        self.op = binding.Operator(cluster)
        X = inputs.orbitals(cluster.nd, case.ns, case.seed)
        self.X = torch.from_numpy(X).to(self.dt).cuda()
        del X
        self.Y = torch.empty_like(self.X)
        self.R = torch.empty_like(self.X)
        self.v0 = torch.from_numpy(inputs.lanczos_start(cluster.nd, case.seed)).cuda()
        self.ws = self.op.workspace(self.code, case.ns, 1)
        self.ub = self.op.upper_bound()
        self.bounds = None
        self.ritz = None

    def step(self, profile_filter=False):
        b = self.binding
        _, _, theta = self.op.lanczos(KSTEPS_LANCZOS, self.v0)
        a0, a, bb = b.select_bounds(theta, 8, ubound=self.ub)
        self.bounds = (a0, a, bb)
        if profile_filter:
            b.profile.enable(True)
        self.op.cheb_filter(self.X, self.case.m, a0, a, bb, Y=self.Y, ws=self.ws)
        if profile_filter:
            b.profile.enable(False)
        self.ritz, Qt = self.op.rayleigh_ritz(self.Y)
        b.rotate(self.Y, Qt, out=self.R)
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


def alg_bytes_per_step_launch(case, cl, s):
    """Algorithmic HBM bytes of one recurrence-step launch, which runs the
    fused step and the projector gather of the same Y_k: read Y_k and Y_{k-1},
    write Y_{k+1} (s bytes per orbital*gridpoint each), read V_eff once (s
    bytes per gridpoint); the gather reads Y_k at the cube points again (s per
    orbital*cube point), chi once per group of 16 orbitals (s per cube point
    and projector) and writes its 8 split partials (s per projector and
    orbital each)."""
    cube = sum(int(np.prod(a.ext)) for a in cl.atoms)
    chi = sum(int(np.prod(a.ext)) * a.nproj for a in cl.atoms)
    ncb = (case.ns + 15) // 16
    gather = s * (case.ns * cube + ncb * chi + 8 * cl.nproj_total * case.ns)
    return 3 * s * cl.nd * case.ns + s * cl.nd + gather


def batch_measure(reps=5, nclusters=64):
    """Batched uneven clusters (grid edge in {32..96}, h = 0.45, 2-24 atoms,
    16-128 orbitals, degree 16-28), FP32 with FP64 coefficients.  Bounds come
    from the device Lanczos (setup, untimed); orbitals are seeded N(0,1) drawn
    on the device.  Returns throughput of each execution mode and of the plain
    unbatched FP64 filters on the same clusters."""
    import torch
    from paper_1603_04334_amd import binding, inputs
    recipe = inputs.batch_recipe(nclusters=nclusters)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4)
    jobs32, jobs64, ops, work = [], [], [], 0
    for r in recipe:
        cl = inputs.make_cluster(r["n"], r["h"], r["natoms"], r["zmax"], r["lmax"], r["seed"])
        op = binding.Operator(cl)
        _, _, theta = op.lanczos(KSTEPS_LANCZOS, torch.from_numpy(inputs.lanczos_start(cl.nd, r["seed"])).cuda())
        a0, a, b = binding.select_bounds(theta, 8, ubound=op.upper_bound())
        op.autotune(binding.SPARC_F32, r["ns"])
        X = torch.randn((r["ns"], cl.nd), generator=gen, device="cuda", dtype=torch.float32)
        jobs32.append((op, X, torch.empty_like(X), r["m"], a0, a, b))
        X64 = X.double()
        jobs64.append((op, X64, torch.empty_like(X64), r["m"], a0, a, b))
        ops.append(op)
        work += cl.nd * r["ns"] * r["m"]
    out = {"workload": f"{nclusters} uneven clusters, grid edge 32-96, h=0.45, 16-128 orbitals, degree 16-28",
           "updates_per_run": work}
    for name, jobs, mode in (("persistent_graph_f32", jobs32, 0), ("grouped_levels_graph_f32", jobs32, 4),
                             ("sequential_f32", jobs32, 3), ("sequential_f64", jobs64, 3)):
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
    for k in ("persistent_graph_f32", "grouped_levels_graph_f32", "sequential_f32"):
        out[k]["vs_sequential_f64"] = out[k]["value"] / out["sequential_f64"]["value"]
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
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        self.X64 = torch.randn(maxnd * maxns, generator=gen, device="cuda", dtype=torch.float64)
        self.X32 = self.X64.float() if any(c["fp32"] for c in specs.values()) else None
        self.v0 = torch.randn(maxnd, generator=gen, device="cuda", dtype=torch.float64)
        torch.cuda.synchronize()
        self.descs = {}
        for sd, c in specs.items():
            cl = inputs.make_cluster(c["n"], c["h"], c["natoms"], c["zmax"], c["lmax"], sd)
            src = self.X32 if c["fp32"] else self.X64
            X0 = src[: cl.nd * c["ns"]].view(c["ns"], cl.nd)
            self.descs[sd] = binding.cluster_desc(cl, X0, self.v0[: cl.nd], c["m"])


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
    failed_sessions = {}
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
                if r["status"] != 0:
                    failed_sessions[i] = r["status"]
                elif k + 1 < SERVE_STEPS:
                    c = sessions[i]["cluster"]
                    open_t[srv.submit(c["seed"], release=k + 2 == SERVE_STEPS)] = (i, k + 1)
            if time.time() > deadline:
                raise RuntimeError("serving run did not finish")
            wait = (t0 + sessions[nxt]["t_arrive"] - binding.clock()) if nxt < len(sessions) else 1e-3
            time.sleep(min(max(wait, 0.0), 5e-4))
    finally:
        srv.close()
    ok = [(i, k, r) for i, k, r in done if r["status"] == 0]
    failed = {}
    for i, k, r in done:
        if r["status"] != 0:
            failed[binding.status_name(r["status"])] = failed.get(binding.status_name(r["status"]), 0) + 1
    failures = []
    for i, k, r in done:
        if r["status"] != 0:
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
            "max_arrival_lag_ms": lag * 1e3}


def serve_measure(rates, nrequests, workers):
    import torch
    nclusters = max(1, nrequests // SERVE_STEPS)
    setup = ServeSetup(nclusters)
    # warm-up: kernels, library handles, allocator pools
    serve_point(setup, 1e6, min(nclusters, 8), workers)
    points = []
    for r in rates:
        points.append(serve_point(setup, r, nclusters, workers))
        print(f"serving point done: {json.dumps(points[-1])}", file=sys.stderr, flush=True)
    out = {"workload": f"{nclusters} cluster sessions x {SERVE_STEPS} filtered-subspace passes (Lanczos bounds on "
                       f"the first), grid edge log-uniform 24-128, h=0.45, 1-64 atoms, N_s = N_e/2+30, degree 20-30, "
                       f"FP32:FP64 = 80:20, Poisson session arrivals at rate/{SERVE_STEPS}, passes chained",
           "workers": workers, "budget_bytes": SERVE_BUDGET, "points": points}
    del setup
    torch.cuda.empty_cache()
    return out


def cpu_baseline(case, cl):
    """The C oracle's FP64 filter on the host, in groups of 8 orbitals of the
    same cluster until about 10 s of work (or all orbitals) are done."""
    import oracle
    from paper_1603_04334_amd import inputs
    a0, a, b = -2.0, 3.0, oracle.upper_bound(cl)
    done, dt = 0, 0.0
    while done < case.ns and dt < 10.0:
        cols = list(range(done, min(case.ns, done + 8)))
        X = inputs.orbitals(cl.nd, case.ns, case.seed, cols=cols)
        t0 = time.perf_counter()
        oracle.cheb_filter(cl, X, case.m, a0, a, b)
        dt += time.perf_counter() - t0
        done += len(cols)
    return {"value": done * cl.nd * case.m / dt, "unit": "orbital*gridpts/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"FP64 C oracle Chebyshev filter (degree {case.m}) of {done} of the {case.ns} "
                      f"orbitals of the same cluster, {dt:.1f} s on the host"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration()
        return
    from paper_1603_04334_amd import binding, inputs
    binding.lib()
    if args.batch_only:
        print(json.dumps(batch_measure()), flush=True)
        return
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    if args.serve_only:
        print(json.dumps(serve_measure(rates, args.serve_requests, args.serve_workers)), flush=True)
        return
    case = inputs.MEDIUM
    cl = inputs.case_cluster(case.name)
    s = 4 if args.dtype == "f32" else 8

    main_pass = Pass(case, cl, args.dtype)
    # timed region: K whole steps
    t_step = timed(main_pass.step, args.steps, args.warmup)
    updates = cl.nd * case.ns * case.m
    # kernel timing: the same steps again with per-launch events on the filter's kernels
    binding.profile.reset()
    torch.cuda.synchronize()
    for _ in range(args.steps):
        main_pass.step(profile_filter=True)
    torch.cuda.synchronize()
    n_launch, ms = binding.profile.read(0)
    n_g, ms_g = binding.profile.read(1)
    n_sc, ms_sc = binding.profile.read(2)
    n_f, ms_f = binding.profile.read(3)
    binding.profile.reset()
    avg_s = ms / 1e3 / max(n_launch, 1)
    alg = alg_bytes_per_step_launch(case, cl, s)
    achieved = alg / avg_s / 1e9
    traffic = read_traffic(args.dtype)
    t_filter = timed(main_pass.filter_only, args.steps, 1)

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
                   "parallelism": "single_gpu"},
        "filter_only": {"value": updates / t_filter, "ms": t_filter * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "step_gather_kernel (fused stencil + local potential + recurrence with Y_{k-1}, and the projector gather of Y_k)",
                     "launches": n_launch, "avg_launch_us": avg_s * 1e6,
                     "alg_bytes_per_launch": alg},
        "gather_kernel": {"launches": n_g, "avg_launch_us": ms_g / max(n_g, 1) * 1e3},
        "scatter_kernel": {"launches": n_sc, "avg_launch_us": ms_sc / max(n_sc, 1) * 1e3},
        "first_step_kernel": {"launches": n_f, "avg_launch_us": ms_f / max(n_f, 1) * 1e3},
        "bounds": list(main_pass.bounds),
    }
    tz, ty, cx = main_pass.op.step_config(main_pass.code, case.ns)
    out["config"]["tile"] = {"z": tz, "y": ty, "chunk_x": cx}
    if not args.no_fp64_compare and args.dtype == "f32":
        del main_pass
        torch.cuda.empty_cache()
        p64 = Pass(case, cl, "f64")
        t64 = timed(p64.step, args.steps, args.warmup)
        t64f = timed(p64.filter_only, args.steps, 1)
        out["fp64"] = {"value": updates / t64, "ms_per_step": t64 * 1e3, "filter_only": updates / t64f,
                       "filter_ms": t64f * 1e3}
        del p64
    if not args.no_batch:
        torch.cuda.empty_cache()
        out["batched"] = batch_measure()
    if not args.no_serve:
        torch.cuda.empty_cache()
        out["serving"] = serve_measure(rates, args.serve_requests, args.serve_workers)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, cl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
