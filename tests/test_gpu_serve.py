"""GPU tests of the request server (CheFSI passes on resident clusters).

A cluster's first request runs the first-SCF rule: three CheFSI passes
(Chebyshev filter, FP64 Rayleigh-Ritz, Fermi level, rotation; Sec. 3.4) from
the caller's random block, with bounds from the device Lanczos (Sec. 4);
every later request runs one pass, with the cutoff at the previous Fermi
level + 0.1 Ha (Sec. 4).  Checked:
 * the Ritz values of consecutive requests equal, bit for bit, those of the
   same library calls made directly on one stream;
 * against the FP64 oracle running the same passes: <= 1e-6 Ha (FP64 and FP32
   orbitals; every pass of an FP32 cluster runs in FP32).  For FP32 clusters
   the bound holds for the occupied states; the unconverged states above the
   Fermi level move to first order in the FP32 accumulation of the filter
   (the oracle filters in FP64 and rounds), bound 2e-5 Ha;
 * a cluster's results do not depend on what else the server runs;
 * admission never reserves more than the budget, and clusters that do not
   fit together run one after another;
 * error paths: oversize cluster, unknown ticket or cluster, duplicate
   description, and a failing cluster (Lanczos with more steps than grid
   points) that fails its own requests and leaves the others untouched.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_RITZ = 1e-6
TOL_RITZ_F32_EMPTY = 2e-5
LANCZOS_K = 40
FIRST_PASSES = 3

# (edge, h, natoms, ns, m, seed): small clusters of uneven size
CLUSTERS = [(24, 0.5, 2, 8, 12, 21), (28, 0.5, 3, 12, 14, 22), (20, 0.55, 1, 6, 10, 23),
            (32, 0.45, 4, 16, 16, 24), (26, 0.5, 2, 10, 12, 25), (30, 0.45, 3, 9, 18, 26),
            # wider blocks: the eigensolver runs in the library path (ns > 64)
            (24, 0.5, 2, 96, 12, 27), (28, 0.5, 3, 130, 14, 28), (32, 0.45, 4, 80, 16, 29),
            (26, 0.5, 2, 110, 12, 30)]
WIDE = [6, 7, 8, 9]


def _b():
    from paper_1603_04334_amd import binding
    binding.lib()
    return binding


def _cluster(i):
    n, h, na, ns, m, seed = CLUSTERS[i]
    cl = inputs.make_cluster(n, h, na, 4, 1, seed, margin=3.0, min_dist=0.0)
    return cl, ns, m, seed


def _desc(b, i, dtype=torch.float64):
    cl, ns, m, seed = _cluster(i)
    X0 = torch.from_numpy(inputs.orbitals(cl.nd, ns, seed)).to(dtype).cuda()
    v0 = torch.from_numpy(inputs.lanczos_start(cl.nd, seed)).cuda()
    torch.cuda.synchronize()
    return b.cluster_desc(cl, X0, v0, m), cl, ns, m, seed, X0, v0


def _wait(srv, tickets, timeout=120.0):
    out = {}
    t_end = time.time() + timeout
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        if time.time() > t_end:
            raise TimeoutError(f"{len(tickets) - len(out)} requests still open")
        time.sleep(0.001)
    return out


def _serve(b, ids, steps, workers=4, budget=0, dtype=torch.float64, release=True):
    """Submit `steps` requests per cluster, interleaved; returns {id: [ritz arrays]}, results."""
    srv = b.Server(workers=workers, budget=budget, lanczos_steps=LANCZOS_K)
    ritz = {i: [np.zeros(CLUSTERS[i][3]) for _ in range(steps)] for i in ids}
    descs = {i: _desc(b, i, dtype) for i in ids}
    tickets = {}
    try:
        for s in range(steps):
            for i in ids:
                d = descs[i][0] if s == 0 else None
                t = srv.submit(i, d, release=release and s == steps - 1, ritz=ritz[i][s])
                tickets[t] = (i, s)
        res = _wait(srv, list(tickets))
        st = srv.stats()
    finally:
        srv.close()
    return ritz, {tickets[t]: r for t, r in res.items()}, st


def _direct(b, i, steps, dtype=torch.float64):
    """The same passes through the library's entry points on one stream:
    three CheFSI passes for the first request, one for each later one, the
    cutoff carried as the last Fermi level + 0.1 Ha."""
    (d, keep), cl, ns, m, seed, X0, v0 = _desc(b, i, dtype)
    op = b.Operator(cl)
    _, _, theta = op.lanczos(LANCZOS_K, v0)
    a0, a, bb = b.select_bounds(theta, 8, 0.1, 1.01, op.upper_bound())
    X = X0.clone()
    out = []
    cut = a
    for s in range(steps):
        th, lf, deg = op.chefsi(X, m, FIRST_PASSES if s == 0 else 1, d.ne, a0, cut, bb)
        out.append(th[-1])
        cut = lf[-1] + 0.1
    torch.cuda.synchronize()
    return out


def _oracle(i, steps, f32=False):
    """The same passes in the oracle, with the server's precisions: Lanczos and
    Rayleigh-Ritz in FP64 on the FP64 operator; for an FP32 cluster the filter
    sees the FP32-rounded operator and block and its output, like the rotated
    orbitals, is rounded to FP32."""
    cl, ns, m, seed = _cluster(i)
    ne = _b().default_electrons(ns)
    X = inputs.orbitals(cl.nd, ns, seed)
    cl32 = inputs.round_cluster_f32(cl) if f32 else cl
    if f32:
        X = inputs.round_to_f32(X)
    _, _, theta = oracle.lanczos(cl, LANCZOS_K, inputs.lanczos_start(cl.nd, seed))
    a0, cut, bb = oracle.select_bounds(theta, 8, ubound=oracle.upper_bound(cl))
    out = []
    for s in range(steps):
        for _ in range(FIRST_PASSES if s == 0 else 1):
            Y = oracle.cheb_filter(cl32, X, m, a0, cut, bb)
            if f32:
                Y = inputs.round_to_f32(Y)
            th, vec, _, _ = oracle.rayleigh_ritz(cl, Y)
            X = oracle.rotate(Y, vec)
            if f32:
                X = inputs.round_to_f32(X)
            lf = oracle.fermi_level(th, ne)
            cut = lf + 0.1
        out.append((th, lf))
    return out


def test_serve_matches_direct_calls_bitwise():
    b = _b()
    ritz, res, _ = _serve(b, [1], 3)
    ref = _direct(b, 1, 3)
    for s in range(3):
        r = res[(1, s)]
        assert r["status"] == 0 and r["step"] == s and r["halvings"] == 0
        assert np.array_equal(ritz[1][s], ref[s]), f"step {s}"
        assert r["lambda_min"] == ref[s][0]
        n, _, _, ns, m, _ = CLUSTERS[1]
        passes = FIRST_PASSES if s == 0 else 1
        assert r["passes"] == passes and r["updates"] == n ** 3 * ns * m * passes


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_serve_oracle_parity(dtype):
    b = _b()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    ids = [0, 2, 3]
    ritz, res, _ = _serve(b, ids, 3, dtype=tdt)
    for i in ids:
        ref = _oracle(i, 3, f32=dtype == "f32")
        for s in range(3):
            assert res[(i, s)]["status"] == 0 and res[(i, s)]["halvings"] == 0
            th, lf = ref[s]
            d = np.abs(ritz[i][s] - th)
            occ = th < lf
            eo, ee = d[occ].max(), d[~occ].max()
            print(f"cluster {i} step {s} {dtype} max |dtheta| occupied {eo:.3e} empty {ee:.3e} "
                  f"|dlambda_f| {abs(res[(i, s)]['lambda_f'] - lf):.3e}")
            assert eo <= TOL_RITZ and abs(res[(i, s)]["lambda_f"] - lf) <= TOL_RITZ
            assert ee <= (TOL_RITZ if dtype == "f64" else TOL_RITZ_F32_EMPTY)


def test_serve_alone_vs_mix_bitwise():
    b = _b()
    alone, _, _ = _serve(b, [3], 4, workers=1)
    mixed, res, _ = _serve(b, list(range(6)), 4, workers=4)
    assert all(r["status"] == 0 for r in res.values())
    for s in range(4):
        assert np.array_equal(alone[3][s], mixed[3][s]), f"step {s}"
    # requests of one cluster ran in order
    for i in range(6):
        for s in range(1, 4):
            assert res[(i, s)]["t_start"] >= res[(i, s - 1)]["t_end"]


def test_serve_wide_blocks_concurrent():
    """Concurrent requests whose Rayleigh-Ritz steps all use the library
    eigensolver: results equal the one-worker run bit for bit and the oracle
    within the Ritz tolerance."""
    b = _b()
    alone = {i: _serve(b, [i], 3, workers=1)[0][i] for i in WIDE}
    mixed, res, _ = _serve(b, WIDE, 3, workers=4)
    bad = {k: (r["status"], r["error"]) for k, r in res.items() if r["status"] != 0}
    assert not bad, f"failed requests (cluster, pass) -> (status, error): {bad}"
    for i in WIDE:
        for s in range(3):
            assert np.array_equal(alone[i][s], mixed[i][s]), f"cluster {i} step {s}"
    ref = _oracle(7, 3)
    for s in range(3):
        err = np.abs(mixed[7][s] - ref[s][0]).max()
        print(f"wide cluster step {s} max |dtheta| {err:.3e}")
        assert err <= TOL_RITZ


def test_serve_admission_budget():
    b = _b()
    ids = [0, 1, 2, 3]
    foot = {}
    for i in ids:
        (d, keep), *_ = _desc(b, i)
        foot[i] = int(b.lib().sparc_cluster_footprint(b.ctypes.byref(d), LANCZOS_K))
    budget = max(foot.values()) + min(foot.values()) // 2  # far below the four together
    srv = b.Server(workers=4, budget=budget, lanczos_steps=LANCZOS_K)
    descs = {i: _desc(b, i) for i in ids}
    tickets = {}
    peak = 0
    try:
        for s in range(2):
            for i in ids:
                t = srv.submit(i, descs[i][0] if s == 0 else None, release=s == 1)
                tickets[t] = (i, s)
        out = {}
        deadline = time.time() + 120
        while len(out) < len(tickets):
            peak = max(peak, srv.stats()["hbm_used"])
            for t in tickets:
                if t not in out:
                    r = srv.poll(t)
                    if r is not None:
                        out[t] = r
            assert time.time() < deadline, "requests did not finish"
            time.sleep(0.0005)
        st = srv.stats()
        recs = srv.clusters()
    finally:
        srv.close()
    assert peak <= budget
    # every session ended with a release: no host record of a cluster remains
    assert recs == (0, len(ids))
    assert st["hbm_used"] == 0 and st["pending"] == 0 and st["running"] == 0
    res = {tickets[t]: r for t, r in out.items()}
    assert all(r["status"] == 0 for r in res.values())
    # a cluster holds its reservation at least from its first start to its last
    # end: at every start, the clusters holding one must fit the budget together
    spans = {i: (res[(i, 0)]["t_start"], res[(i, 1)]["t_end"]) for i in ids}
    most = 0
    for i in ids:
        t = spans[i][0]
        live = [j for j in ids if spans[j][0] <= t <= spans[j][1]]
        assert sum(foot[j] for j in live) <= budget, f"resident together beyond the budget: {live}"
        most = max(most, len(live))
    assert most < len(ids)


def test_serve_errors_and_failure_isolation():
    b = _b()
    from paper_1603_04334_amd.binding import SparcError
    SPARC_E_ARG, SPARC_E_NOMEM, SPARC_E_TICKET, SPARC_E_JOB = -1, -4, -7, -8
    # oversize: a budget below one cluster's footprint
    srv = b.Server(workers=2, budget=1 << 20, lanczos_steps=LANCZOS_K)
    try:
        (d, keep), *_ = _desc(b, 0)
        with pytest.raises(SparcError) as e:
            srv.submit(0, (d, keep))
        assert e.value.status == SPARC_E_NOMEM
    finally:
        srv.close()

    srv = b.Server(workers=3, lanczos_steps=LANCZOS_K)
    try:
        with pytest.raises(SparcError) as e:
            srv.poll(12345)
        assert e.value.status == SPARC_E_TICKET
        with pytest.raises(SparcError) as e:
            srv.submit(77)  # unknown cluster without a description
        assert e.value.status == SPARC_E_ARG
        # a 3^3 grid has fewer points than Lanczos steps: its first request fails
        bad = inputs.free_cluster(3, 0.5, radius=1)
        Xb = torch.randn(2, bad.nd, dtype=torch.float64, device="cuda")
        vb = torch.randn(bad.nd, dtype=torch.float64, device="cuda")
        good = _desc(b, 2)
        torch.cuda.synchronize()
        tg0 = srv.submit(2, good[0])
        with pytest.raises(SparcError) as e:
            srv.submit(2, good[0])  # duplicate description
        assert e.value.status == SPARC_E_ARG
        tb0 = srv.submit(9, b.cluster_desc(bad, Xb, vb, 4))
        tb1 = srv.submit(9)
        tg1 = srv.submit(2, release=True)
        res = _wait(srv, [tg0, tb0, tb1, tg1])
        assert res[tb0]["status"] == SPARC_E_ARG and "N_d" in res[tb0]["error"]
        assert res[tb1]["status"] == SPARC_E_JOB
        with pytest.raises(SparcError) as e:
            srv.submit(9)
        assert e.value.status == SPARC_E_JOB
        assert res[tg0]["status"] == 0 and res[tg1]["status"] == 0
        with pytest.raises(SparcError) as e:
            srv.poll(tg0)  # retired
        assert e.value.status == SPARC_E_TICKET
        assert srv.stats()["hbm_used"] == 0
        # both clusters are finished (one released, one failed): their host
        # records are gone and only their ids are kept
        assert srv.clusters() == (0, 2)
    finally:
        srv.close()
    # the good cluster's results equal those of a run without the failing one
    ref = _direct(b, 2, 2)
    assert res[tg0]["lambda_min"] == ref[0][0] and res[tg1]["lambda_min"] == ref[1][0]
