"""Batched filters over uneven clusters: every mode reproduces the standalone
filter bit for bit (the items run the same arithmetic), and sampled results
agree with the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (grid, h, atoms, lmax, ns, m, dtype)
JOBS = [
    ((20, 20, 20), 0.45, 2, 1, 16, 16, torch.float32),
    ((24, 28, 32), 0.45, 3, 1, 24, 21, torch.float32),
    ((32, 32, 32), 0.45, 4, 1, 40, 17, torch.float32),
    ((16, 18, 20), 0.5, 0, 1, 9, 12, torch.float32),    # no atoms
    ((22, 22, 22), 0.45, 2, 2, 17, 19, torch.float64),
    ((26, 20, 24), 0.45, 3, 1, 33, 8, torch.float64),
]

# FP32 patches (tile_z, tile_y) of the vector step
SHAPES32 = [(32, 16), (32, 32), (32, 64), (64, 16), (64, 32), (80, 32), (160, 24)]


def _setup():
    from paper_1603_04334_amd import binding
    binding.lib()
    jobs = []
    for idx, (n, h, natoms, lmax, ns, m, dt) in enumerate(JOBS):
        if natoms:
            cl = inputs.make_cluster(n, h, natoms, 8, lmax, seed=40 + idx, min_dist=0.0, margin=3.0)
        else:
            cl = inputs.free_cluster(n, h, v0=-0.2)
        X = inputs.orbitals(cl.nd, ns, seed=40 + idx)
        if dt == torch.float32:
            X = inputs.round_to_f32(X)
        op = binding.Operator(cl)
        a0, a, b = -3.0 - 0.1 * idx, 1.0 + 0.2 * idx, oracle.upper_bound(cl)
        Xd = torch.from_numpy(X).to(dt).cuda()
        ref = op.cheb_filter(Xd, m, a0, a, b)
        jobs.append(dict(cl=cl, X=X, Xd=Xd, op=op, m=m, bounds=(a0, a, b), ref=ref, dt=dt))
    torch.cuda.synchronize()
    return binding, jobs


@pytest.mark.parametrize("mode", [0, 1, 2, 3, 4, 5])
def test_batch_bitwise_equals_standalone(mode):
    binding, jobs = _setup()
    outs = [torch.full_like(j["Xd"], float("nan")) for j in jobs]
    batch = binding.Batch([(j["op"], j["Xd"], o, j["m"], *j["bounds"]) for j, o in zip(jobs, outs)], mode=mode)
    for rep in range(2):  # the second run replays the captured graph in modes 0 and 4
        for o in outs:
            o.fill_(float("nan"))
        batch.run()
        assert batch.check() == 0
        torch.cuda.synchronize()
        for j, o in zip(jobs, outs):
            assert torch.equal(o, j["ref"]), (mode, rep, j["cl"].n)
    items, levels, grid = batch.info()
    if mode not in (3, 5):
        # per degree step: gather and stencil items, then scatter items
        assert items > 0 and levels == 2 * max(j["m"] for j in jobs)
    batch.close()


def test_batch_against_oracle_sampled():
    binding, jobs = _setup()
    outs = [torch.empty_like(j["Xd"]) for j in jobs]
    batch = binding.Batch([(j["op"], j["Xd"], o, j["m"], *j["bounds"]) for j, o in zip(jobs, outs)], mode=0)
    batch.run()
    assert batch.check() == 0
    for j, o in zip(jobs, outs):
        got = o[:2].double().cpu().numpy()
        if j["dt"] == torch.float32:
            ref = oracle.cheb_filter(inputs.round_cluster_f32(j["cl"]), j["X"][:2], j["m"], *j["bounds"])
            tol = 5e-5
        else:
            ref = oracle.cheb_filter(j["cl"], j["X"][:2], j["m"], *j["bounds"])
            tol = 1e-12
        err = (np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
        assert err <= tol, (j["cl"].n, err)
    batch.close()


def test_autotune_and_launch_choices():
    """The autotuner picks a patch height, an x split, a column group and a
    column block of the vector step.  The x split, the column group and the
    column block (one or two columns per workgroup; with 5 columns the last
    pair is cut short) never change a bit (the projection
    partials are kept per x-segment, whatever the split); another patch height
    sums the partials in another order, so results then agree to rounding."""
    from paper_1603_04334_amd import binding
    binding.lib()
    cl = inputs.make_cluster((30, 33, 40), 0.45, 3, 8, 1, seed=77, min_dist=0.0, margin=3.0)
    X = inputs.round_to_f32(inputs.orbitals(cl.nd, 5, seed=77))
    op = binding.Operator(cl)
    Xd = torch.from_numpy(X).float().cuda()
    bounds = (-3.0, 1.5, oracle.upper_bound(cl))
    ref = op.cheb_filter(Xd, 9, *bounds)
    assert op.step_config(binding.SPARC_F32, 5)[:2] == (32, 32)
    tz, ty, cx, cg, cb, us = op.autotune(binding.SPARC_F32, 5)
    assert us > 0 and (tz, ty) in SHAPES32 and 1 <= cx <= 30 and 1 <= cg <= 5
    assert cb in (1, 2)
    assert op.step_config(binding.SPARC_F32, 5) == (tz, ty, cx, cg, cb)
    tuned = op.cheb_filter(Xd, 9, *bounds)
    oref = oracle.cheb_filter(inputs.round_cluster_f32(cl), X, 9, *bounds)
    for tzp, ty in SHAPES32:
        base = None
        for ch, cg, cb in ((0, 0, 1), (8, 1, 2), (16, 3, 1), (30, 8, 2), (0, 2, 2)):
            if (tzp // 4) * ty > 512:
                cb = 1  # one column per workgroup on patches of more than 512 threads
            op.set_launch(binding.SPARC_F32, tzp, ty, ch, cg, cb)
            assert op.step_config(binding.SPARC_F32, 5)[:2] == (tzp, ty)
            assert op.step_config(binding.SPARC_F32, 5)[4] == cb
            got = op.cheb_filter(Xd, 9, *bounds)
            if base is None:
                base = got
            assert torch.equal(got, base), (ty, ch, cg, cb)
            g = got.double().cpu().numpy()
            err = (np.linalg.norm(g - oref, axis=1) / np.linalg.norm(oref, axis=1)).max()
            assert err <= 5e-5, (ty, ch, cg, err)
        if (tzp, ty) == (32, 32):
            assert torch.equal(base, ref)
        if (tzp, ty) == (tz, ty) == (32, 32):
            assert torch.equal(tuned, ref)
    with pytest.raises(binding.SparcError):
        op.set_launch(binding.SPARC_F32, 32, 8, 0)  # 8-row patches are FP64 only
    with pytest.raises(binding.SparcError):
        op.set_launch(binding.SPARC_F32, 32, 32, 0, 0, 3)  # one or two columns per workgroup
    with pytest.raises(binding.SparcError):
        op.set_launch(binding.SPARC_F32, 160, 24, 0, 0, 2)  # 960 threads: one column per workgroup
