"""GPU parity of the nonlocal atomic forces (Sec. 3.6, Eqs. NonlocForce:Discrete
and NonLocForce:U:W, Alg. 4) through sparc_nonlocal_force against the oracle.

The library contracts each orbital with chi and with -grad_h chi (exactly
equal to contracting grad_h psi with chi under zero padding); the oracle
forms grad_h psi as the paper does.  Both sum in FP64 (an FP32 block is
widened exactly on both sides), so they differ by rounding order only, in
sums whose terms cancel: the bound is 1e-10 of the largest force component
(the rounding level of 1e5-term FP64 sums of terms up to ~100 times the
result is about 1e-12)."""
import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


def _b():
    from paper_1603_04334_amd import binding
    binding.lib()
    return binding


def _occ(ns, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.uniform(0.0, 1.0, ns))[::-1].copy()


def _check(cl, X, occ, dtype, label):
    b = _b()
    op = b.Operator(cl)
    Xd = torch.from_numpy(X).to(dtype).cuda()
    g = torch.from_numpy(occ).cuda()
    f = op.nonlocal_force(Xd, g)
    f2 = op.nonlocal_force(Xd, g)  # tables already built: the asynchronous path
    torch.cuda.synchronize()
    got, got2 = f.cpu().numpy(), f2.cpu().numpy()
    ref = oracle.nonlocal_force(cl, Xd.double().cpu().numpy(), occ)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"force {label} {dtype} natoms {len(cl.atoms)} ns {X.shape[0]}: max |f| {np.abs(ref).max():.3e} "
          f"rel err {err:.2e}", flush=True)
    assert np.array_equal(got, got2)
    assert err <= TOL
    return got


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_force_small(dtype):
    c = inputs.SMALL
    cl = inputs.case_cluster(c.name)
    _check(cl, inputs.orbitals(cl.nd, c.ns, c.seed), _occ(c.ns, 1), dtype, "24^3")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_force_nine_projectors_and_wall_cubes(dtype):
    """l <= 2 (9 projectors per atom), 37 orbitals (three 16-column tiles,
    ragged), atoms 1 bohr from the walls so that cubes and their widened
    gradient boxes are clipped by the grid."""
    cl = inputs.make_cluster((30, 26, 34), 0.45, 7, 6, 2, seed=13, min_dist=1.0, margin=1.0)
    assert any(a.lo[d] == 0 or a.lo[d] + a.ext[d] == cl.n[d] for a in cl.atoms for d in range(3))
    _check(cl, inputs.orbitals(cl.nd, 37, 13), _occ(37, 2), dtype, "30x26x34 l<=2")


def test_force_no_atoms_and_errors():
    b = _b()
    free = inputs.free_cluster(12, 0.5)
    op = b.Operator(free)
    X = torch.ones(2, free.nd, dtype=torch.float64, device="cuda")
    g = torch.ones(2, dtype=torch.float64, device="cuda")
    assert op.nonlocal_force(X, g).shape == (0, 3)
    c = inputs.SMALL
    cl = inputs.case_cluster(c.name)
    op = b.Operator(cl)
    X = torch.from_numpy(inputs.orbitals(cl.nd, 4, 1)).cuda()
    g = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(b.SparcError) as ei:
        op.nonlocal_force(X, g, ws=torch.empty(64, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == b.SPARC_E_WORKSPACE
    f = torch.empty(len(cl.atoms), 3, dtype=torch.float64, device="cuda")
    with pytest.raises(b.SparcError) as ei:
        op.nonlocal_force(X, g, force=X.view(-1)[:6].view(2, 3))
    assert ei.value.status == b.SPARC_E_ALIAS
    op.nonlocal_force(X, g, force=f)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_force_full_workload_sampled_orbitals(dtype):
    """The 160^3 grid with 128 atoms x 9 projectors and 600 orbitals drawn on
    the device: the library runs over all 600 columns with the occupations of
    four sampled orbitals nonzero (the first, the last and two between), and
    the oracle computes the forces of those four."""
    b = _b()
    c = inputs.LARGE
    cl = inputs.case_cluster(c.name)
    X = inputs.device_orbitals(cl.nd, c.ns, 37, dtype=dtype)
    pick = [0, 211, 457, c.ns - 1]
    occ = np.zeros(c.ns)
    occ[pick] = [1.0, 0.8, 0.35, 0.05]
    op = b.Operator(cl)
    f = op.nonlocal_force(X, torch.from_numpy(occ).cuda())
    cols = X[pick].double().cpu().numpy()
    torch.cuda.synchronize()
    got = f.cpu().numpy()
    del X
    torch.cuda.empty_cache()
    ref = oracle.nonlocal_force(cl, cols, occ[pick])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"force 160^3 x {c.ns} {dtype}, 4 occupied: max |f| {np.abs(ref).max():.3e} rel err {err:.2e}", flush=True)
    assert err <= TOL
