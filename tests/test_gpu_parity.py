"""GPU parity: the HIP library (through the C ABI) against the CPU FP64 oracle.

Tolerances (per orbital, max over orbitals of |Y - Y_ref|_2 / |Y_ref|_2):
FP64 <= 1e-12, FP32 <= 5e-5 (the FP32 run and the oracle see the same
FP32-rounded X, V_eff and chi; the oracle computes in FP64).  Ritz values:
<= 1e-6 Ha.
"""
import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 5e-5
TOL_RITZ = 1e-6


def _b():
    from paper_1603_04334_amd import binding
    binding.lib()
    return binding


def rel_err(Y, Yref):
    Y = np.asarray(Y, dtype=np.float64)
    num = np.linalg.norm(Y - Yref, axis=1)
    den = np.linalg.norm(Yref, axis=1)
    return float((num / den).max())


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _bounds(cl, seed, k=40):
    _, _, theta = oracle.lanczos(cl, min(k, cl.nd), inputs.lanczos_start(cl.nd, seed))
    return oracle.select_bounds(theta, 8, ubound=oracle.upper_bound(cl))


@pytest.fixture(scope="module")
def small():
    c = inputs.SMALL
    cl = inputs.case_cluster(c.name)
    X = inputs.orbitals(cl.nd, c.ns, c.seed)
    return c, cl, X, _bounds(cl, c.seed)


def test_h_apply_small_f64(small):
    c, cl, X, _ = small
    op = _b().Operator(cl)
    Y = host(op.h_apply(dev(X)))
    print("h_apply f64 err", rel_err(Y, oracle.h_apply(cl, X)))
    assert rel_err(Y, oracle.h_apply(cl, X)) <= TOL64


def test_h_apply_small_f32(small):
    c, cl, X, _ = small
    op = _b().Operator(cl)
    X32 = inputs.round_to_f32(X)
    Y = host(op.h_apply(dev(X32, torch.float32)))
    ref = oracle.h_apply(inputs.round_cluster_f32(cl), X32)
    print("h_apply f32 err", rel_err(Y, ref))
    assert rel_err(Y, ref) <= TOL32


def test_filter_small_f64(small):
    c, cl, X, (a0, a, b) = small
    op = _b().Operator(cl)
    Y = host(op.cheb_filter(dev(X), c.m, a0, a, b))
    ref = oracle.cheb_filter(cl, X, c.m, a0, a, b)
    print("filter f64 err", rel_err(Y, ref))
    assert rel_err(Y, ref) <= TOL64


def test_filter_small_f32(small):
    c, cl, X, (a0, a, b) = small
    op = _b().Operator(cl)
    X32 = inputs.round_to_f32(X)
    Y = host(op.cheb_filter(dev(X32, torch.float32), c.m, a0, a, b))
    ref = oracle.cheb_filter(inputs.round_cluster_f32(cl), X32, c.m, a0, a, b)
    print("filter f32 err", rel_err(Y, ref))
    assert rel_err(Y, ref) <= TOL32


RAGGED = [
    # (grid, h, natoms, lmax, ns, radius, m)
    ((13, 17, 29), 0.5, 2, 1, 3, 6, 7),
    ((12, 40, 33), 0.45, 3, 2, 1, 6, 5),
    ((20, 70, 65), 0.4, 4, 1, 5, 6, 4),
    ((11, 12, 10), 0.7, 1, 2, 17, 3, 6),
    ((16, 16, 16), 0.6, 2, 1, 2, 1, 9),
    ((4, 5, 3), 1.0, 0, 1, 2, 6, 3),      # grid smaller than the stencil radius, no atoms
]


@pytest.mark.parametrize("case", RAGGED, ids=[f"{c[0]}-r{c[5]}-ns{c[4]}" for c in RAGGED])
def test_ragged_shapes_and_padded_ld(case):
    n, h, natoms, lmax, ns, radius, m = case
    if natoms:
        cl = inputs.make_cluster(n, h, natoms, 8, lmax, seed=sum(n), min_dist=0.0, margin=2.5, radius=radius)
    else:
        cl = inputs.free_cluster(n, h, v0=-0.3, radius=radius)
    rng = np.random.default_rng(len(n) + ns)
    X = rng.standard_normal((ns, cl.nd))
    op = _b().Operator(cl)
    # leading dimension larger than N_d
    big = torch.zeros((ns, cl.nd + 37), dtype=torch.float64, device="cuda")
    big[:, : cl.nd] = dev(X)
    Xv = big[:, : cl.nd]
    outbig = torch.full((ns, cl.nd + 5), 7.0, dtype=torch.float64, device="cuda")
    Yv = outbig[:, : cl.nd]
    op.h_apply(Xv, Yv)
    got = host(Yv)
    assert rel_err(got, oracle.h_apply(cl, X)) <= TOL64
    assert torch.all(outbig[:, cl.nd:] == 7.0)  # padding untouched
    a0, a, b = -3.0, 2.0, oracle.upper_bound(cl)
    Yf = host(op.cheb_filter(Xv, m, a0, a, b))
    assert rel_err(Yf, oracle.cheb_filter(cl, X, m, a0, a, b)) <= TOL64


def test_edge_atom_touching_walls():
    # projector cubes that start at node 0 and end at the last node
    cl = inputs.make_cluster((14, 15, 16), 0.45, 3, 8, 2, seed=5, min_dist=0.0, margin=1.0)
    assert any(min(a.lo) == 0 or any(a.lo[d] + a.ext[d] == cl.n[d] for d in range(3)) for a in cl.atoms)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((4, cl.nd))
    op = _b().Operator(cl)
    assert rel_err(host(op.h_apply(dev(X))), oracle.h_apply(cl, X)) <= TOL64


def test_medium_sampled_columns():
    # the full medium workload on the GPU; two sampled columns by the oracle
    c = inputs.MEDIUM
    cl = inputs.case_cluster(c.name)
    a0, a, b = _bounds(cl, c.seed)
    X = inputs.orbitals(cl.nd, c.ns, c.seed)
    cols = [0, 37]
    op = _b().Operator(cl)
    Y64 = host(op.cheb_filter(dev(X), c.m, a0, a, b))
    ref = oracle.cheb_filter(cl, X[cols], c.m, a0, a, b)
    e64 = rel_err(Y64[cols], ref)
    X32 = inputs.round_to_f32(X)
    Y32 = host(op.cheb_filter(dev(X32, torch.float32), c.m, a0, a, b))
    ref32 = oracle.cheb_filter(inputs.round_cluster_f32(cl), X32[cols], c.m, a0, a, b)
    e32 = rel_err(Y32[cols], ref32)
    print("medium sampled errors f64 %.3e f32 %.3e" % (e64, e32))
    assert e64 <= TOL64 and e32 <= TOL32
    # property at full size: columns are independent, so filtering a single
    # column alone reproduces its value in the full launch bit for bit
    one = host(op.cheb_filter(dev(X[cols[1]:cols[1] + 1]), c.m, a0, a, b))
    assert np.array_equal(one[0], Y64[cols[1]])


def test_alone_vs_mix_bitwise(small):
    c, cl, X, (a0, a, b) = small
    op = _b().Operator(cl)
    full = host(op.cheb_filter(dev(X), c.m, a0, a, b))
    for i in (0, 5):
        alone = host(op.cheb_filter(dev(X[i:i + 1]), c.m, a0, a, b))
        assert np.array_equal(alone[0], full[i])
    again = host(op.cheb_filter(dev(X), c.m, a0, a, b))
    assert np.array_equal(again, full)  # deterministic


def test_lanczos_parity(small):
    c, cl, X, _ = small
    op = _b().Operator(cl)
    v0 = inputs.lanczos_start(cl.nd, c.seed)
    alpha, beta, theta = op.lanczos(40, dev(v0))
    ra, rb, rt = oracle.lanczos(cl, 40, v0)
    print("lanczos max |dtheta|", np.abs(theta - rt).max())
    assert np.abs(theta - rt).max() <= TOL_RITZ
    assert np.abs(alpha - ra).max() <= 1e-8 and np.abs(beta - rb).max() <= 1e-8
    ub = op.upper_bound()
    assert abs(ub - oracle.upper_bound(cl)) <= 1e-9 * abs(ub)
    from paper_1603_04334_amd import binding
    got = binding.select_bounds(theta, 8, ubound=ub)
    ref = oracle.select_bounds(rt, 8, ubound=oracle.upper_bound(cl))
    assert np.allclose(got, ref, rtol=0, atol=TOL_RITZ)


def test_rayleigh_ritz_and_rotation(small):
    c, cl, X, (a0, a, b) = small
    op = _b().Operator(cl)
    ref_filtered = oracle.cheb_filter(cl, X, c.m, a0, a, b)
    rt, rvec, _, _ = oracle.rayleigh_ritz(cl, ref_filtered)
    # FP64 RR on the oracle's block
    theta, Qt = op.rayleigh_ritz(dev(ref_filtered))
    print("RR f64 max |dtheta|", np.abs(theta - rt).max())
    assert np.abs(theta - rt).max() <= TOL_RITZ
    # FP32 filter on the GPU + FP64 RR on the GPU vs the FP64 oracle pipeline
    Y32 = op.cheb_filter(dev(inputs.round_to_f32(X), torch.float32), c.m, a0, a, b)
    theta32, _ = op.rayleigh_ritz(Y32)
    print("FP32 filter + FP64 RR max |dtheta|", np.abs(theta32 - rt).max())
    assert np.abs(theta32 - rt).max() <= TOL_RITZ
    # rotation with the GPU's eigenvectors, checked against the oracle's GEMM
    from paper_1603_04334_amd import binding
    Yd = dev(ref_filtered)
    R = host(binding.rotate(Yd, Qt))
    Q = host(Qt).T
    assert rel_err(R, oracle.rotate(ref_filtered, Q)) <= 1e-12
    # the rotated block is M-orthonormal: R R^T = I
    assert np.abs(R @ R.T - np.eye(c.ns)).max() < 1e-9


def test_argument_errors(small):
    c, cl, X, (a0, a, b) = small
    binding = _b()
    op = binding.Operator(cl)
    Xd = dev(X)
    with pytest.raises(binding.SparcError) as e:
        op.cheb_filter(Xd, 0, a0, a, b)
    assert e.value.status == binding.SPARC_E_BOUNDS
    with pytest.raises(binding.SparcError) as e:
        op.cheb_filter(Xd, 5, a, a0, b)
    assert e.value.status == binding.SPARC_E_BOUNDS
    with pytest.raises(binding.SparcError) as e:
        op.cheb_filter(Xd, 5, a0, a, b, ws=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.status == binding.SPARC_E_WORKSPACE
    with pytest.raises(binding.SparcError) as e:
        op.h_apply(Xd, Xd)
    assert e.value.status == binding.SPARC_E_ALIAS
    lib = binding.lib()
    ws = op.workspace(0, c.ns, 1)
    Y = torch.empty_like(Xd)
    st = lib.sparc_cheb_filter(op.handle, 0, Xd.data_ptr(), cl.nd - 1, Y.data_ptr(), cl.nd, c.ns, 5, a0, a, b,
                               ws.data_ptr(), ws.numel(), None)
    assert st == binding.SPARC_E_SHAPE
    st = lib.sparc_h_apply(op.handle, 7, Xd.data_ptr(), cl.nd, Y.data_ptr(), cl.nd, c.ns, ws.data_ptr(), ws.numel(), None)
    assert st == binding.SPARC_E_ARG
    # the projection addresses points by 32-bit offsets from a pass's first
    # column: a leading dimension with 8 ldy + nd >= 2^32 is refused before
    # anything is read
    theta = np.zeros(c.ns)
    for ldy, want in ((cl.nd - 1, binding.SPARC_E_SHAPE), ((1 << 29), binding.SPARC_E_SHAPE)):
        st = lib.sparc_rayleigh_ritz(op.handle, 0, Xd.data_ptr(), ldy, c.ns, theta.ctypes.data_as(binding._dp), None,
                                     ws.data_ptr(), ws.numel(), None)
        assert st == want, ldy


@pytest.mark.parametrize("ns", [1, 7, 33, 64, 70])
def test_rayleigh_ritz_sizes(ns):
    # one-workgroup Jacobi path (ns <= 64) and library path (ns > 64)
    cl = inputs.make_cluster(16, 0.5, 2, 4, 1, seed=21, min_dist=0.0, margin=3.0)
    rng = np.random.default_rng(ns)
    Y = rng.standard_normal((ns, cl.nd))
    rt, _, Hs, Ms = oracle.rayleigh_ritz(cl, Y)
    op = _b().Operator(cl)
    theta, Qt = op.rayleigh_ritz(dev(Y))
    assert np.abs(theta - rt).max() <= TOL_RITZ * max(1.0, np.abs(rt).max() * 1e-3)
    Q = host(Qt).T
    # M-orthonormal eigenvectors of the oracle's projected pencil
    assert np.abs(Q.T @ Ms @ Q - np.eye(ns)).max() < 1e-9
    assert np.abs(Hs @ Q - Ms @ Q * theta).max() < 1e-8 * max(1.0, np.abs(Hs).max())
    # a padded leading dimension (even, so H Y takes the same vector launch)
    # changes only the addresses: the same Ritz values and vectors bit for bit
    big = torch.zeros((ns, cl.nd + 38), dtype=torch.float64, device="cuda")
    big[:, : cl.nd] = dev(Y)
    theta_p, Qt_p = op.rayleigh_ritz(big[:, : cl.nd])
    assert np.array_equal(theta_p, theta) and torch.equal(Qt_p, Qt)


@pytest.mark.parametrize("ns", [1, 7, 64, 70, 130])
def test_rayleigh_ritz_f32_block_sizes(ns):
    """FP32 blocks of one tile, a ragged tile, and 2-3 tiles (diagonal and
    off-diagonal tile pairs, a ragged last tile) through the FP64
    Rayleigh-Ritz: Ritz values and the projected pencil against the oracle
    fed the same FP32 values."""
    cl = inputs.make_cluster(16, 0.5, 2, 4, 1, seed=22, min_dist=0.0, margin=3.0)
    Y = inputs.round_to_f32(np.random.default_rng(100 + ns).standard_normal((ns, cl.nd)))
    rt, _, Hs, Ms = oracle.rayleigh_ritz(cl, Y)
    op = _b().Operator(cl)
    theta, Qt = op.rayleigh_ritz(dev(Y, torch.float32))
    assert np.abs(theta - rt).max() <= 1e-9 * max(1.0, np.abs(rt).max())
    Q = host(Qt).T
    assert np.abs(Q.T @ Ms @ Q - np.eye(ns)).max() < 1e-9
    assert np.abs(Hs @ Q - Ms @ Q * theta).max() < 1e-8 * max(1.0, np.abs(Hs).max())


@pytest.mark.parametrize("n", [(17, 15, 22), (17, 15, 21)], ids=["z-even", "z-odd"])
def test_rayleigh_ritz_f32_block_grids(n):
    """FP64 Rayleigh-Ritz of an FP32 block (FP64 H Y on the widened values,
    FP64 projection) on grids with an even and an odd z extent, with a padded
    leading dimension: Ritz values and the projected pencil against the
    oracle fed the same FP32 values (the library applies its FP64 operator to
    them)."""
    cl = inputs.make_cluster(n, 0.5, 2, 4, 1, seed=23, min_dist=0.0, margin=2.0)
    ns = 12
    Y = inputs.round_to_f32(np.random.default_rng(5).standard_normal((ns, cl.nd)))
    rt, _, Hs, Ms = oracle.rayleigh_ritz(cl, Y)
    op = _b().Operator(cl)
    pad = 2 if n[2] % 2 == 0 else 1
    big = torch.zeros((ns, cl.nd + pad), dtype=torch.float32, device="cuda")
    big[:, : cl.nd] = dev(Y, torch.float32)
    theta, Qt = op.rayleigh_ritz(big[:, : cl.nd])
    print(f"{n} f32 block RR max |dtheta| {np.abs(theta - rt).max():.2e}")
    assert np.abs(theta - rt).max() <= 1e-9 * max(1.0, np.abs(rt).max())
    Q = host(Qt).T
    assert np.abs(Q.T @ Ms @ Q - np.eye(ns)).max() < 1e-9


def test_lanczos_medium_grid():
    c = inputs.MEDIUM
    cl = inputs.case_cluster(c.name)
    op = _b().Operator(cl)
    v0 = inputs.lanczos_start(cl.nd, c.seed)
    _, _, theta = op.lanczos(40, dev(v0))
    _, _, rt = oracle.lanczos(cl, 40, v0)
    print("medium lanczos max |dtheta|", np.abs(theta - rt).max())
    assert np.abs(theta - rt).max() <= TOL_RITZ


@pytest.fixture(scope="module")
def wide():
    # the widest orbital block of the serving workload (253 columns) on a 36^3 grid
    cl = inputs.make_cluster(36, 0.45, 3, 8, 1, seed=31)
    ns, m, seed = 253, 16, 31
    X = inputs.orbitals(cl.nd, ns, seed)
    return cl, ns, m, seed, X, _bounds(cl, seed)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_wide_block_pass(wide, dtype):
    """Filter, FP64 Rayleigh-Ritz (library eigensolver path) and rotation of a
    253-column block against the oracle's pass."""
    cl, ns, m, seed, X, (a0, a, b) = wide
    binding = _b()
    op = binding.Operator(cl)
    if dtype == "f32":
        clr, Xr, tdt, tol = inputs.round_cluster_f32(cl), inputs.round_to_f32(X), torch.float32, TOL32
    else:
        clr, Xr, tdt, tol = cl, X, torch.float64, TOL64
    Yd = op.cheb_filter(dev(Xr, tdt), m, a0, a, b)
    ref = oracle.cheb_filter(clr, Xr, m, a0, a, b)
    err = rel_err(host(Yd), ref)
    print(f"wide {dtype} filter err {err:.3e}")
    assert err <= tol
    theta, Qt = op.rayleigh_ritz(Yd)
    rt, _, _, _ = oracle.rayleigh_ritz(clr, ref)
    print(f"wide {dtype} max |dtheta| {np.abs(theta - rt).max():.3e}")
    assert np.abs(theta - rt).max() <= TOL_RITZ
    R = host(binding.rotate(Yd, Qt))
    gram = R @ R.T
    assert np.abs(gram - np.eye(ns)).max() < (1e-9 if dtype == "f64" else 1e-3)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_single_column_matches_block(small, dtype):
    """A lone column is cut into many more x-chunks than a block of two (the
    launch keeps the chip busy): the chunking must not change a bit."""
    c, cl, X, (a0, a, b) = small
    op = _b().Operator(cl)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X2 = dev(X[:2], tdt)
    one = op.h_apply(X2[:1].contiguous())
    two = op.h_apply(X2)
    torch.cuda.synchronize()
    assert torch.equal(one[0], two[0])
    f1 = op.cheb_filter(X2[1:].contiguous(), 7, a0, a, b)
    f2 = op.cheb_filter(X2, 7, a0, a, b)
    torch.cuda.synchronize()
    assert torch.equal(f1[0], f2[1])


@pytest.mark.parametrize("n,k", [(10, 200), (12, 300)])
def test_lanczos_long_run_stays_orthogonal(n, k):
    """Long runs on small grids lose orthogonality in the three-term recurrence;
    the device's partial re-orthogonalisation must keep T_k equal to the fully
    re-orthogonalised oracle's (a loss would show up as spurious copies of
    converged Ritz values)."""
    cl = inputs.make_cluster(n, 0.5, 1, 4, 1, seed=n, margin=1.5, min_dist=0.0)
    v0 = inputs.lanczos_start(cl.nd, n)
    op = _b().Operator(cl)
    alpha, beta, theta = op.lanczos(k, dev(v0))
    ra, rb, rt = oracle.lanczos(cl, k, v0)
    print(f"n={n} k={k} max |dtheta| {np.abs(theta - rt).max():.2e} |dalpha| {np.abs(alpha - ra).max():.2e}")
    assert np.abs(theta - rt).max() <= TOL_RITZ
    assert np.abs(alpha - ra).max() <= 1e-8 and np.abs(beta - rb).max() <= 1e-8


@pytest.fixture(scope="module")
def large():
    c = inputs.LARGE
    return c, inputs.case_cluster(c.name)


def test_large_workload_pass(large):
    """The largest single-GPU workload (160^3 grid, h = 0.35, 128 atoms with 9
    projectors each, 600 orbitals, m = 30), the configuration the benchmark
    times: device Lanczos against the oracle's, FP64 and FP32 filters on
    sampled columns against the oracle, FP64 Rayleigh-Ritz of both blocks
    (the FP32 filter's Ritz values against the FP64 filter's), and the
    rotation: Ritz pairs through the oracle's H (Rayleigh quotients,
    orthonormality) and sampled rows of Y Q."""
    c, cl = large
    binding = _b()
    op = binding.Operator(cl)
    v0 = inputs.lanczos_start(cl.nd, c.seed)
    _, _, theta = op.lanczos(40, dev(v0))
    _, _, rt = oracle.lanczos(cl, 40, v0)
    print("large lanczos max |dtheta| %.2e" % np.abs(theta - rt).max())
    assert np.abs(theta - rt).max() <= TOL_RITZ
    a0, a, b = binding.select_bounds(theta, 8, ubound=op.upper_bound())
    oa0, oa, ob = oracle.select_bounds(rt, 8, ubound=oracle.upper_bound(cl))
    assert max(abs(a0 - oa0), abs(a - oa), abs(b - ob)) <= TOL_RITZ

    cols = [0, 299, 599]
    X32 = inputs.device_orbitals(cl.nd, c.ns, c.seed)
    Xs = X32[cols].double().cpu().numpy()
    # FP64 filter, sampled columns
    Y64 = op.cheb_filter(X32.double(), c.m, a0, a, b)
    e64 = rel_err(host(Y64[cols]), oracle.cheb_filter(cl, Xs, c.m, a0, a, b))
    # FP32 filter, sampled columns against the oracle on the FP32-rounded inputs
    Y32 = op.cheb_filter(X32, c.m, a0, a, b)
    e32 = rel_err(host(Y32[cols]), oracle.cheb_filter(inputs.round_cluster_f32(cl), Xs, c.m, a0, a, b))
    print("large filter errors f64 %.2e f32 %.2e" % (e64, e32))
    assert e64 <= TOL64 and e32 <= TOL32
    # column independence at full size: a column filtered alone is bit-identical
    one = op.cheb_filter(X32[cols[1]:cols[1] + 1].contiguous(), c.m, a0, a, b)
    torch.cuda.synchronize()
    assert torch.equal(one[0], Y32[cols[1]])
    del X32, one

    # FP64 Rayleigh-Ritz on both filtered blocks
    th32, _ = op.rayleigh_ritz(Y32, want_vectors=False)
    del Y32
    torch.cuda.empty_cache()
    th64, Qt = op.rayleigh_ritz(Y64)
    d = np.abs(th32 - th64).max()
    print("large Ritz values, FP32 filter vs FP64 filter: max |d| %.2e Ha" % d)
    assert d <= TOL_RITZ
    # rotation of the FP64 block; Ritz pairs checked with the oracle's H
    R = binding.rotate(Y64, Qt)
    pick = [0, 1, 300, 599]
    Rp = host(R[pick])
    HR = oracle.h_apply(cl, Rp)
    rq = np.einsum("ij,ij->i", Rp, HR) / np.einsum("ij,ij->i", Rp, Rp)
    print("large Rayleigh quotients vs Ritz values: max |d| %.2e" % np.abs(rq - th64[pick]).max())
    assert np.abs(rq - th64[pick]).max() <= TOL_RITZ
    gram = Rp @ Rp.T
    assert np.abs(gram - np.eye(len(pick))).max() < 1e-9
    # sampled grid rows of R = Y Q against the product on the host
    rows = np.random.default_rng(3).choice(cl.nd, 48, replace=False)
    idx = torch.from_numpy(rows).cuda()
    Yr = Y64[:, idx].cpu().numpy()              # (ns, rows)
    Q = Qt.cpu().numpy().T                       # column-major Q as returned
    ref = Q.T @ Yr                               # row c of R at the sampled rows
    got = R[:, idx].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print("large rotation sampled rows rel err %.2e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("ns,nd", [(1, 700), (7, 5000), (33, 3089), (64, 5000), (64, 131)])
def test_rotation_f32_blocks(ns, nd):
    # FP32 blocks (vector kernel, FP32 sums): against the oracle's FP64
    # product of the same FP32 values, with padded leading dimension and a
    # ragged tail of points
    binding = _b()
    rng = np.random.default_rng(1000 + ns)
    Y = inputs.round_to_f32(rng.standard_normal((ns, nd)))
    Q, _ = np.linalg.qr(rng.standard_normal((ns, ns)))
    Ypad = torch.zeros((ns, nd + 5), dtype=torch.float32, device="cuda")
    Ypad[:, :nd] = dev(Y, torch.float32)
    R = host(binding.rotate(Ypad[:, :nd], dev(Q.T)))
    ref = oracle.rotate(Y, Q)
    err = rel_err(R, ref)
    print("FP32 rotation ns", ns, "nd", nd, "max per-column relative error", err)
    assert err <= 2e-6


VEC = [
    # (grid, h, natoms, lmax, ns, radius, m): grids the vector step takes
    # (z extent a multiple of 4): partial z and y patches, x extents that
    # are not a multiple of the 8-plane projection segment, fewer x planes
    # than the stencil radius, radius below 6
    ((21, 19, 36), 0.45, 3, 2, 3, 6, 6),
    ((5, 40, 64), 0.5, 2, 1, 2, 6, 4),
    ((33, 24, 8), 0.6, 1, 1, 4, 4, 5),
    ((18, 18, 20), 0.5, 2, 2, 1, 6, 7),
    # z extent above the widest patch (160 nodes): a full and a ragged z patch
    ((6, 30, 172), 0.5, 2, 1, 2, 6, 4),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", VEC, ids=[f"{c[0]}-r{c[5]}-ns{c[4]}" for c in VEC])
def test_vector_step_edges(case, dtype):
    """The vector step kernels (16-byte units, fused projector scatter and
    gather) against the oracle: padded leading dimensions (multiples of the
    unit), every patch height of the dtype, H X and the filter."""
    n, h, natoms, lmax, ns, radius, m = case
    binding = _b()
    cl = inputs.make_cluster(n, h, natoms, 8, lmax, seed=sum(n) + 1, min_dist=0.0, margin=1.0, radius=radius)
    rng = np.random.default_rng(sum(n) + ns)
    X = rng.standard_normal((ns, cl.nd))
    if dtype == "f32":
        tdt, code, tol, heights = torch.float32, binding.SPARC_F32, TOL32, ((32, 16), (32, 32), (32, 64), (64, 16),
                                                                            (64, 32), (80, 32), (160, 24))
        X, ocl, pad = inputs.round_to_f32(X), inputs.round_cluster_f32(cl), 4
    else:
        tdt, code, tol, heights = torch.float64, binding.SPARC_F64, TOL64, ((32, 8), (32, 16), (32, 32), (64, 8),
                                                                            (64, 16), (64, 24))
        ocl, pad = cl, 2
    op = binding.Operator(cl)
    big = torch.zeros((ns, cl.nd + 4 * pad), dtype=tdt, device="cuda")
    big[:, : cl.nd] = dev(X, tdt)
    Xv = big[:, : cl.nd]
    a0, a, b = -3.0, 2.0, oracle.upper_bound(cl)
    href = oracle.h_apply(ocl, X)
    fref = oracle.cheb_filter(ocl, X, m, a0, a, b)
    for tzp, ty in heights:
        # patches of more than 512 threads take one column per workgroup
        wide = (tzp // pad) * ty > 512
        if wide:
            with pytest.raises(binding.SparcError):
                op.set_launch(code, tzp, ty, 0, 0, 2)
        for cb in ((1,) if wide else (1, 2)):
            op.set_launch(code, tzp, ty, 0, 0, cb)
            assert op.step_config(code, ns)[:2] == (tzp, ty) and op.step_config(code, ns)[4] == cb
            outbig = torch.full((ns, cl.nd + 2 * pad), 7.0, dtype=tdt, device="cuda")
            op.h_apply(Xv, outbig[:, : cl.nd])
            assert rel_err(host(outbig[:, : cl.nd]), href) <= tol, (ty, cb)
            assert torch.all(outbig[:, cl.nd:] == 7.0)  # padding untouched
            e = rel_err(host(op.cheb_filter(Xv, m, a0, a, b)), fref)
            print(f"{n} {dtype} patch {ty}x{tzp} col_block {cb} filter err {e:.2e}")
            assert e <= tol, (ty, cb)


def test_crowded_patches_fall_back():
    """More projector cubes on one patch than the vector kernels keep: the
    library takes a lower patch (or the scalar kernels), with the same
    results as the oracle."""
    binding = _b()
    cl = inputs.make_cluster((12, 40, 32), 0.5, 36, 4, 1, seed=9, min_dist=0.0, margin=1.0)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2, cl.nd))
    op = binding.Operator(cl)
    print("crowded: patch f32", op.step_config(binding.SPARC_F32, 2), "f64", op.step_config(binding.SPARC_F64, 2))
    a0, a, b = -3.0, 2.0, oracle.upper_bound(cl)
    assert rel_err(host(op.h_apply(dev(X))), oracle.h_apply(cl, X)) <= TOL64
    assert rel_err(host(op.cheb_filter(dev(X), 6, a0, a, b)), oracle.cheb_filter(cl, X, 6, a0, a, b)) <= TOL64
    X32 = inputs.round_to_f32(X)
    ocl = inputs.round_cluster_f32(cl)
    got = host(op.cheb_filter(dev(X32, torch.float32), 6, a0, a, b))
    assert rel_err(got, oracle.cheb_filter(ocl, X32, 6, a0, a, b)) <= TOL32
