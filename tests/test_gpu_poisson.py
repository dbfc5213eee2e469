"""GPU parity of the electrostatic potential solve (Sec. 3.3; CG with block
Jacobi and l_max = 6 from Sec. 4) through sparc_poisson_solve against the
oracle.

Both sides solve the same discrete problem to ||r|| <= tol ||c - d|| with
the same preconditioner, in FP64, and differ in rounding order only: the
multipole moments agree to 1e-12 relative, the CG iterates follow the same
recurrence (iteration counts within one), and the solutions agree to
1e-8 of their peak (the residual tolerance 1e-12 times the condition
number of the operator, (n/pi)^2 ~ 1e2 on these grids, with margin).  At the
full 160^3 grid the oracle's preconditioned CG is too slow; there the
library's solution is checked through the oracle's operator, moments and
correction: its true residual c - d - A phi."""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
from oracle import poisson
from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


def _b():
    from paper_1603_04334_amd import binding
    binding.lib()
    return binding


def _charge(n, h, centres, sigmas, qs):
    X, Y, Z = (v.reshape(-1) for v in np.meshgrid(*poisson.node_positions(n, h), indexing="ij"))
    f = np.zeros(X.size)
    for c, s, q in zip(centres, sigmas, qs):
        r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        f += q * np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    return f, (X, Y, Z)


def _solve(n, h, f, **kw):
    b = _b()
    P = b.Poisson(n, h, **{k: v for k, v in kw.items() if k in ("lmax", "block", "radius")})
    c = torch.from_numpy(f).cuda()
    phi, it, res, Q = P.solve(c, tol=kw.get("tol", TOL))
    torch.cuda.synchronize()
    return P, c, phi.cpu().numpy(), it, res, Q


def test_gaussian_charge_against_oracle_and_closed_form():
    n, h, sigma, q = (32, 32, 32), 0.3, 0.8, 2.0
    c = np.array([0.7, -0.5, 0.4])
    f, (X, Y, Z) = _charge(n, h, [c], [sigma], [q])
    _, _, phi, it, res, Q = _solve(n, h, f)
    ref, it_ref, res_ref, _ = poisson.poisson_solve(n, h, 6, f, lmax=6, tol=TOL)
    Qref = poisson.multipole_moments(n, h, f, 6)
    eq = np.abs(Q - Qref).max() / np.abs(Qref).max()
    ep = np.abs(phi - ref).max() / np.abs(ref).max()
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    exact = q * erf(r / (math.sqrt(2) * sigma)) / r
    ex = np.abs(phi - exact).max() / exact.max()
    print(f"poisson 32^3: iters {it} (oracle {it_ref}), rel resid {res:.2e}, moments err {eq:.2e}, "
          f"phi err {ep:.2e}, vs closed form {ex:.2e}", flush=True)
    assert res <= TOL and abs(it - it_ref) <= 1
    assert eq <= 1e-12 and ep <= 1e-8 and ex <= 1e-6


@pytest.mark.parametrize("block", [(4, 4, 4), (2, 4, 8), (3, 5, 7)])
def test_ragged_grid_dipole_blocks(block):
    """A dipole (two opposite Gaussians) on a grid whose edges are not
    multiples of the block edges (cut-short blocks on every axis)."""
    n, h = (30, 27, 33), 0.32
    f, _ = _charge(n, h, [(0.8, 0.2, -0.3), (-0.9, -0.1, 0.5)], [0.7, 0.9], [1.0, -1.0])
    _, _, phi, it, res, Q = _solve(n, h, f, block=block)
    ref, it_ref, _, _ = poisson.poisson_solve(n, h, 6, f, lmax=6, tol=TOL, block=block)
    ep = np.abs(phi - ref).max() / np.abs(ref).max()
    print(f"poisson {n} block {block}: iters {it} (oracle {it_ref}) phi err {ep:.2e}", flush=True)
    assert res <= TOL and abs(it - it_ref) <= 1 and ep <= 1e-8


def test_lmax_and_stencil_radius():
    """l_max = 2 and a radius-4 stencil: the same problem definition on both sides."""
    n, h = (24, 26, 22), 0.4
    f, _ = _charge(n, h, [(0.5, 0.6, -0.2)], [0.9], [1.5])
    _, _, phi, it, res, Q = _solve(n, h, f, lmax=2, radius=4)
    ref, it_ref, _, _ = poisson.poisson_solve(n, h, 4, f, lmax=2, tol=TOL)
    assert Q.size == 9
    assert np.abs(Q - poisson.multipole_moments(n, h, f, 2)).max() <= 1e-12 * np.abs(Q).max()
    assert abs(it - it_ref) <= 1 and np.abs(phi - ref).max() <= 1e-8 * np.abs(ref).max()


def test_warm_start_and_reproducibility():
    b = _b()
    n, h = (28, 28, 28), 0.35
    f, _ = _charge(n, h, [(0.3, 0.0, 0.1)], [0.8], [1.0])
    P = b.Poisson(n, h)
    c = torch.from_numpy(f).cuda()
    phi1, it1, _, _ = P.solve(c, tol=TOL)
    phi2, it2, _, _ = P.solve(c, tol=TOL)
    torch.cuda.synchronize()
    assert it1 == it2 and torch.equal(phi1, phi2)
    # from the converged solution: no iteration needed
    phi3, it3, res3, _ = P.solve(c, phi=phi1.clone(), use_guess=True, tol=1e-9)
    assert it3 == 0 and res3 <= 1e-9
    # from a perturbed one: fewer iterations than from zero, same answer
    guess = phi1 + 1e-3 * torch.sin(torch.arange(phi1.numel(), device="cuda", dtype=torch.float64))
    phi4, it4, _, _ = P.solve(c, phi=guess, use_guess=True, tol=TOL)
    torch.cuda.synchronize()
    assert it4 < it1
    assert (phi4 - phi1).abs().max().item() <= 1e-8 * phi1.abs().max().item()
    # max_iter stops early and reports the residual reached
    _, it5, res5, _ = P.solve(c, tol=TOL, max_iter=5)
    assert it5 == 5 and res5 > TOL


def test_errors():
    b = _b()
    with pytest.raises(b.SparcError) as ei:
        b.Poisson((8, 8, 8), 0.5, lmax=7)
    assert ei.value.status == b.SPARC_E_ARG
    with pytest.raises(b.SparcError) as ei:
        b.Poisson((8, 8, 8), 0.5, block=(8, 8, 8))
    assert ei.value.status == b.SPARC_E_ARG
    P = b.Poisson((8, 8, 8), 0.5)
    c = torch.zeros(512, dtype=torch.float64, device="cuda")
    with pytest.raises(b.SparcError) as ei:
        P.solve(c, tol=0.0)
    assert ei.value.status == b.SPARC_E_ARG
    with pytest.raises(b.SparcError) as ei:
        P.solve(c, ws=torch.empty(64, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == b.SPARC_E_WORKSPACE
    with pytest.raises(b.SparcError) as ei:
        P.solve(c, phi=c)
    assert ei.value.status == b.SPARC_E_ALIAS
    # zero charge: zero potential, no iteration
    phi, it, res, _ = P.solve(c)
    torch.cuda.synchronize()
    assert it == 0 and torch.count_nonzero(phi).item() == 0


def test_full_grid_residual_through_the_oracle():
    """The 160^3, h = 0.35 grid of the benchmark cluster with a neutral
    synthetic total charge (each atom: a compact negative pseudocharge -Z and
    a broader positive electron cloud +Z): the library's phi satisfies the
    oracle's discrete equation, ||c - d - A phi|| <= 10 tol ||c - d|| with d
    from the oracle's moments (so the moments, the correction and the solve
    are all checked), and its moments match the oracle's."""
    c = inputs.LARGE
    cl = inputs.case_cluster(c.name)
    n, h = cl.n, cl.h
    cen = 0.5 * (np.array(n) + 1) * h
    pos = [a.pos - cen for a in cl.atoms]
    Z = [a.Z for a in cl.atoms]
    f, _ = _charge(n, h, pos + pos, [0.6] * len(pos) + [1.1] * len(pos), [-z for z in Z] + Z)
    tol = 1e-10
    P, cd, phi_d, it, res, Q = _solve(n, h, f, tol=tol)
    Qref = poisson.multipole_moments(n, h, f, 6)
    eq = np.abs(Q - Qref).max() / np.abs(Qref).max()
    d = poisson.charge_correction(n, h, 6, lambda X, Y, Z_: poisson.boundary_potential(Qref, 6, X, Y, Z_))
    rhs = f - d
    r = rhs - poisson.poisson_apply(n, h, 6, phi_d)
    rel = np.linalg.norm(r) / np.linalg.norm(rhs)
    print(f"poisson 160^3: iters {it}, recursive resid {res:.2e}, true resid {rel:.2e}, moments err {eq:.2e}",
          flush=True)
    assert res <= tol and rel <= 10 * tol and eq <= 1e-10
