"""Pins of the oracle's electrostatic potential solve (Sec. 3.3, Eqs.
FD:PoissonDiscrete, Phi:correction, phi:BC:discrete; CG with block Jacobi and
l_max = 6 from Sec. 4)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre
from scipy.special import erf

import oracle
from oracle import poisson


def test_real_harmonics_orthonormal_and_addition_theorem():
    """<Y_lm, Y_l'm'> = delta on the sphere (Gauss-Legendre in cos(theta) times
    a uniform azimuth grid, exact for these degrees), and the addition
    theorem sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b) with numpy's
    Legendre polynomials."""
    lmax = 6
    t, wt = legendre.leggauss(12)
    phi = np.arange(16) * 2 * np.pi / 16
    T, P = np.meshgrid(t, phi, indexing="ij")
    s = np.sqrt(1 - T * T)
    Y = poisson.real_harmonics(lmax, s * np.cos(P), s * np.sin(P), T).reshape((lmax + 1) ** 2, -1)
    W = (wt[:, None] * np.full(16, 2 * np.pi / 16)[None, :]).reshape(-1)
    G = (Y * W) @ Y.T
    assert np.abs(G - np.eye((lmax + 1) ** 2)).max() < 1e-13
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, 3))
    a /= np.linalg.norm(a)
    b /= np.linalg.norm(b)
    Ya = poisson.real_harmonics(lmax, *a)
    Yb = poisson.real_harmonics(lmax, *b)
    for l in range(lmax + 1):
        lhs = sum(Ya[l * l + l + m] * Yb[l * l + l + m] for m in range(-l, l + 1))
        coef = np.zeros(l + 1)
        coef[l] = 1
        assert abs(lhs - (2 * l + 1) / (4 * np.pi) * legendre.legval(np.dot(a, b), coef)) < 1e-13


def _gauss(n, h, centre, sigma, q):
    X, Y, Z = (v.reshape(-1) for v in np.meshgrid(*poisson.node_positions(n, h), indexing="ij"))
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    return q * np.exp(-r2 / (2 * sigma ** 2)) / (2 * np.pi * sigma ** 2) ** 1.5, (X, Y, Z)


def test_multipoles_of_a_displaced_charge():
    """A normalised Gaussian charge q at c: the discrete moments equal those of
    a point charge, q |c|^l Y_lm(c) (|x|^l Y_lm is harmonic, so its mean over
    a radially symmetric charge is its value at the centre; the grid sum of
    a Gaussian 2.4 h wide, cut by the box 9 widths out, is exact to
    rounding), and the expansion reproduces q/|x - c| far away up to the
    truncation at l_max = 6, (|c|/|x|)^7."""
    n, h = (48, 46, 50), 0.25
    c, q = np.array([0.6, -0.4, 0.5]), 1.7
    f, _ = _gauss(n, h, c, 0.6, q)
    Q = poisson.multipole_moments(n, h, f, 6)
    rc = np.linalg.norm(c)
    Yc = poisson.real_harmonics(6, *c)
    for l in range(7):
        for m in range(-l, l + 1):
            i = l * l + l + m
            assert abs(Q[i] - q * rc ** l * Yc[i]) < 1e-12 * q
    pts = np.array([[30.0, 1.0, -2.0], [-4.0, 25.0, 3.0], [2.0, 2.0, -28.0]])
    phi = poisson.boundary_potential(Q, 6, pts[:, 0], pts[:, 1], pts[:, 2])
    exact = q / np.linalg.norm(pts - c, axis=1)
    assert np.abs(phi / exact - 1).max() < 3 * (rc / 25.0) ** 7
    # truncating at l = 0 keeps only the monopole: visibly worse
    phi0 = poisson.boundary_potential(Q[:1], 0, pts[:, 0], pts[:, 1], pts[:, 2])
    assert np.abs(phi0 / exact - 1).max() > 1e-3


def test_charge_correction_reproduces_the_full_stencil():
    """For any phi defined everywhere, -(1/4 pi) lap_h phi evaluated with phi's
    true values off the grid equals the zero-Dirichlet operator on the grid
    values plus the charge correction d (Eq. Phi:correction), with d from
    phi's off-grid values; that is, Eq. FD:PoissonDiscrete with charge - d on
    the right is the full-space equation.  The full stencil is applied
    independently on a padded array."""
    n, h, no = (11, 12, 13), 0.4, 6
    fun = lambda X, Y, Z: np.sin(0.7 * X + 0.2) * np.cos(0.5 * Y) + 0.3 * Z * Z + 1.0 / (3 + X * X)  # noqa: E731
    xs = poisson.node_positions(n, h)
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    phi = fun(X, Y, Z).reshape(-1)
    # full stencil on a padded array of true values
    ext = [(np.arange(-no, n[d] + no) + 1 - 0.5 * (n[d] + 1)) * h for d in range(3)]
    Xe, Ye, Ze = np.meshgrid(*ext, indexing="ij")
    F = fun(Xe, Ye, Ze)
    w = oracle.fd_weights(no, h)
    core = tuple(slice(no, no + n[d]) for d in range(3))
    lap = 6 * w[0] * F[core]
    for ax in range(3):
        for p in range(1, no + 1):
            for s in (-1, 1):
                sl = list(core)
                sl[ax] = slice(no + s * p, no + s * p + n[ax])
                lap = lap + w[p] * F[tuple(sl)]
    full = (-lap / (4 * np.pi)).reshape(-1)
    d = poisson.charge_correction(n, h, no, fun)
    got = poisson.poisson_apply(n, h, no, phi) + d
    assert np.abs(got - full).max() < 1e-12 * np.abs(full).max()
    assert np.abs(d).max() > 1e-2  # the correction matters here


def test_solve_recovers_a_manufactured_potential():
    """With the right-hand side and the correction of a known phi, CG with
    block Jacobi returns phi on the grid (the discrete problem is exact for
    it), to the solver tolerance."""
    n, h, no = (14, 13, 15), 0.35, 6
    fun = lambda X, Y, Z: np.exp(-0.1 * (X * X + 2 * Y * Y + Z * Z)) + 0.2 * X - 0.1 * Y * Z  # noqa: E731
    X, Y, Z = np.meshgrid(*poisson.node_positions(n, h), indexing="ij")
    phi = fun(X, Y, Z).reshape(-1)
    charge = poisson.poisson_apply(n, h, no, phi) + poisson.charge_correction(n, h, no, fun)
    # charge - d(fun) = apply(phi): the solve must return phi
    sol, it, res, _ = poisson.poisson_solve(n, h, no, charge, tol=1e-12, phi_off=fun)
    assert res <= 1e-12 and it > 5
    assert np.abs(sol - phi).max() < 1e-9 * np.abs(phi).max()


def test_block_jacobi_is_exact_on_one_block_and_helps():
    """One block covering the grid makes the preconditioner the exact inverse
    (CG converges in one step); B = 4 needs fewer iterations than B = 1
    (point Jacobi, a constant scaling here)."""
    n, h, no = (6, 7, 8), 0.5, 6
    rng = np.random.default_rng(4)
    charge = rng.standard_normal(n[0] * n[1] * n[2])
    zero = lambda X, Y, Z: 0.0 * X  # noqa: E731
    _, it1, res1, _ = poisson.poisson_solve(n, h, no, charge, tol=1e-12, block=8, phi_off=zero)
    assert it1 == 1 and res1 < 1e-12
    n = (24, 22, 26)
    charge = rng.standard_normal(n[0] * n[1] * n[2])
    _, it4, _, _ = poisson.poisson_solve(n, h, no, charge, tol=1e-10, block=4, phi_off=zero)
    _, itp, _, _ = poisson.poisson_solve(n, h, no, charge, tol=1e-10, block=1, phi_off=zero)
    assert it4 < itp


@pytest.mark.parametrize("centre", [(0.0, 0.0, 0.0), (0.7, -0.5, 0.4)])
def test_gaussian_charge_potential(centre):
    """A Gaussian charge in a box whose walls cut deep into its potential:
    with the multipole boundary correction (l_max = 6) phi matches the exact
    q erf(r / (sqrt 2 sigma)) / r on the grid to 1e-6 of its peak; zero
    Dirichlet walls (no correction) miss by more than 10%."""
    n, h, sigma, q = (32, 32, 32), 0.3, 0.8, 2.0
    c = np.array(centre)
    f, (X, Y, Z) = _gauss(n, h, c, sigma, q)
    r = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    exact = np.where(r > 1e-12, q * erf(r / (math.sqrt(2) * sigma)) / np.where(r > 1e-12, r, 1.0),
                     q * math.sqrt(2 / math.pi) / sigma)
    phi, it, res, _ = poisson.poisson_solve(n, h, 6, f, lmax=6, tol=1e-12)
    assert res <= 1e-12
    assert np.abs(phi - exact).max() < 1e-6 * exact.max()
    zero = lambda X, Y, Z: 0.0 * X  # noqa: E731
    phi_d, _, _, _ = poisson.poisson_solve(n, h, 6, f, tol=1e-10, phi_off=zero)
    assert np.abs(phi_d - exact).max() > 0.1 * exact.max()
