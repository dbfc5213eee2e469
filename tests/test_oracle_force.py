"""Pins of the oracle's finite-difference gradient (Sec. 3.1 Eq.
gradient:approximate) and nonlocal force (Sec. 3.6 Eqs. NonlocForce:Discrete,
NonLocForce:U:W, Alg. 4)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd1_central_order12.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, frac = line.split()
            out[int(p)] = Fraction(frac)
    return [out[p] for p in range(1, 7)]


def test_gradient_weights_table_fornberg_and_low_orders():
    g = _golden()
    fb = oracle.fornberg_first_derivative(6)
    assert fb[0] == 0 and fb[1:] == g  # two independent exact routes agree
    for h in (1.0, 0.5, 0.35):
        w = oracle.gradient_weights(6, h)
        for p in range(1, 7):
            assert math.isclose(w[p] * h, float(g[p - 1]), rel_tol=1e-14)
    # textbook central differences: n_o = 1 and 2
    assert np.allclose(oracle.gradient_weights(1, 1.0)[1:], [0.5], rtol=1e-15)
    assert np.allclose(oracle.gradient_weights(2, 1.0)[1:], [2.0 / 3.0, -1.0 / 12.0], rtol=1e-15)
    for no in range(1, 7):
        fb = oracle.fornberg_first_derivative(no)
        assert np.allclose(oracle.gradient_weights(no, 1.0)[1:], [float(c) for c in fb[1:]], rtol=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_gradient_polynomial_exactness(axis):
    """Order 2 n_o = 12: exact on x^k for k <= 12 at nodes 6 or more from the
    walls, not for k = 13; the other two components vanish."""
    n, h = (20, 21, 22), 0.3
    x = inputs.node_coords(n[axis], h) - 3.1  # shift: no symmetry helps
    shape = [1, 1, 1]
    shape[axis] = n[axis]
    interior = [slice(6, n[d] - 6) for d in range(3)]
    for k, exact in ((1, True), (7, True), (12, True), (13, False)):
        f = np.broadcast_to((x ** k).reshape(shape), n).reshape(-1)
        g = oracle.gradient(n, h, 6, f).reshape((3,) + n)
        ref = np.broadcast_to((k * x ** (k - 1)).reshape(shape), n)
        err = np.abs(g[axis][tuple(interior)] - ref[tuple(interior)]).max() / np.abs(ref).max()
        assert (err < 1e-9) == exact, (k, err)
        for d in range(3):
            if d != axis:  # constant along d: zero away from the walls
                assert np.abs(g[d][tuple(interior)]).max() == 0.0


def test_gradient_summation_by_parts():
    """With zero padding the gradient matrix is antisymmetric:
    sum (nabla_d f) u = -sum f (nabla_d u) for any two grid functions."""
    rng = np.random.default_rng(3)
    n, h = (9, 10, 11), 0.4
    f, u = rng.standard_normal((2, n[0] * n[1] * n[2]))
    gf, gu = oracle.gradient(n, h, 6, f), oracle.gradient(n, h, 6, u)
    for d in range(3):
        a, b = np.dot(gf[d], u), -np.dot(f, gu[d])
        assert abs(a - b) < 1e-11 * np.abs(gf[d] * u).sum()


SIG = 0.5   # Gaussian width of the test projectors (bohr)
RC = 3.4    # cube half-width: exp(-RC^2 / (2 SIG^2)) ~ 1e-10 at its faces


def _projectors(pos, n, h, lo, ext):
    """s and p-like projectors exp(-r^2/2s^2) * {1, x, y, z} on the cube of
    nodes lo .. lo+ext-1, centred at pos (analytic, smooth to rounding)."""
    xs = [inputs.node_coords(n[d], h)[lo[d]:lo[d] + ext[d]] - pos[d] for d in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    e = np.exp(-(X * X + Y * Y + Z * Z) / (2 * SIG * SIG))
    return np.stack([e, X * e / SIG, Y * e / SIG, Z * e / SIG])


def _cluster(positions, gammas, n, h, shift=None):
    atoms = []
    for J, (pos, gam) in enumerate(zip(positions, gammas)):
        lo = tuple(int(math.ceil((pos[d] - RC) / h)) - 1 for d in range(3))  # node i sits at (i+1) h
        hi = tuple(int(math.floor((pos[d] + RC) / h)) - 1 for d in range(3))
        ext = tuple(hi[d] - lo[d] + 1 for d in range(3))
        assert all(lo[d] >= 0 and hi[d] < n[d] for d in range(3))
        p = np.array(pos, dtype=np.float64)
        if shift is not None and shift[0] == J:
            p[shift[1]] += shift[2]
        atoms.append(inputs.Atom(pos=p, Z=1, sigma=1.0, lo=lo, ext=ext, chi=_projectors(p, n, h, lo, ext),
                                 gamma=np.asarray(gam, dtype=np.float64)))
    return inputs.Cluster(n=n, h=h, radius=6, veff=np.zeros(n[0] * n[1] * n[2]), atoms=atoms, seed=0)


def _energy(cl, Psi, g):
    """E_nl = 2 sum_n g_n sum_lm gamma_Jl Y_Jnlm^2 (the nonlocal band energy,
    two electrons per orbital), Y = h^3 sum psi chi."""
    E = 0.0
    for a in cl.atoms:
        sl = tuple(slice(a.lo[d], a.lo[d] + a.ext[d]) for d in range(3))
        for k in range(Psi.shape[0]):
            psi = Psi[k].reshape(cl.n)[sl]
            Y = cl.h ** 3 * np.array([np.sum(psi * c) for c in a.chi])
            E += 2.0 * g[k] * np.sum(a.gamma * Y * Y)
    return E


def test_force_is_minus_the_energy_derivative():
    """f_J = -dE_nl/dR_J: the analytic projectors are moved by +-delta along each
    axis and the energy differenced centrally.  The two agree up to the
    12th-order error of the finite-difference gradient on the projectors
    (h / sigma = 0.4), below 1e-7 of the force (3e-9 measured); a dropped factor, a
    wrong sign, a swapped axis or the wrong atom fails by O(1)."""
    n, h = (40, 39, 41), 0.2
    positions = [(3.95, 3.9, 4.01), (4.3, 4.1, 3.8)]   # overlapping cubes
    gammas = [(1.3, -0.7, 0.4, 0.9), (-0.5, 1.1, 0.8, -1.2)]
    rng = np.random.default_rng(11)
    ns = 3
    # smooth orbitals: low-order polynomials times a broad envelope
    xs = [inputs.node_coords(n[d], h) - 4.0 for d in range(3)]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    env = np.exp(-(X * X + Y * Y + Z * Z) / 8.0)
    Psi = np.stack([(env * (c[0] + c[1] * X + c[2] * Y + c[3] * Z + c[4] * X * Y)).reshape(-1)
                    for c in rng.standard_normal((ns, 5))])
    g = np.array([1.0, 0.7, 0.2])
    f = oracle.nonlocal_force(_cluster(positions, gammas, n, h), Psi, g)
    delta = 1e-4
    fd = np.zeros_like(f)
    for J in range(2):
        for d in range(3):
            ep = _energy(_cluster(positions, gammas, n, h, (J, d, delta)), Psi, g)
            em = _energy(_cluster(positions, gammas, n, h, (J, d, -delta)), Psi, g)
            fd[J, d] = -(ep - em) / (2 * delta)
    err = np.abs(f - fd).max() / np.abs(fd).max()
    assert np.abs(fd).max() > 1e-3
    assert err < 1e-7, (f, fd, err)


def test_force_of_random_orbitals_via_summation_by_parts():
    """For any orbitals W = h^3 sum (nabla psi) chi = -h^3 sum psi (nabla chi),
    with nabla chi the gradient of chi placed on the grid: a second route to
    the force through the projectors' gradients."""
    rng = np.random.default_rng(2)
    cl = inputs.make_cluster((20, 21, 22), 0.5, 3, 6, 1, seed=9, min_dist=1.0, margin=3.0)
    Psi = rng.standard_normal((4, cl.nd))
    g = np.array([1.0, 1.0, 0.5, 0.1])
    f = oracle.nonlocal_force(cl, Psi, g)
    h3 = cl.h ** 3
    ref = np.zeros_like(f)
    for J, a in enumerate(cl.atoms):
        sl = tuple(slice(a.lo[d], a.lo[d] + a.ext[d]) for d in range(3))
        for p in range(a.nproj):
            chi = np.zeros(cl.n)
            chi[sl] = a.chi[p]
            gchi = oracle.gradient(cl.n, cl.h, cl.radius, chi.reshape(-1))
            for k in range(Psi.shape[0]):
                Yk = h3 * np.dot(Psi[k], chi.reshape(-1))
                for d in range(3):
                    ref[J, d] += -4.0 * g[k] * a.gamma[p] * Yk * (-h3 * np.dot(Psi[k], gchi[d]))
    assert np.abs(f - ref).max() < 1e-10 * np.abs(ref).max()
