"""Pins of the oracle's operator pieces against what the paper and mathematics fix.

* finite-difference weights vs an exact Fornberg solve and the tabulated values
* polynomial exactness and O(h^{2 n_o}) convergence (Sec. 3.1)
* closed-form discrete-sine eigenpairs (odd reflection) and Kronecker-sum
  eigenpairs of the exact 1D Toeplitz matrix (zero Dirichlet)
* symmetry of H, brute-force dense H, rank/eigenvalues of V_nl
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_weights():
    out = {}
    with open(os.path.join(GOLDEN, "fd2_central_order12.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            p, frac = line.split()
            out[int(p)] = Fraction(frac)
    return [out[p] for p in range(7)]


def test_weights_match_table_and_fornberg():
    g = _golden_weights()
    fb = oracle.fornberg_second_derivative(6)
    assert fb == g  # exact rational agreement of two independent routes
    for h in (1.0, 0.5, 0.35):
        w = oracle.fd_weights(6, h)
        # 1D centre coefficient is 2*w_0 (p = 0 term counted in +p and -p slots)
        assert math.isclose(2 * w[0] * h * h, float(g[0]), rel_tol=1e-14)
        for p in range(1, 7):
            assert math.isclose(w[p] * h * h, float(g[p]), rel_tol=1e-14)


@pytest.mark.parametrize("no", [1, 2, 3, 4, 5, 6])
def test_weights_sum_rule_and_low_orders(no):
    w = oracle.fd_weights(no, 1.0)
    fb = oracle.fornberg_second_derivative(no)
    assert math.isclose(2 * w[0], float(fb[0]), rel_tol=1e-14)
    for p in range(1, no + 1):
        assert math.isclose(w[p], float(fb[p]), rel_tol=1e-13)
    # constants are annihilated: 2 w_0 + 2 sum_p w_p = 0
    assert abs(2 * w[0] + 2 * w[1:].sum()) < 1e-13
    if no == 1:
        assert np.allclose(w, [-1.0, 1.0])


def _coords(n, h):
    return inputs.node_coords(n, h)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_polynomial_exactness_interior(axis):
    # lap_h x^q is exact for q <= 2 n_o + 1 = 13 at nodes >= n_o from the walls
    n = (20, 21, 22)
    h = 0.25
    xs = _coords(n[axis], h) - 0.5 * (n[axis] + 1) * h  # centred coordinate
    sl = [slice(6, n[d] - 6) for d in range(3)]
    for q in range(0, 16):
        shape = [1, 1, 1]
        shape[axis] = n[axis]
        f = np.broadcast_to((xs ** q).reshape(shape), n).copy()
        lap = oracle.laplacian(n, h, 6, f).reshape(n)
        exact = q * (q - 1) * xs ** (q - 2) if q >= 2 else np.zeros_like(xs)
        ex = np.broadcast_to(exact.reshape(shape), n)
        err = np.abs(lap - ex)[tuple(sl)].max()
        scale = max(1.0, np.abs(ex[tuple(sl)]).max(), np.abs(f[tuple(sl)]).max() / h ** 2)
        if q <= 13:
            assert err / scale < 1e-10, (q, err, scale)
        else:
            # q = 14, 15 are not reproduced exactly: the order is exactly 12
            assert err / scale > 1e-8, (q, err, scale)


def test_convergence_order_twelve():
    # Gaussian with analytic Laplacian; the error falls as h^12 (Sec. 3.1)
    s = 1.1
    L = 13.0
    errs, hs = [], []
    for nn in (25, 33, 41):
        h = L / (nn + 1)
        n = (nn, nn, nn)
        xs = _coords(nn, h) - L / 2
        X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
        r2 = X * X + Y * Y + Z * Z
        f = np.exp(-r2 / (2 * s * s))
        exact = f * (r2 / s ** 4 - 3 / s ** 2)
        lap = oracle.laplacian(n, h, 6, f).reshape(n)
        errs.append(np.abs(lap - exact).max())
        hs.append(h)
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 10.5 < slope < 13.5, (slope, errs)


def _sine_vec(n, k):
    vs = [np.sin(math.pi * k[d] * np.arange(1, n[d] + 1) / (n[d] + 1)) for d in range(3)]
    return np.einsum("i,j,k->ijk", *vs).reshape(-1)


@pytest.mark.parametrize("k", [(1, 1, 1), (3, 2, 5), (7, 1, 2), (11, 9, 4)])
def test_sine_eigenpairs_odd_reflection(k):
    # closed-form eigenpairs of the stencil under odd-reflection ghosts
    n = (12, 10, 11)
    h = 0.45
    c = [float(v) for v in oracle.fornberg_second_derivative(6)]
    lam = 0.0
    for d in range(3):
        t = math.pi * k[d] / (n[d] + 1)
        lam += -0.5 * (c[0] + 2 * sum(c[p] * math.cos(p * t) for p in range(1, 7))) / h ** 2
    cl = inputs.free_cluster(n, h, v0=0.0)
    v = _sine_vec(n, k)
    Hv = oracle.h_apply(cl, v, bc=1)[0]
    assert np.abs(Hv - lam * v).max() < 1e-11 * max(1.0, abs(lam))
    # under zero padding the same vector is NOT an eigenvector (radius > 1)
    Hv0 = oracle.h_apply(cl, v, bc=0)[0]
    assert np.linalg.norm(Hv0 - lam * v) > 1e-4 * np.linalg.norm(lam * v)


def _toeplitz_eigs(n, h):
    return [np.linalg.eigh(oracle.toeplitz_1d(6, h, n[d])) for d in range(3)]


@pytest.mark.parametrize("idx", [(0, 0, 0), (2, 5, 1), (9, 3, 7), (13, 12, 8)])
def test_kronecker_eigenpairs_zero_dirichlet(idx):
    n = (14, 13, 9)
    h = 0.5
    eig = _toeplitz_eigs(n, h)
    lam = sum(eig[d][0][idx[d]] for d in range(3))
    v = np.einsum("i,j,k->ijk", *[eig[d][1][:, idx[d]] for d in range(3)]).reshape(-1)
    v0 = -0.7
    cl = inputs.free_cluster(n, h, v0=v0)
    Hv = oracle.h_apply(cl, v, bc=0)[0]
    assert np.abs(Hv - (lam + v0) * v).max() < 1e-12 * max(1.0, abs(lam))


def test_radius_one_modes_coincide():
    # with n_o = 1 the zero and odd-reflection modes give the same operator
    n = (7, 6, 5)
    cl = inputs.free_cluster(n, 0.6, radius=1)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(cl.nd)
    assert np.allclose(oracle.h_apply(cl, x, bc=0), oracle.h_apply(cl, x, bc=1), atol=1e-13)


def _tiny_cluster(seed=7, natoms=2, lmax=1, n=(8, 9, 10), h=1.0):
    return inputs.make_cluster(n, h, natoms, 4, lmax, seed, min_dist=0.0, margin=4.0)


def test_symmetry_of_h():
    cl = inputs.make_cluster(18, 0.5, 3, 8, 2, seed=11, min_dist=1.0)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(cl.nd)
    v = rng.standard_normal(cl.nd)
    Hu = oracle.h_apply(cl, u)[0]
    Hv = oracle.h_apply(cl, v)[0]
    lhs, rhs = u @ Hv, Hu @ v
    assert abs(lhs - rhs) < 1e-13 * (np.linalg.norm(u) * np.linalg.norm(Hv))


@pytest.mark.parametrize("lmax,bc", [(1, 0), (2, 0), (1, 1)])
def test_h_apply_matches_dense_brute_force(lmax, bc):
    cl = _tiny_cluster(lmax=lmax)
    H = oracle.dense_hamiltonian(cl, bc=bc)
    assert np.allclose(H, H.T, atol=1e-14 * np.abs(H).max())
    rng = np.random.default_rng(3)
    X = rng.standard_normal((3, cl.nd))
    got = oracle.h_apply(cl, X, bc=bc)
    ref = (H @ X.T).T
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()


def test_nonlocal_spectrum_one_atom():
    # V_nl of one atom has rank nproj with eigenvalues eig(h^3 Gamma chi^T chi)
    cl = _tiny_cluster(natoms=1, lmax=2, n=(10, 10, 10), h=0.8)
    a = cl.atoms[0]
    free = inputs.free_cluster(cl.n, cl.h, v0=0.0)
    H = oracle.dense_hamiltonian(cl) - oracle.dense_hamiltonian(free) - np.diag(cl.veff)
    ev = np.linalg.eigvalsh(H)
    chi = a.chi.reshape(a.nproj, -1)
    G = chi @ chi.T
    Gam = np.diag(a.gamma)
    ref = np.sort(np.linalg.eigvals(cl.h ** 3 * Gam @ G).real)
    big = np.sort(ev[np.abs(ev) > 1e-10 * np.abs(ev).max()])
    assert len(big) == a.nproj
    assert np.allclose(big, ref, rtol=1e-9, atol=1e-13)
    # and the oracle's matrix-free V_nl reproduces the same operator
    rng = np.random.default_rng(5)
    x = rng.standard_normal(cl.nd)
    got = oracle.h_apply(cl, x)[0] - oracle.h_apply(free, x)[0] - cl.veff * x
    assert np.allclose(got, H @ x, atol=1e-13 * np.abs(H @ x).max())


def test_upper_bound_dominates_spectrum():
    cl = _tiny_cluster(lmax=1)
    lam = np.linalg.eigvalsh(oracle.dense_hamiltonian(cl))
    ub = oracle.upper_bound(cl)
    assert ub >= lam[-1]
    # and is not absurdly loose: within 15% of lambda_max for this grid
    assert ub < 1.15 * lam[-1] + 1.0
