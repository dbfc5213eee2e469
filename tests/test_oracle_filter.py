"""Pins of the oracle's Chebyshev filter, Lanczos bounds and Rayleigh-Ritz.

* scalar identity p(H) v = p(lambda) v on closed-form eigenvectors, with
  C_m taken from cos(m acos x) / cosh(m acosh x)
* brute force Q p(Lambda) Q^T X on tiny grids
* commutation with H, column independence, m = 1, unit gain at a0, the
  scaled/unscaled relation, and the printed form of the algorithm being wrong
* Lanczos interlacing / bounds, Rayleigh-Ritz on invariant subspaces
"""
import math

import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs


def _eig_zero_bc(n, h, idx):
    eig = [np.linalg.eigh(oracle.toeplitz_1d(6, h, n[d])) for d in range(3)]
    lam = sum(eig[d][0][idx[d]] for d in range(3))
    v = np.einsum("i,j,k->ijk", *[eig[d][1][:, idx[d]] for d in range(3)]).reshape(-1)
    return lam, v


def _sine(n, h, k):
    c = [float(v) for v in oracle.fornberg_second_derivative(6)]
    lam = 0.0
    for d in range(3):
        t = math.pi * k[d] / (n[d] + 1)
        lam += -0.5 * (c[0] + 2 * sum(c[p] * math.cos(p * t) for p in range(1, 7))) / h ** 2
    vs = [np.sin(math.pi * k[d] * np.arange(1, n[d] + 1) / (n[d] + 1)) for d in range(3)]
    return lam, np.einsum("i,j,k->ijk", *vs).reshape(-1)


@pytest.mark.parametrize("m", [1, 2, 7, 20, 31])
@pytest.mark.parametrize("idx", [(0, 0, 0), (4, 1, 2), (11, 10, 7)])
def test_scalar_identity_zero_bc(m, idx):
    n, h, v0 = (12, 11, 9), 0.5, 0.3
    lam, v = _eig_zero_bc(n, h, idx)
    lam += v0
    cl = inputs.free_cluster(n, h, v0=v0)
    a0, a, b = v0 - 0.2, v0 + 3.0, v0 + 45.0
    y = oracle.cheb_filter(cl, v, m, a0, a, b)[0]
    g = oracle.filter_gain(lam, m, a0, a, b)
    assert np.abs(y - g * v).max() <= 1e-12 * max(1.0, abs(g)) * np.abs(v).max()


@pytest.mark.parametrize("k", [(1, 1, 1), (2, 3, 1), (9, 8, 10)])
def test_scalar_identity_sine_odd_bc(k):
    n, h = (10, 9, 11), 0.45
    lam, v = _sine(n, h, k)
    cl = inputs.free_cluster(n, h, v0=0.0)
    for (m, a0, a, b) in [(20, 0.0, 4.0, 60.0), (25, -1.0, 10.0, 80.0)]:
        y = oracle.cheb_filter(cl, v, m, a0, a, b, bc=1)[0]
        g = oracle.filter_gain(lam, m, a0, a, b)
        assert np.abs(y - g * v).max() <= 1e-12 * max(1.0, abs(g)) * np.abs(v).max()


def test_unit_gain_at_a0():
    n, h = (10, 12, 11), 0.5
    lam, v = _eig_zero_bc(n, h, (0, 0, 0))
    cl = inputs.free_cluster(n, h)
    y = oracle.cheb_filter(cl, v, 24, lam, lam + 2.0, 50.0)[0]
    assert np.abs(y - v).max() < 1e-12


def _tiny_cluster(lmax=1, seed=7):
    return inputs.make_cluster((8, 9, 10), 1.0, 2, 4, lmax, seed, min_dist=0.0, margin=4.0)


@pytest.mark.parametrize("m", [1, 5, 20])
def test_filter_matches_dense_spectral_form(m):
    cl = _tiny_cluster(lmax=2)
    H = oracle.dense_hamiltonian(cl)
    lam, Q = np.linalg.eigh(H)
    a0, a, b = lam[0], lam[40] + 0.1, lam[-1] * 1.001
    rng = np.random.default_rng(2)
    X = rng.standard_normal((4, cl.nd))
    Y = oracle.cheb_filter(cl, X, m, a0, a, b)
    ref = (Q @ (oracle.filter_gain(lam, m, a0, a, b)[:, None] * (Q.T @ X.T))).T
    assert np.abs(Y - ref).max() < 1e-11 * np.abs(ref).max()


def test_scaled_vs_unscaled():
    cl = _tiny_cluster()
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2, cl.nd))
    m, a0, a, b = 12, -3.0, 1.0, 40.0
    Ys = oracle.cheb_filter(cl, X, m, a0, a, b, scaled=True)
    Yu = oracle.cheb_filter(cl, X, m, a0, a, b, scaled=False)
    e, c = (b - a) / 2, (b + a) / 2
    Cm = oracle.cheb_closed_form(m, np.array([(a0 - c) / e]))[0]
    assert np.abs(Yu - Cm * Ys).max() < 1e-11 * np.abs(Yu).max()


def test_commutes_with_h():
    cl = inputs.make_cluster(14, 0.5, 2, 4, 1, seed=3, min_dist=0.0, margin=3.0)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((2, cl.nd))
    args = (9, -2.5, 2.0, 45.0)
    lhs = oracle.cheb_filter(cl, oracle.h_apply(cl, X), *args)
    rhs = oracle.h_apply(cl, oracle.cheb_filter(cl, X, *args))
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()


def test_column_independence_and_linearity():
    cl = inputs.make_cluster(12, 0.5, 2, 4, 1, seed=5, min_dist=0.0, margin=3.0)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((3, cl.nd))
    args = (11, -2.0, 3.0, 48.0)
    Y = oracle.cheb_filter(cl, X, *args)
    for i in range(3):
        assert np.array_equal(Y[i], oracle.cheb_filter(cl, X[i], *args)[0])
    Z = oracle.cheb_filter(cl, 2.0 * X[0] - 0.5 * X[1], *args)[0]
    assert np.abs(Z - (2.0 * Y[0] - 0.5 * Y[1])).max() < 1e-12 * np.abs(Z).max()


def test_degree_one():
    cl = inputs.make_cluster(10, 0.6, 1, 4, 1, seed=9, min_dist=0.0, margin=3.0)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((2, cl.nd))
    a0, a, b = -4.0, 1.0, 30.0
    e, c = (b - a) / 2, (b + a) / 2
    s1 = e / (a0 - c)
    ref = (s1 / e) * (oracle.h_apply(cl, X) - c * X)
    Y = oracle.cheb_filter(cl, X, 1, a0, a, b)
    assert np.abs(Y - ref).max() < 1e-13 * np.abs(ref).max()


def _printed_algorithm(H, X, m, lam1, lamc, lamN):
    """Alg. 2 exactly as printed (used only to show it is not C_m-proportional)."""
    e = (lamN - lamc) / 2
    c = (lamN + lamc) / 2
    sigma = e / (lam1 - c)
    Psi = X.copy()
    Pf = (sigma / e) * (H @ Psi - c * Psi)
    for _ in range(2, m + 1):
        Pt = (2 * sigma / e) * (H @ Pf - c * Pf) - (sigma ** 2 / (2 - sigma ** 2)) * Psi
        Psi, Pf = Pf, Pt
        sigma = sigma / (2 - sigma ** 2)
    return Pf


def test_printed_algorithm_is_not_the_filter_but_oracle_is():
    cl = _tiny_cluster()
    H = oracle.dense_hamiltonian(cl)
    lam, Q = np.linalg.eigh(H)
    m, a0, a, b = 20, lam[0], lam[30] + 0.1, lam[-1] * 1.01
    rng = np.random.default_rng(0)
    x = rng.standard_normal(cl.nd)
    coeff = Q.T @ x
    gains = oracle.filter_gain(lam, m, a0, a, b)
    printed = Q.T @ _printed_algorithm(H, x, m, a0, a, b)
    ours = Q.T @ oracle.cheb_filter(cl, x, m, a0, a, b)[0]
    # ours reproduces the spectral gains; the printed recurrence does not (not even up to scale)
    assert np.allclose(ours, gains * coeff, atol=1e-11 * np.abs(coeff).max())
    ratio = printed / (gains * coeff)
    assert np.std(ratio) > 1e-3 * np.abs(np.mean(ratio))


# ----------------------------------------------------------------------------- Lanczos and RR

def test_lanczos_interlacing_and_bounds():
    cl = _tiny_cluster(lmax=2)
    lam = np.linalg.eigvalsh(oracle.dense_hamiltonian(cl))
    v0 = inputs.lanczos_start(cl.nd, 1)
    alpha, beta, theta = oracle.lanczos(cl, 40, v0)
    assert theta[0] >= lam[0] - 1e-10 and theta[-1] <= lam[-1] + 1e-10
    # Cauchy interlacing: the j-th smallest Ritz value is >= lambda_j, and the
    # j-th largest <= lambda_{N-j+1}
    k = len(theta)
    assert np.all(theta >= lam[:k] - 1e-9)
    assert np.all(theta[::-1] <= lam[::-1][:k] + 1e-9)
    # extremal Ritz values have converged after 40 steps on a 720-point grid
    assert abs(theta[0] - lam[0]) < 1e-6 and abs(theta[-1] - lam[-1]) < 1e-3 * abs(lam[-1])
    a0, a, b = oracle.select_bounds(theta, 8, ubound=oracle.upper_bound(cl))
    assert b >= lam[-1] and a0 >= lam[0] - 1e-10 and a0 < a < b


def test_lanczos_tridiagonal_is_projection():
    # T_k = V^T H V for the Lanczos basis: check alpha, beta against the dense H
    cl = _tiny_cluster()
    H = oracle.dense_hamiltonian(cl)
    v0 = inputs.lanczos_start(cl.nd, 2)
    k = 12
    alpha, beta, theta = oracle.lanczos(cl, k, v0)
    # rebuild the Krylov basis by plain Gram-Schmidt on the dense matrix
    V = np.zeros((k, cl.nd))
    V[0] = v0 / np.linalg.norm(v0)
    for j in range(1, k):
        w = H @ V[j - 1]
        for _ in range(2):
            w -= V[:j].T @ (V[:j] @ w)
        V[j] = w / np.linalg.norm(w)
    T = V @ H @ V.T
    assert np.allclose(np.diag(T), alpha, atol=1e-9)
    assert np.allclose(np.abs(np.diag(T, 1)), beta, atol=1e-9)
    assert np.allclose(np.sort(np.linalg.eigvalsh(T)), theta, atol=1e-9)


def test_rayleigh_ritz_invariant_subspace():
    # on an exactly invariant subspace (mixed eigenvectors) the Ritz values are the eigenvalues
    n, h, v0 = (11, 10, 12), 0.5, -0.4
    cl = inputs.free_cluster(n, h, v0=v0)
    idxs = [(0, 0, 0), (1, 0, 0), (0, 2, 1), (3, 1, 4), (2, 2, 2)]
    lams, vecs = zip(*[_eig_zero_bc(n, h, i) for i in idxs])
    lams = np.array(lams) + v0
    rng = np.random.default_rng(1)
    M = rng.standard_normal((5, 5))
    Y = M @ np.array(vecs)  # a non-orthogonal basis of the span
    theta, vec, Hs, Ms = oracle.rayleigh_ritz(cl, Y)
    assert np.allclose(theta, np.sort(lams), atol=1e-10)
    # rotated block spans the same eigenvectors
    R = oracle.rotate(Y, vec)
    HR = oracle.h_apply(cl, R)
    assert np.abs(HR - theta[:, None] * R).max() < 1e-9 * np.abs(R).max()


def test_rayleigh_ritz_matches_dense_projection():
    cl = _tiny_cluster(lmax=2)
    H = oracle.dense_hamiltonian(cl)
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((6, cl.nd))
    theta, vec, Hs, Ms = oracle.rayleigh_ritz(cl, Y)
    Qo, _ = np.linalg.qr(Y.T)
    ref = np.linalg.eigvalsh(Qo.T @ H @ Qo)
    assert np.allclose(theta, ref, atol=1e-9 * np.abs(ref).max())


# ----------------------------------------------------------------------------- filter bounds

# Ascending Ritz values with distinct gaps, so that an off-by-one in the cutoff
# index or a wrong shift gives a different number.
_THETA = np.array([-3.0, -2.5, -1.0, 0.0, 0.5, 1.25, 2.0, 2.75, 3.5, 10.0])


def test_select_bounds_exact_values():
    """Alg. 2 takes lambda_1, the cutoff lambda_c and lambda_Nd; the reading
    fixes lambda_1 := theta_1, lambda_c := theta_8 + 0.1 Ha (the 0.1 Ha margin
    of Sec. 4) and lambda_Nd := 1.01 theta_max.  Exact expected values:"""
    a0, a, b = oracle.select_bounds(_THETA, 8)
    assert (a0, a, b) == (-3.0, 2.75 + 0.1, 1.01 * 10.0)
    # the 8th value, not the 7th or 9th
    assert a != 2.0 + 0.1 and a != 3.5 + 0.1
    # input order does not matter
    perm = np.random.default_rng(3).permutation(len(_THETA))
    assert oracle.select_bounds(_THETA[perm], 8) == (a0, a, b)
    # other cutoff indices and shifts
    assert oracle.select_bounds(_THETA, 1, shift=0.25) == (-3.0, -3.0 + 0.25, 10.1)
    assert oracle.select_bounds(_THETA, 3, shift=0.5, bfactor=1.5) == (-3.0, -1.0 + 0.5, 15.0)


def test_select_bounds_upper_clamp_and_short_runs():
    # b is lowered to a guaranteed upper bound only when that is smaller
    assert oracle.select_bounds(_THETA, 8, ubound=9.0)[2] == 9.0
    assert oracle.select_bounds(_THETA, 8, ubound=11.0)[2] == 1.01 * 10.0
    assert oracle.select_bounds(_THETA, 8, ubound=10.1)[2] == 1.01 * 10.0
    # fewer Ritz values than wanted states: the cutoff sits above the largest
    th = np.array([-1.0, 4.0, 20.0])
    assert oracle.select_bounds(th, 8) == (-1.0, 20.0 + 0.1, 1.01 * 20.0)
    # bounds that do not satisfy a0 < a < b are refused
    with pytest.raises(ValueError):
        oracle.select_bounds(np.array([-1.0, 4.0, 5.0]), 8)      # a = 5.1 > b = 5.05
    with pytest.raises(ValueError):
        oracle.select_bounds(_THETA, 8, ubound=2.0)              # b below the cutoff


def test_select_bounds_on_exact_spectrum():
    """With the exact spectrum of a dense H as the Ritz values, the bounds
    bracket the spectrum as Alg. 2 needs: a0 is lambda_1 itself, the cutoff
    lies 0.1 Ha above lambda_8, and b is at least lambda_max."""
    cl = _tiny_cluster(lmax=2)
    lam = np.linalg.eigvalsh(oracle.dense_hamiltonian(cl))
    a0, a, b = oracle.select_bounds(lam, 8, ubound=oracle.upper_bound(cl))
    assert a0 == lam[0]
    assert a == lam[7] + 0.1
    assert np.sum(lam < a) >= 8 and lam[-1] <= b
