"""Pins of the oracle's repeated CheFSI passes (Sec. 3.4, last paragraph;
Sec. 4 cutoff rule) against the spectrum of the dense Hamiltonian of tiny
grids."""
import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs


@pytest.fixture(scope="module")
def tiny():
    cl = inputs.make_cluster((9, 10, 11), 0.55, 2, 6, 1, seed=17, min_dist=1.0, margin=1.5)
    lam = np.linalg.eigvalsh(oracle.dense_hamiltonian(cl))
    return cl, lam


def _bounds(cl, lam, ns):
    # Lanczos-style bounds: the lowest eigenvalue, a cutoff above the wanted
    # states, and the largest eigenvalue times 1.01
    return float(lam[0]), float(lam[ns - 1] + 0.1), float(1.01 * lam[-1])


def test_passes_converge_to_the_lowest_eigenvalues(tiny):
    """Three passes from a random block (the first-SCF rule) bring the
    occupied Ritz values to the exact lowest eigenvalues; every Ritz value of
    every pass lies above its exact counterpart (min-max), and the error of
    the occupied states shrinks from pass to pass."""
    cl, lam = tiny
    ns, ne, m = 20, 16.0, 20
    a0, a, b = _bounds(cl, lam, ns)
    X = inputs.orbitals(cl.nd, ns, 3)
    _, rec = oracle.chefsi_passes(cl, X, m, 4, ne, a0, a, b)
    nocc = int(ne // 2)
    errs = []
    for r in rec:
        th = r["theta"]
        assert np.all(th >= lam[:ns] - 1e-10)
        errs.append(float(np.max(th[:nocc] - lam[:nocc])))
    assert errs[2] < 1e-7 and errs[3] < 1e-9, errs
    assert errs[0] > errs[1] > errs[2] > errs[3], errs


def test_fermi_level_and_cutoff_rule(tiny):
    """Each pass reports the Fermi level of its own Ritz values; the cutoff
    of every later pass is that Fermi level plus 0.1 Ha, and with converged
    states and an even electron count the Fermi level lies between the
    highest occupied and the lowest empty exact eigenvalue."""
    cl, lam = tiny
    ns, ne, m = 14, 16.0, 12
    a0, a, b = _bounds(cl, lam, ns)
    _, rec = oracle.chefsi_passes(cl, inputs.orbitals(cl.nd, ns, 4), m, 3, ne, a0, a, b)
    assert rec[0]["cutoff"] == a
    for p in range(1, 3):
        assert rec[p]["cutoff"] == rec[p - 1]["lambda_f"] + 0.1
    for r in rec:
        g = oracle.occupations(r["theta"], r["lambda_f"])
        assert abs(2.0 * g.sum() - ne) < 1e-9
    assert lam[7] - 1e-9 < rec[-1]["lambda_f"] < lam[8] + 1e-9


def test_rotated_block_is_orthonormal_ritz_basis(tiny):
    """The rotation returns M_s-orthonormal Ritz vectors: Psi^T Psi = I and
    Psi^T H Psi = diag(theta) for the last pass."""
    cl, lam = tiny
    ns = 10
    a0, a, b = _bounds(cl, lam, ns)
    Psi, rec = oracle.chefsi_passes(cl, inputs.orbitals(cl.nd, ns, 5), [8, 12], 2, 12.0, a0, a, b)
    assert rec[0]["degree"] == 8 and rec[1]["degree"] == 12
    G = Psi @ Psi.T
    assert np.abs(G - np.eye(ns)).max() < 1e-10
    Hs = Psi @ oracle.h_apply(cl, Psi).T
    assert np.abs(Hs - np.diag(rec[-1]["theta"])).max() < 1e-9


def test_a0_above_the_cutoff_is_lowered(tiny):
    """A lambda_1 estimate a0 above the first pass's Fermi level + 0.1 Ha
    (a Lanczos estimate that had not converged): the next pass takes a0 =
    the lowest Ritz value of the previous pass, and since a0 only scales
    the filter's output, every pass's Ritz values and Fermi level equal
    those of the same passes run with the exact lambda_1."""
    cl, lam = tiny
    ns, ne, m = 12, 2.0, 16
    _, a, b = _bounds(cl, lam, ns)
    X = inputs.orbitals(cl.nd, ns, 6)
    high = float(lam[6])
    _, rec = oracle.chefsi_passes(cl, X, m, 3, ne, high, a, b)
    _, ref = oracle.chefsi_passes(cl, X, m, 3, ne, float(lam[0]), a, b)
    assert rec[0]["lambda_f"] + 0.1 <= high  # the case this pins
    assert rec[0]["a0"] == high and rec[1]["a0"] == rec[0]["theta"][0] and rec[2]["a0"] == rec[1]["a0"]
    assert all(r["a0"] == lam[0] for r in ref)
    for r, q in zip(rec, ref):
        # equal to rounding: the low states to the last bits, the damped
        # ones (above the cutoff) with the filter's rounding amplified by its
        # damping ratio
        assert np.abs(r["theta"][:4] - q["theta"][:4]).max() < 1e-12
        assert np.abs(r["theta"] - q["theta"]).max() < 1e-8
        assert abs(r["lambda_f"] - q["lambda_f"]) < 1e-12
    assert abs(rec[-1]["theta"][0] - lam[0]) < 1e-8
