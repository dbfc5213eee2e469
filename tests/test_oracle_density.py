"""Pins of the oracle's occupations, Fermi level and electron density
(Sec. 3.4 Eq. FermiEnergyConstraintFormulation and the density that
follows; k_B T = 1e-3 Ha from Sec. 4)."""
import math

import numpy as np
import pytest

import oracle
from paper_1603_04334_amd import inputs

KT = 1e-3


def test_occupations_closed_forms():
    # g = 1/2 at the Fermi level, g(l_f + d) = 1 - g(l_f - d), exp tails
    g = oracle.occupations([0.3, 0.3 + 2e-3, 0.3 - 2e-3, 0.3 + 0.5, 0.3 - 1.0], 0.3, KT)
    assert g[0] == 0.5
    assert abs(g[1] + g[2] - 1.0) < 1e-15
    assert abs(g[1] - 1.0 / (1.0 + math.e ** 2)) < 1e-15
    # far above the Fermi level g ~ exp(-500), representable without overflow
    assert abs(g[3] / math.exp(-500.0) - 1.0) < 1e-12
    assert g[4] == 1.0


def test_fermi_level_two_levels_symmetric():
    # two levels and two electrons: g_1 + g_2 = 1 forces l_f to the midpoint
    # (gaps of up to 1.2 Ha = 1200 kT, where the tails are still representable)
    for a, b in ((-0.6, 0.6), (-0.37, 0.0025), (2.0, 2.0001)):
        lf = oracle.fermi_level([a, b], 2.0, KT)
        assert abs(lf - 0.5 * (a + b)) < 1e-12


def test_fermi_level_degenerate_closed_form():
    # N_s equal levels at e: 2 N_s g = N_e, so l_f = e - kT ln(2 N_s / N_e - 1)
    for ns, ne in ((5, 3.0), (40, 17.0), (8, 15.5)):
        e = -0.8
        lf = oracle.fermi_level([e] * ns, ne, KT)
        assert abs(lf - (e - KT * math.log(2.0 * ns / ne - 1.0))) < 1e-12


def test_fermi_level_constraint_and_gap():
    rng = np.random.default_rng(5)
    th = np.sort(rng.uniform(-2.0, 1.0, 60))
    for ne in (10.0, 37.0, 80.0, 119.0):
        lf = oracle.fermi_level(th, ne, KT)
        assert abs(2.0 * oracle.occupations(th, lf, KT).sum() - ne) < 1e-9
    # an even count with a gap much wider than kT: l_f sits inside the gap,
    # the occupied states are filled and the empty ones are empty
    th = np.array([-1.0, -0.9, -0.85, -0.2, -0.1, 0.4])
    lf = oracle.fermi_level(th, 6.0, KT)
    assert -0.85 < lf < -0.2
    g = oracle.occupations(th, lf, KT)
    assert np.all(g[:3] == 1.0) and np.all(g[3:] < 1e-100)
    # midway between the highest filled and the lowest empty level
    assert abs(lf - 0.5 * (-0.85 - 0.2)) < 1e-12
    with pytest.raises(ValueError):
        oracle.fermi_level(th, 12.0, KT)


def test_density_integrates_to_electron_count():
    """With orthonormal orbitals (columns of an orthogonal matrix, as the
    rotation returns them) the midpoint-rule integral h^3 sum_x rho(x) equals
    2 sum_n g_n = N_e."""
    rng = np.random.default_rng(7)
    nd, ns, h = 900, 12, 0.4
    Q, _ = np.linalg.qr(rng.standard_normal((nd, ns)))
    th = np.sort(rng.uniform(-1.0, 0.5, ns))
    ne = 15.0
    lf = oracle.fermi_level(th, ne, KT)
    g = oracle.occupations(th, lf, KT)
    rho = oracle.density(Q.T, g, h)
    assert abs(h ** 3 * rho.sum() - ne) < 1e-10
    assert np.all(rho >= 0)


def test_density_single_state_closed_form():
    # one sine orbital of a grid, fully occupied: rho = 2 psi^2 / h^3
    n, h = (6, 7, 8), 0.5
    psi = np.einsum("i,j,k->ijk", *[np.sin(np.pi * np.arange(1, m + 1) / (m + 1)) for m in n]).reshape(-1)
    psi /= np.linalg.norm(psi)
    rho = oracle.density(psi, [1.0], h)
    assert np.allclose(rho, 2.0 * psi ** 2 / h ** 3, rtol=0, atol=1e-15)
    # linear in the occupations and additive over orbitals
    rho2 = oracle.density(np.stack([psi, psi]), [0.25, 0.5], h)
    assert np.allclose(rho2, 0.75 * rho, rtol=1e-15)
