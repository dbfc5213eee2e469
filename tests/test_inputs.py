"""Host-side checks of the seeded synthetic cluster generator."""
import numpy as np

from paper_1603_04334_amd import inputs


def test_small_case_shape_and_placement():
    c = inputs.SMALL
    cl = inputs.make_cluster(c.n, c.h, c.natoms, c.zmax, c.lmax, c.seed, min_dist=c.min_dist)
    assert cl.nd == 24 ** 3 and len(cl.atoms) == 2
    L = (c.n + 1) * c.h
    for a in cl.atoms:
        assert np.all(a.pos >= 4.0) and np.all(a.pos <= L - 4.0)
        assert a.nproj == 4 and a.chi.shape == (4,) + a.ext
        for d in range(3):
            assert a.lo[d] >= 0 and a.lo[d] + a.ext[d] <= c.n
        assert 1 <= a.Z <= 4 and 0.8 <= a.sigma <= 1.2
        assert np.all(np.abs(a.gamma) <= 2.0)
        # gamma shared over m for each l
        assert a.gamma[1] == a.gamma[2] == a.gamma[3]
    assert cl.veff.max() <= 0.0


def test_reproducible_and_column_streams():
    a = inputs.orbitals(1000, 6, seed=3)
    b = inputs.orbitals(1000, 6, seed=3, cols=[4, 1])
    assert np.array_equal(a[4], b[0]) and np.array_equal(a[1], b[1])
    c1 = inputs.make_cluster(20, 0.5, 3, 8, 2, seed=9)
    c2 = inputs.make_cluster(20, 0.5, 3, 8, 2, seed=9)
    assert np.array_equal(c1.veff, c2.veff)
    assert all(np.array_equal(x.chi, y.chi) for x, y in zip(c1.atoms, c2.atoms))


def test_min_spacing_and_lmax2():
    cl = inputs.make_cluster(40, 0.4, 12, 8, 2, seed=2, min_dist=2.0)
    P = np.array([a.pos for a in cl.atoms])
    d = np.sqrt(((P[:, None] - P[None]) ** 2).sum(-1)) + np.eye(len(P)) * 1e9
    assert d.min() >= 2.0
    assert all(a.nproj == 9 for a in cl.atoms)


def test_real_harmonics_orthonormal():
    # quadrature over the sphere: int Y_a Y_b dOmega = delta_ab
    rng = np.random.default_rng(0)
    v = rng.standard_normal((200000, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    Y = np.array(inputs.real_ylm(2, v[:, 0], v[:, 1], v[:, 2]))
    G = (Y @ Y.T) * 4 * np.pi / v.shape[0]
    assert np.allclose(G, np.eye(9), atol=0.03)


def test_batch_and_serving_recipes():
    b = inputs.batch_recipe()
    assert len(b) == 64
    assert all(32 <= r["n"] <= 96 and r["n"] % 8 == 0 and 16 <= r["ns"] <= 128 and 16 <= r["m"] <= 28 for r in b)
    assert all(2 <= r["natoms"] <= 24 for r in b)
    s = inputs.serving_recipe(nclusters=10, rate=100.0)
    assert len(s) == 10 and all(r["steps"] == 5 for r in s)
    t = [r["t_arrive"] for r in s]
    assert all(x < y for x, y in zip(t, t[1:]))
    # the clusters do not depend on the rate; the arrivals scale with it
    s2 = inputs.serving_recipe(nclusters=10, rate=200.0)
    assert [r["cluster"] for r in s2] == [r["cluster"] for r in s]
    assert np.allclose([r["t_arrive"] for r in s2], [x / 2 for x in t])
    # N_s = N_e/2 + 30 with N_e the sum of the Z that make_cluster draws
    c = s[0]["cluster"]
    cl = inputs.make_cluster(c["n"], c["h"], c["natoms"], c["zmax"], c["lmax"], c["seed"])
    assert c["ne"] == sum(a.Z for a in cl.atoms)
    assert c["ns"] == min(256, max(8, (c["ne"] + 1) // 2 + 30))
