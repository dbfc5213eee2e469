"""Dump of a filter job to .npz and its reload (host side; the replay itself
is a GPU test in test_gpu_replay.py)."""
import os

import numpy as np

from paper_1603_04334_amd import inputs, replay

BUILD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build")


def test_job_roundtrip_is_exact():
    cl = inputs.make_cluster((9, 10, 11), 0.55, 3, 6, 2, seed=4, min_dist=0.0, margin=1.5)
    rng = np.random.default_rng(1)
    for dt in (np.float64, np.float32):
        X = rng.standard_normal((3, cl.nd)).astype(dt)
        Y = rng.standard_normal((3, cl.nd)).astype(dt)
        os.makedirs(BUILD, exist_ok=True)
        path = os.path.join(BUILD, f"job_{np.dtype(dt).name}.npz")
        replay.save_filter_job(path, cl, X, 7, -2.0, 1.5, 30.0, Y)
        c2, X2, m, bounds, Y2 = replay.load_filter_job(path)
        assert (c2.n, c2.h, c2.radius, c2.seed) == (cl.n, cl.h, cl.radius, cl.seed)
        assert np.array_equal(c2.veff, cl.veff)
        assert len(c2.atoms) == len(cl.atoms)
        for a, b in zip(c2.atoms, cl.atoms):
            assert (a.lo, a.ext, a.Z) == (b.lo, b.ext, b.Z)
            assert np.array_equal(a.chi, b.chi) and np.array_equal(a.gamma, b.gamma)
            assert np.array_equal(a.pos, b.pos) and a.sigma == b.sigma
        assert X2.dtype == dt and np.array_equal(X2, X) and np.array_equal(Y2, Y)
        assert m == 7 and bounds == (-2.0, 1.5, 30.0)
        # plain arrays only: loadable without unpickling
        with np.load(path, allow_pickle=False) as z:
            assert "X" in z.files and "chi" in z.files
