"""A filter job dumped to .npz and replayed through the library gives the same
block bit for bit (FP64 and FP32)."""
import os

import numpy as np
import pytest

from paper_1603_04334_amd import inputs, replay

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BUILD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_replay_reproduces_the_job(dtype):
    from paper_1603_04334_amd import binding
    cl = inputs.make_cluster((13, 12, 16), 0.5, 2, 6, 1, seed=9, min_dist=0.0, margin=2.0)
    X = torch.from_numpy(inputs.orbitals(cl.nd, 5, 2)).to(dtype).cuda()
    op = binding.Operator(cl)
    Y = op.cheb_filter(X, 9, -3.0, 1.0, 60.0)
    os.makedirs(BUILD, exist_ok=True)
    path = os.path.join(BUILD, f"replay_{str(dtype)[-7:]}.npz")
    replay.save_filter_job(path, cl, X, 9, -3.0, 1.0, 60.0, Y)
    Yn, Ys, same = replay.replay_filter_job(path)
    assert same and Yn.dtype == Ys.dtype and np.array_equal(Yn, Y.cpu().numpy())
