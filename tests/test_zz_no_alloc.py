"""H X without allocation (sparc_h_apply_noalloc), called through the C ABI,
against sparc_h_apply on the same inputs: two calls in a row, the second
with a smaller input, in FP64 and FP32, and a call whose projections do not
fit the fixed scratch array."""
import ctypes

import numpy as np
import pytest

from paper_1603_04334_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _call(b, op, X, Y):
    dt = b.SPARC_F64 if X.dtype == torch.float64 else b.SPARC_F32
    return b.lib().sparc_h_apply_noalloc(op.handle, dt, ctypes.c_void_p(X.data_ptr()), X.stride(0),
                                         ctypes.c_void_p(Y.data_ptr()), Y.stride(0), X.shape[0],
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_h_apply_twice(dtype):
    from paper_1603_04334_amd import binding as b
    b.lib()
    assert b.lib().sparc_noalloc_scratch_bytes() == 16 << 20
    big = inputs.make_cluster((28, 30, 32), 0.45, 4, 8, 2, seed=61, min_dist=0.0, margin=3.0)
    small = inputs.make_cluster((16, 18, 20), 0.5, 2, 8, 1, seed=62, min_dist=0.0, margin=2.5)
    for cl, ns in ((big, 37), (small, 3)):  # the second call is smaller
        op = b.Operator(cl)
        X = torch.from_numpy(np.random.default_rng(ns).standard_normal((ns, cl.nd))).to(dtype).cuda()
        ref = op.h_apply(X)
        Y = torch.full_like(X, float("nan"))
        assert _call(b, op, X, Y) == 0
        torch.cuda.synchronize()
        assert torch.equal(Y, ref)
        op.close()


def test_noalloc_rejects_oversize():
    from paper_1603_04334_amd import binding as b
    b.lib()
    cl = inputs.make_cluster((16, 16, 16), 0.5, 20, 8, 2, seed=63, min_dist=0.0, margin=2.0)
    op = b.Operator(cl)
    ns = 2000  # 180 projectors x 2000 columns x 8 splits x 8 bytes > 16 MiB
    X = torch.zeros((ns, cl.nd), dtype=torch.float64, device="cuda")
    Y = torch.empty_like(X)
    assert _call(b, op, X, Y) == b.SPARC_E_WORKSPACE
    assert "scratch" in b.lib().sparc_last_error().decode()
    # a width that fits runs
    assert _call(b, op, X[:100], Y[:100]) == 0
    torch.cuda.synchronize()
    op.close()
