"""The allocation-free variant of the surrogate's loss and gradient
(pic1d_mlp_loss_grad_static), called through the C ABI, against the workspace
entry point pic1d_mlp_loss_grad on the same inputs: two calls in a row, the
second with a smaller batch, so that the second reads a scratch array the first
left filled.  Both run the same kernels in the same order, so the results agree
to the bit."""
import ctypes

import numpy as np
import pytest

from paper_2609_17661_amd import pic1d

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _inputs(seed, n):
    from oracle import mlp as omlp
    rng = np.random.default_rng(seed)
    X = (omlp.IN_LO + (omlp.IN_HI - omlp.IN_LO) * rng.random((n, 4))).astype(np.float32)
    T = rng.standard_normal((n, 3)).astype(np.float32)
    return X, T


def _params(seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(pic1d.mlp_param_count()) * 0.08).astype(np.float32)


def test_static_scratch_loss_grad_equals_the_workspace_entry_point():
    import torch
    p = torch.from_numpy(_params(5)).cuda()
    for n in (2048, 777):
        X, T = _inputs(100 + n, n)
        x = torch.from_numpy(X).cuda()
        t = torch.from_numpy(T).cuda()
        _print("loss_grad_static n", n)
        l_ref, g_ref = pic1d.mlp_loss_grad(p, x, t)
        l_st, g_st = pic1d.mlp_loss_grad_static(p, x, t)
        torch.cuda.synchronize()
        a = g_st.cpu().numpy()
        b = g_ref.cpu().numpy()
        _print("  loss", l_st, l_ref, "max |dg|", float(np.abs(a - b).max()))
        assert np.isfinite(l_ref) and l_ref > 0.0
        assert l_st == l_ref
        np.testing.assert_array_equal(a, b)


def test_static_scratch_rejects_batches_beyond_its_maximum():
    import torch
    lib = pic1d.load()
    p = torch.from_numpy(_params(6)).cuda()
    X, T = _inputs(7, 2049)
    x = torch.from_numpy(X).cuda()
    t = torch.from_numpy(T).cuda()
    g = torch.empty(pic1d.mlp_param_count(), dtype=torch.float32, device="cuda")
    loss = ctypes.c_double(0.0)
    # checked on the host before anything is launched
    rc = lib.pic1d_mlp_loss_grad_static(ctypes.c_void_p(p.data_ptr()), 2049, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                        ctypes.byref(loss), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1
    assert b"2048" in lib.pic1d_last_error(None)
