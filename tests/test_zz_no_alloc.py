"""GPU: the MLP gradient entry point that allocates nothing
(amg_mlp_backward_noalloc, deltas in the library's static device array)
against amg_mlp_backward with a caller workspace, called through the C ABI:
two calls in a row, the second with fewer samples, bit for bit; the
over-size batch is rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def test_backward_noalloc_equals_workspace_form():
    from paper_2511_21268_amd import amg
    assert torch.cuda.is_available()
    L = amg.lib()
    from paper_2511_21268_amd.learned import Trainer
    tr = Trainer(seed=9)
    rng = np.random.default_rng(21)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for B in (3001, 45):
        print(f"case mlp backward noalloc B={B}", flush=True)
        X = torch.from_numpy(rng.standard_normal((B, amg.MLP_NFEAT)).astype(np.float32)).cuda()
        T = torch.from_numpy(rng.standard_normal((B, 4)).astype(np.float32)).cuda()
        act = torch.empty(B, amg.MLP_NACT, dtype=torch.float32, device="cuda")
        Y = torch.empty(B, 4, dtype=torch.float32, device="cuda")
        amg._check(L.amg_mlp_forward(_ptr(tr.w), _ptr(X), B, _ptr(Y), _ptr(act), st))
        dl = torch.empty(B, amg.MLP_NDEL, dtype=torch.float32, device="cuda")
        g_ref = torch.full((amg.MLP_NPARAM,), np.nan, dtype=torch.float32, device="cuda")
        l_ref = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
        amg._check(L.amg_mlp_backward(_ptr(tr.w), _ptr(X), _ptr(act), _ptr(Y), _ptr(T), B, _ptr(dl),
                                      _ptr(g_ref), _ptr(l_ref), st))
        g = torch.full((amg.MLP_NPARAM,), np.nan, dtype=torch.float32, device="cuda")
        loss = torch.full((1,), np.nan, dtype=torch.float32, device="cuda")
        amg._check(L.amg_mlp_backward_noalloc(_ptr(tr.w), _ptr(X), _ptr(act), _ptr(Y), _ptr(T), B,
                                              _ptr(g), _ptr(loss), st))
        torch.cuda.synchronize()
        assert torch.isfinite(g).all() and torch.isfinite(loss).all()
        assert torch.equal(g, g_ref) and torch.equal(loss, l_ref)
        # and the gradient is the one of the mean squared error (finite check of the loss)
        ref_loss = float(((Y - T) ** 2).mean())
        assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss
    X1 = torch.zeros(1, amg.MLP_NFEAT, dtype=torch.float32, device="cuda")
    g1 = torch.zeros(amg.MLP_NPARAM, dtype=torch.float32, device="cuda")
    st_code = L.amg_mlp_backward_noalloc(_ptr(tr.w), _ptr(X1), _ptr(X1), _ptr(X1), _ptr(X1),
                                         amg.MLP_NOALLOC_MAX_B + 1, _ptr(g1), None, st)
    assert st_code == amg.AMG_ERR_ARG
    assert b"exceeds" in L.amg_last_error()
