"""Pins of the oracle's MLP (learned smoother network): BF16 decoding of known
bit patterns, closed-form special cases of the forward pass, and the analytic
gradient against central finite differences."""
import numpy as np
import pytest


def test_bf16_decoding(oracle):
    lib = oracle.lib()
    lib.or_bf16_value.restype = __import__("ctypes").c_double
    assert lib.or_bf16_value(0x3F80) == 1.0
    assert lib.or_bf16_value(0xC000) == -2.0
    assert lib.or_bf16_value(0x3E80) == 0.25
    assert lib.or_bf16_value(0x0000) == 0.0


def _bf16(x):
    """Round-to-nearest-even BF16 bits of float32 values (for building weights)."""
    import torch
    return torch.tensor(np.asarray(x, np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)


def test_forward_special_cases(oracle):
    P = oracle.MLP_NPARAM
    w = np.zeros(P, np.float32)
    w[P - 4:] = [0.5, -1.0, 2.0, 0.25]                 # b3 only: output is b3
    X = np.random.default_rng(0).standard_normal((5, 8))
    Y = oracle.mlp_forward(_bf16(w), X)
    assert np.array_equal(Y, np.tile([0.5, -1.0, 2.0, 0.25], (5, 1)))
    # one path: h1[0] = tanh(x0), h2[0] = tanh(h1[0]), y0 = 2 h2[0]
    w = np.zeros(P, np.float32)
    w[0] = 1.0                                         # W1[0][0]
    w[512 + 64] = 1.0                                  # W2[0][0]
    w[512 + 64 + 4096 + 64] = 2.0                      # W3[0][0]
    Y = oracle.mlp_forward(_bf16(w), X)
    assert np.allclose(Y[:, 0], 2 * np.tanh(np.tanh(X[:, 0])), rtol=1e-15, atol=0)
    assert np.all(Y[:, 1:] == 0)


def test_gradient_against_finite_differences(oracle):
    rng = np.random.default_rng(1)
    P = oracle.MLP_NPARAM
    w = rng.uniform(-0.3, 0.3, P)
    X = rng.standard_normal((7, 8))
    T = rng.standard_normal((7, 4))
    wb = _bf16(w)
    import ctypes as C
    oracle.lib().or_bf16_value.restype = C.c_double
    wv = np.array([oracle.lib().or_bf16_value(int(b)) for b in wb])
    loss, g = oracle.mlp_loss_grad(wb, X, T)
    assert loss == pytest.approx(oracle.mlp_loss_w(wv, X, T), rel=1e-15)
    idx = np.concatenate([rng.integers(0, P, 60), [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4991, 4992, 4995]])
    for k in idx:
        h = 1e-6 * max(1.0, abs(wv[k]))
        wp = wv.copy(); wp[k] += h
        wm = wv.copy(); wm[k] -= h
        fd = (oracle.mlp_loss_w(wp, X, T) - oracle.mlp_loss_w(wm, X, T)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])
