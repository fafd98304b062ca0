"""Pins of the oracle's direct periodic 3x3x3 convolution (learned warm start).

Forward: against torch's conv3d with circular padding (a library routine,
CPU, float64).  Backward: against central finite differences of a scalar
loss, and against torch autograd.
"""
import numpy as np
import pytest

import oracle


def _rand(seed, cin=3, cout=4, n=(6, 4, 8)):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((cin, n[2], n[1], n[0]))
    w = rng.standard_normal((cout, cin, 3, 3, 3))
    b = rng.standard_normal(cout)
    return x, w, b, n


def test_conv_forward_matches_torch_circular():
    torch = pytest.importorskip("torch")
    x, w, b, n = _rand(0)
    y = oracle.conv3d_fwd(x, w, b, n)
    xt = torch.from_numpy(x)[None]
    xp = torch.nn.functional.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular")
    yt = torch.nn.functional.conv3d(xp, torch.from_numpy(w), torch.from_numpy(b))[0].numpy()
    np.testing.assert_allclose(y, yt, atol=1e-12)


def test_conv_backward_matches_finite_differences():
    x, w, b, n = _rand(1, cin=2, cout=3, n=(4, 4, 4))
    rng = np.random.default_rng(2)
    g = rng.standard_normal((3,) + x.shape[1:])  # dL/dy for L = <g, y>

    def L(xx, ww, bb):
        return float(np.sum(g * oracle.conv3d_fwd(xx, ww, bb, n)))

    dx = oracle.conv3d_bwd_data(g, w, n)
    dw, db = oracle.conv3d_bwd_weight(x, g, 2, 3, n)
    eps = 1e-6
    for idx in [(0, 1, 2, 3), (1, 0, 0, 0), (1, 3, 3, 3)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (L(xp, w, b) - L(xm, w, b)) / (2 * eps)
        assert abs(fd - dx[idx]) < 1e-7 * max(1, abs(fd))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 1, 2, 2, 2)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += eps
        wm[idx] -= eps
        fd = (L(x, wp, b) - L(x, wm, b)) / (2 * eps)
        assert abs(fd - dw[idx]) < 1e-7 * max(1, abs(fd))
    for c in range(3):
        bp, bm = b.copy(), b.copy()
        bp[c] += eps
        bm[c] -= eps
        fd = (L(x, w, bp) - L(x, w, bm)) / (2 * eps)
        assert abs(fd - db[c]) < 1e-7 * max(1, abs(fd))


def test_conv_backward_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    x, w, b, n = _rand(3)
    g = np.random.default_rng(4).standard_normal((4,) + x.shape[1:])
    xt = torch.from_numpy(x)[None].requires_grad_(True)
    wt = torch.from_numpy(w).requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    xp = torch.nn.functional.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular")
    y = torch.nn.functional.conv3d(xp, wt, bt)
    (y[0] * torch.from_numpy(g)).sum().backward()
    np.testing.assert_allclose(oracle.conv3d_bwd_data(g, w, n), xt.grad[0].numpy(), atol=1e-11)
    dw, db = oracle.conv3d_bwd_weight(x, g, 3, 4, n)
    np.testing.assert_allclose(dw, wt.grad.numpy(), atol=1e-10)
    np.testing.assert_allclose(db, bt.grad.numpy(), atol=1e-11)
