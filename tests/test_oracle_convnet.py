"""Pins of the FP64 warm-start-network reference (oracle/convnet.py) against
independent routines: scipy's 2D correlation with wrap boundaries, torch's
bf16 rounding, and finite differences of the loss."""
import numpy as np
import pytest
from scipy import signal

from oracle import convnet


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 500), [1.0, 1 + 2 ** -8,
                       1 + 3 * 2 ** -9, -2.5, 0.0]]).astype(np.float32)
    want = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(convnet.bf16(x), want)


def test_conv_forward_is_periodic_correlation():
    rng = np.random.default_rng(4)
    n, h, w, cin, cout = 2, 7, 9, 3, 4
    x = rng.normal(0, 1, (n, h, w, cin))
    W = rng.normal(0, 1, (9, cout, cin))
    b = rng.normal(0, 1, cout)
    out = convnet.conv_fwd(x, W, b)
    for k in range(n):
        for co in range(cout):
            ref = np.full((h, w), b[co])
            for ci in range(cin):
                K = W[:, co, ci].reshape(3, 3)  # K[dy + 1, dx + 1]
                ref += signal.correlate2d(x[k, :, :, ci], K, mode="same", boundary="wrap")
            assert np.allclose(out[k, :, :, co], ref, atol=1e-12)


def test_conv_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    n, h, w, cin, cout = 1, 5, 6, 2, 3
    x = rng.normal(0, 1, (n, h, w, cin))
    W = rng.normal(0, 1, (9, cout, cin))
    b = rng.normal(0, 1, cout)
    dout = rng.normal(0, 1, (n, h, w, cout))
    for relu_in in (False, True):
        da, dW, db = convnet.conv_bwd(x, W, dout, relu_in=relu_in)
        L = lambda x_, W_, b_: float((dout * convnet.conv_fwd(x_, W_, b_, relu_in=relu_in)).sum())
        eps = 1e-6
        for idx in [(0, 1, 2, 0), (0, 4, 5, 1), (0, 0, 0, 1)]:
            if relu_in and abs(x[idx]) < 1e-3:
                continue
            xp, xm = x.copy(), x.copy()
            xp[idx] += eps
            xm[idx] -= eps
            assert da[idx] == pytest.approx((L(xp, W, b) - L(xm, W, b)) / (2 * eps), rel=1e-6, abs=1e-8)
        for idx in [(0, 0, 0), (4, 2, 1), (8, 1, 0)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            assert dW[idx] == pytest.approx((L(x, Wp, b) - L(x, Wm, b)) / (2 * eps), rel=1e-6)
        assert np.allclose(db, dout.sum(axis=(0, 1, 2)))


def test_net_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    shapes = [(3, 4), (4, 4), (4, 2)]
    params = [(rng.normal(0, 0.5, (9, co, ci)), rng.normal(0, 0.1, co)) for ci, co in shapes]
    x = rng.normal(0, 1, (2, 5, 5, 3))
    y = rng.normal(0, 1, (2, 5, 5, 2))

    def loss(ps):
        zs = convnet.net_forward(x, ps)
        return convnet.mse(zs[-1], y, 2)

    l0, g = loss(params)
    grads = convnet.net_backward(convnet.net_forward(x, params), params, g)
    eps = 1e-6
    for l, idx in [(0, (0, 1, 2)), (1, (4, 3, 3)), (2, (8, 1, 0)), (1, (2, 0, 1))]:
        pp = [(W.copy(), b.copy()) for W, b in params]
        pm = [(W.copy(), b.copy()) for W, b in params]
        pp[l][0][idx] += eps
        pm[l][0][idx] -= eps
        fd = (loss(pp)[0] - loss(pm)[0]) / (2 * eps)
        assert grads[l][0][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)
