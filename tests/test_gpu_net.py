"""GPU tests of the warm-start network kernels (bf16 MFMA, FP32 accumulate)
against the FP64 reference, which rounds the same matrix-core operands to
bf16, and of the learned warm start itself."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.mark.parametrize("n,h,w,cin,cout,creal,relu", [(2, 16, 24, 16, 32, 32, False),
                                                       (1, 32, 32, 32, 32, 32, True),
                                                       (3, 8, 16, 32, 16, 3, True),
                                                       (1, 128, 128, 16, 32, 32, False)])
def test_conv_kernels_match_reference(n, h, w, cin, cout, creal, relu):
    from oracle import convnet
    from paper_0710_5470_amd import lbm
    _say("conv", n, h, w, cin, cout, creal, relu)
    rng = np.random.default_rng(n * 1000 + h + cin + cout)
    x = rng.normal(0, 1, (n, h, w, cin)).astype(np.float32)
    W = rng.normal(0, 0.3, (9, cout, cin)).astype(np.float32)
    W[:, creal:, :] = 0.0
    b = rng.normal(0, 0.1, cout).astype(np.float32)
    b[creal:] = 0.0
    dout = rng.normal(0, 1, (n, h, w, cout)).astype(np.float32)
    dout[..., creal:] = 0.0
    dev = torch.device("cuda")
    tx, tW, tb, td = (torch.tensor(a, device=dev) for a in (x, W, b, dout))
    s = lbm._shape(n, h, w, cin, cout, creal)
    out = torch.empty(n, h, w, cout, device=dev)
    lbm.lbm_net_conv3x3_fwd(s, tx, relu, tW, tb, out)
    din = torch.empty_like(tx)
    lbm.lbm_net_conv3x3_bwd_data(s, td, tW, tx if relu else None, din)
    ws = torch.empty(lbm.lbm_net_conv3x3_bwd_weight_workspace(s), dtype=torch.uint8, device=dev)
    dW = torch.empty_like(tW)
    db = torch.empty_like(tb)
    lbm.lbm_net_conv3x3_bwd_weight(s, td, tx, relu, dW, db, ws)
    torch.cuda.synchronize()
    ref = convnet.conv_fwd(x.astype(np.float64), W.astype(np.float64), b.astype(np.float64),
                           relu_in=relu, round_bf16=True)
    ref[..., creal:] = 0.0
    da, dWr, dbr = convnet.conv_bwd(x.astype(np.float64), W.astype(np.float64),
                                    dout.astype(np.float64), relu_in=relu, round_bf16=True)
    e = (_rel(out.cpu().numpy(), ref), _rel(din.cpu().numpy(), da), _rel(dW.cpu().numpy(), dWr),
         _rel(db.cpu().numpy(), dbr))
    _say("rel errors fwd %.2e data %.2e weight %.2e bias %.2e" % e)
    assert max(e) < 1e-4


def test_network_gradient_matches_reference():
    """Loss and all 12 parameter gradients of the 6-layer network."""
    from oracle import convnet
    from paper_0710_5470_amd import warmstart
    net = warmstart.WarmNet(seed=3)
    rng = np.random.default_rng(9)
    x = np.zeros((2, 32, 32, 16), dtype=np.float32)
    x[..., :6] = rng.normal(0, 1, (2, 32, 32, 6))
    y = np.zeros((2, 32, 32, 16), dtype=np.float32)
    y[..., :3] = rng.normal(0, 1, (2, 32, 32, 3))
    dev = torch.device("cuda")
    loss, grads = net.loss_and_grad(torch.tensor(x, device=dev), torch.tensor(y, device=dev))
    params = net.numpy_params()
    zs = convnet.net_forward(x.astype(np.float64), params, round_bf16=True)
    lref, g = convnet.mse(zs[-1], y.astype(np.float64), 3)
    gref = convnet.net_backward(zs, params, g, round_bf16=True)
    assert loss == pytest.approx(lref, rel=1e-3)
    for l, ((dW, db), (dWr, dbr)) in enumerate(zip(grads, gref)):
        a, b = dW.cpu().numpy(), dWr
        err = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say("layer %d weight-gradient relative error %.2e" % (l, err))
        assert err < 2e-2
        assert np.linalg.norm(db.cpu().numpy() - dbr) / np.linalg.norm(dbr) < 2e-2


def test_training_reduces_loss():
    from paper_0710_5470_amd import warmstart
    net = warmstart.WarmNet(seed=5)
    rng = np.random.default_rng(11)
    x = np.zeros((4, 32, 32, 16), dtype=np.float32)
    x[..., :6] = rng.normal(0, 1, (4, 32, 32, 6))
    y = np.zeros((4, 32, 32, 16), dtype=np.float32)
    y[..., 0] = 0.5 * x[..., 5] + 0.25 * np.roll(x[..., 5], 1, axis=1)
    dev = torch.device("cuda")
    tx, ty = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    l0 = net.train_step(tx, ty, 1e-3)
    for _ in range(150):
        l1 = net.train_step(tx, ty, 1e-3)
    assert l1 < 0.2 * l0
