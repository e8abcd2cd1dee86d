"""The allocation-free weight gradient (lbm_net_conv3x3_bwd_weight_noalloc)
against the workspace entry point (lbm_net_conv3x3_bwd_weight): the same
kernels and summation order, so the results must be bitwise equal.  Two
calls in a row, the second on a smaller input, so the second runs on a
scratch array still holding the first call's partials."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _case(n, h, w, cin, cout, creal, relu, seed):
    from paper_0710_5470_amd import lbm
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, h, w, cin)).astype(np.float32)
    dout = rng.normal(0, 1, (n, h, w, cout)).astype(np.float32)
    dout[..., creal:] = 0.0
    dev = torch.device("cuda")
    tx, td = torch.tensor(x, device=dev), torch.tensor(dout, device=dev)
    return lbm._shape(n, h, w, cin, cout, creal), x, dout, tx, td


def _workspace_result(s, td, tx, relu, cin, cout):
    from paper_0710_5470_amd import lbm
    dev = tx.device
    ws = torch.empty(lbm.lbm_net_conv3x3_bwd_weight_workspace(s), dtype=torch.uint8, device=dev)
    dW = torch.full((9, cout, cin), float("nan"), device=dev)
    db = torch.full((cout,), float("nan"), device=dev)
    lbm.lbm_net_conv3x3_bwd_weight(s, td, tx, relu, dW, db, ws)
    torch.cuda.synchronize()
    return dW.cpu().numpy(), db.cpu().numpy()


def test_noalloc_weight_gradient_equals_workspace_entry_point():
    from oracle import convnet
    from paper_0710_5470_amd import lbm
    # first the network's training shape (16 images of 128^2, 32 -> 32
    # channels: 256 partials, 9.5 MB of the 16 MiB scratch), then a smaller,
    # ragged one (3 partials, the last of 32 pixels)
    cases = [(16, 128, 128, 32, 32, 32, True, 11), (2, 40, 26, 16, 32, 3, False, 12)]
    for n, h, w, cin, cout, creal, relu, seed in cases:
        _say("noalloc bwd weight", n, h, w, cin, cout, creal, relu)
        s, x, dout, tx, td = _case(n, h, w, cin, cout, creal, relu, seed)
        dW = torch.full((9, cout, cin), float("nan"), device=tx.device)
        db = torch.full((cout,), float("nan"), device=tx.device)
        lbm.lbm_net_conv3x3_bwd_weight_noalloc(s, td, tx, relu, dW, db)
        torch.cuda.synchronize()
        g_w, g_b = dW.cpu().numpy(), db.cpu().numpy()
        r_w, r_b = _workspace_result(s, td, tx, relu, cin, cout)
        assert np.isfinite(g_w).all() and np.isfinite(g_b).all()
        assert np.array_equal(g_w, r_w) and np.array_equal(g_b, r_b)
        if n * h * w <= 4096:  # the smaller case also against the FP64 reference
            _, dWr, dbr = convnet.conv_bwd(x.astype(np.float64), np.zeros((9, cout, cin)),
                                           dout.astype(np.float64), relu_in=relu, round_bf16=True)
            e = max(float(np.abs(g_w - dWr).max() / np.abs(dWr).max()),
                    float(np.abs(g_b - dbr).max() / np.abs(dbr).max()))
            _say("  rel err against the reference %.2e" % e)
            assert e < 1e-4


def test_noalloc_rejects_inputs_beyond_the_scratch():
    """32 images of 128^2 at 32 -> 32 channels need 512 partials (18.9 MB):
    LBM_E_LIMIT, and the outputs are not touched."""
    from paper_0710_5470_amd import lbm
    _say("noalloc limit")
    s = lbm._shape(32, 128, 128, 32, 32, 32)
    assert lbm.lbm_net_conv3x3_bwd_weight_workspace(s) > 16 << 20
    dev = torch.device("cuda")
    tx = torch.zeros(16, device=dev)
    dW = torch.full((9, 32, 32), 7.0, device=dev)
    db = torch.full((32,), 7.0, device=dev)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.lbm_net_conv3x3_bwd_weight_noalloc(s, tx, tx, True, dW, db)
    assert ei.value.code == lbm.E_LIMIT
    torch.cuda.synchronize()
    assert bool((dW == 7.0).all()) and bool((db == 7.0).all())
