"""TEST INFRASTRUCTURE ONLY: FP64 reference of the warm-start network.

Plain numpy, written from the definition of a periodic 3x3 convolution:
    out[n, y, x, co] = b[co] + sum_{dy, dx, ci} W[tap][co][ci] a(in[n, y+dy, x+dx, ci])
with tap = 3 (dy + 1) + (dx + 1), indices taken modulo the image size, and
a = max(., 0) when the input is a relu'd pre-activation.  Backward passes
are the adjoints of that linear map.  Optionally rounds the operands that
the GPU feeds to its bf16 matrix cores (activations and weights) to bf16
(round to nearest even) so both sides multiply the same numbers; the sums
stay FP64 here.
"""
import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(a):
    """Round FP32-representable values to bf16, nearest even."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _shift(x, dy, dx):
    """y[n, i, j] = x[n, i + dy, j + dx] (periodic)."""
    return np.roll(np.roll(x, -dy, axis=1), -dx, axis=2)


def conv_fwd(x, W, b, relu_in=False, round_bf16=False):
    """x [n, h, w, cin], W [9, cout, cin], b [cout] -> [n, h, w, cout]."""
    a = np.maximum(x, 0.0) if relu_in else np.asarray(x, dtype=np.float64)
    Wr = W
    if round_bf16:
        a, Wr = bf16(a), bf16(W)
    out = np.zeros(x.shape[:3] + (W.shape[1],))
    for tap, (dy, dx) in enumerate(TAPS):
        out += _shift(a, dy, dx) @ Wr[tap].T
    return out + b


def conv_bwd(x, W, dout, relu_in=False, round_bf16=False):
    """Gradients of sum(dout * conv_fwd(x, W, b)) with respect to x, W, b.
    The matrix-core operands are dout with x (weight gradient) and dout with
    W (input gradient)."""
    a = np.maximum(x, 0.0) if relu_in else np.asarray(x, dtype=np.float64)
    d, Wr = dout, W
    if round_bf16:
        a, Wr, d = bf16(a), bf16(W), bf16(dout)
    dW = np.zeros_like(W, dtype=np.float64)
    da = np.zeros(x.shape)
    for tap, (dy, dx) in enumerate(TAPS):
        sa = _shift(a, dy, dx)
        dW[tap] = np.einsum("nhwo,nhwi->oi", d, sa)
        da += _shift(d @ Wr[tap], -dy, -dx)
    if relu_in:
        da = da * (x > 0)
    db = dout.sum(axis=(0, 1, 2))
    return da, dW, db


def net_forward(x, params, round_bf16=False):
    """params: list of (W, b); relu between layers, none on the output.
    Returns the list of pre-activations z_l (z_0 = the input)."""
    zs = [x]
    for l, (W, b) in enumerate(params):
        zs.append(conv_fwd(zs[-1], W, b, relu_in=l > 0, round_bf16=round_bf16))
    return zs


def net_backward(zs, params, dout, round_bf16=False):
    grads = [None] * len(params)
    d = dout
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        da, dW, db = conv_bwd(zs[l], W, d, relu_in=l > 0, round_bf16=round_bf16)
        grads[l] = (dW, db)
        d = da
    return grads


def mse(pred, target, creal):
    d = pred[..., :creal] - target[..., :creal]
    n = d.size
    loss = float((d * d).sum() / n)
    g = np.zeros_like(pred)
    g[..., :creal] = 2.0 * d / n
    return loss, g
