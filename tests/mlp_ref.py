"""Plain numpy reference of the learned preconditioner's network (test infrastructure).

Layers 140 -> 128 -> 128 -> 128 (ReLU) -> 128 (linear); parameters packed per layer as W
(in x out, row-major) then b (out).  The device forward pass (matrix cores, FP16 inputs) multiplies
each layer's input rounded to FP16 by FP16-rounded W and adds FP32 b; the reference does the same
arithmetic in float64 so that only the accumulation order differs.  The backward pass takes the
layers' unrounded outputs, as the device's does.
"""
import numpy as np

SIZES = [(140, 128), (128, 128), (128, 128), (128, 128)]


def param_count():
    return sum(i * o + o for i, o in SIZES)


def unpack(w, half=True):
    out, off = [], 0
    for i, o in SIZES:
        W = w[off:off + i * o].reshape(i, o).astype(np.float64)
        if half:
            W = w[off:off + i * o].astype(np.float16).astype(np.float64).reshape(i, o)
        off += i * o
        b = w[off:off + o].astype(np.float64)
        off += o
        out.append((W, b))
    return out


def forward(w, X, half=True):
    acts = [np.asarray(X, np.float64)]
    layers = unpack(w, half)
    for l, (W, b) in enumerate(layers):
        x = acts[-1].astype(np.float16).astype(np.float64) if half else acts[-1]
        z = x @ W + b
        acts.append(np.maximum(z, 0.0) if l < 3 else z)
    return acts


def loss_grad(w, X, T, half=True):
    """Mean over samples of the squared error summed over outputs, and its gradient (packed)."""
    acts = forward(w, X, half)
    M = X.shape[0]
    d = acts[-1] - np.asarray(T, np.float64)
    loss = float(np.sum(d * d) / M)
    dY = 2.0 * d / M
    layers = unpack(w, half)
    grads = [None] * 4
    for l in range(3, -1, -1):
        W, _ = layers[l]
        grads[l] = (acts[l].T @ dY, dY.sum(0))
        if l > 0:
            dY = (dY @ W.T) * (acts[l] > 0)
    g = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return loss, g
