"""CPU pins of the numpy network reference used to check the device MLP kernels."""
import numpy as np

from mlp_ref import SIZES, forward, loss_grad, param_count


def _setup(seed=0, m=9):
    rng = np.random.default_rng(seed)
    w = np.concatenate([np.concatenate([rng.standard_normal(i * o) * np.sqrt(2.0 / i), rng.standard_normal(o) * 0.1])
                        for i, o in SIZES])
    X = rng.standard_normal((m, 140))
    T = rng.standard_normal((m, 128))
    return w, X, T


def test_param_count():
    assert param_count() == 140 * 128 + 3 * 128 * 128 + 4 * 128


def test_backprop_matches_central_differences():
    """Explicit backprop of the reference against central differences (float64, full-precision
    weights) on a sample of weights and biases of every layer."""
    w, X, T = _setup()
    _, g = loss_grad(w, X, T, half=False)
    rng = np.random.default_rng(3)
    h = 1e-6
    for idx in rng.choice(w.size, 60, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        fd = (loss_grad(wp, X, T, half=False)[0] - loss_grad(wm, X, T, half=False)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), (idx, fd, g[idx])


def test_relu_and_linear_structure():
    """Hidden activations are non-negative, the output layer is affine in the last hidden layer."""
    w, X, _ = _setup(m=4)
    acts = forward(w, X, half=False)
    for a in acts[1:4]:
        assert np.all(a >= 0)
    off = sum(i * o + o for i, o in SIZES[:3])
    W = w[off:off + 128 * 128].reshape(128, 128)
    b = w[off + 128 * 128:]
    assert np.allclose(acts[4], acts[3] @ W + b)
