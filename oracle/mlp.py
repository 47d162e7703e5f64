"""FP64 reference for the surrogate network's training (test infrastructure only).

Network: u (3) -> [W_l, b_l, SiLU] x layers (width `hidden`) -> W_out, b_out -> y (2);
parameters packed layer by layer as W [n_in][n_out] (input-major) then b [n_out], the
same layout the C oracle and the library use.  Loss: L = (1/B) sum_b sum_o (y_bo - t_bo)^2.
Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
import numpy as np


def shapes(hidden=128, layers=4):
    dims = [3] + [hidden] * layers + [2]
    return [(dims[i], dims[i + 1]) for i in range(len(dims) - 1)]


def unpack(params, hidden=128, layers=4):
    out, o = [], 0
    for n_in, n_out in shapes(hidden, layers):
        W = params[o:o + n_in * n_out].reshape(n_in, n_out)
        o += n_in * n_out
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == params.size
    return out


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, U, hidden=128, layers=4):
    """Y [B, 2] and the cache of pre-activations and layer inputs."""
    h = np.asarray(U, dtype=np.float64)
    cache = []
    lw = unpack(np.asarray(params, dtype=np.float64), hidden, layers)
    for li, (W, b) in enumerate(lw):
        z = h @ W + b
        cache.append((h, z))
        h = z if li == len(lw) - 1 else z * _sig(z)
    return h, cache


def backward(params, cache, dY, hidden=128, layers=4):
    """Gradient of sum(dY * Y) with respect to the packed parameters."""
    lw = unpack(np.asarray(params, dtype=np.float64), hidden, layers)
    grads = [None] * len(lw)
    g = dY
    for li in range(len(lw) - 1, -1, -1):
        h_in, z = cache[li]
        if li != len(lw) - 1:
            s = _sig(z)
            g = g * (s * (1.0 + z * (1.0 - s)))          # SiLU'
        W, _ = lw[li]
        grads[li] = (h_in.T @ g, g.sum(axis=0))
        g = g @ W.T
    return np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])


def loss_and_grad(params, U, Tgt, hidden=128, layers=4):
    Y, cache = forward(params, U, hidden, layers)
    B = U.shape[0]
    r = Y - Tgt
    loss = float(np.sum(r * r) / B)
    return loss, backward(params, cache, 2.0 * r / B, hidden, layers)


def adam_step(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
