"""Binary64 reference of the learned selector's network (test infrastructure only).

COMPAR delegates the choice of variant to the runtime's performance models,
which are trained from measured executions (Sec. 3.2 on the matrix-multiply
results, and the call for better-trained models in Sec. 5).  The learned
selector here is a small regression network from the call context to the
logarithm of each variant's run time:

    inputs  x = (log2 M, log2 N, log2 K, log10 tol), standardised with the
              training set's per-feature mean and population standard deviation
              (a zero deviation is replaced by 1)
    layers  4 -> 64 (ReLU) -> 64 (ReLU) -> 4, affine layers z = W h + b
    outputs standardised ln(median microseconds) per variant; the targets are
            standardised per output column the same way as the inputs
    loss    mean squared error over all n x 4 outputs
    update  Adam (Kingma & Ba, 2015) with bias correction, full batch

Parameters are packed layer by layer as [W (out x in, row-major), b (out)].
The ReLU derivative at exactly zero is taken as 0.
"""
from __future__ import annotations

import numpy as np

SIZES = (4, 64, 64, 4)


def unpack(params, sizes=SIZES):
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for i in range(len(sizes) - 1):
        fi, fo = sizes[i], sizes[i + 1]
        W = p[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = p[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == p.size, (off, p.size)
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def standardize_stats(X):
    """Per-column mean and population standard deviation (0 replaced by 1)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return mu, sd


def features(M, N, K, tol):
    """Raw selector features for arrays of shapes and tolerances."""
    M, N, K, tol = (np.asarray(v, dtype=np.float64) for v in (M, N, K, tol))
    return np.stack([np.log2(M), np.log2(N), np.log2(K), np.log10(tol)], axis=1)


def forward(params, X, sizes=SIZES):
    """Network output for standardised inputs X (n x 4); also returns the activations."""
    layers = unpack(params, sizes)
    h = np.asarray(X, dtype=np.float64)
    acts = [h]
    zs = []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = np.maximum(z, 0.0) if li < len(layers) - 1 else z
        acts.append(h)
    return h, (acts, zs)


def loss_and_grad(params, X, Y, sizes=SIZES):
    """MSE loss over all outputs and its gradient with respect to the packed parameters."""
    Y = np.asarray(Y, dtype=np.float64)
    yhat, (acts, zs) = forward(params, X, sizes)
    n_out = Y.size
    diff = yhat - Y
    loss = float(np.sum(diff * diff) / n_out)
    layers = unpack(params, sizes)
    grads = [None] * len(layers)
    delta = 2.0 * diff / n_out                      # dL/dz of the last layer
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = acts[li]
        grads[li] = (delta.T @ h_in, delta.sum(axis=0))
        if li > 0:
            dh = delta @ W
            delta = dh * (zs[li - 1] > 0.0)
    return loss, pack(grads)


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(params0, X, Y, steps, lr, b1=0.9, b2=0.999, eps=1e-8, sizes=SIZES, record=None):
    """Full-batch Adam from params0 on standardised (X, Y); returns (params, losses).

    ``losses[t]`` is the loss evaluated before update t+1.  ``record`` is an
    optional set of step counts at which to keep a copy of the parameters.
    """
    p = np.asarray(params0, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses, kept = [], {}
    for t in range(1, steps + 1):
        loss, g = loss_and_grad(p, X, Y, sizes)
        losses.append(loss)
        p, m, v = adam_step(p, g, m, v, t, lr, b1, b2, eps)
        if record is not None and t in record:
            kept[t] = p.copy()
    if record is not None:
        return p, np.asarray(losses), kept
    return p, np.asarray(losses)


def predict_log_us(params, mu_x, sd_x, mu_y, sd_y, Xraw, sizes=SIZES):
    """Predicted ln(microseconds) per variant for raw features."""
    Xs = (np.asarray(Xraw, dtype=np.float64) - mu_x) / sd_x
    y, _ = forward(params, Xs, sizes)
    return y * sd_y + mu_y
