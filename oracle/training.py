"""Online training step: loss, gradients through MLP and hash grid, Adam.

Test infrastructure (see the package docstring).

Sec. 3.4: one Adam step per frame on a batch of (position -> visibility of
every light) examples.  Sec. 3.3: the paper trains with the L2 loss; the
1080p training workload uses binary cross-entropy on the logits.  Both are
the mean over the B*M (sample, light) pairs (normalisation unstated in the
paper).  The loss is taken on the raw sigmoid output, not the clamped one.

Gradient of the hash table (backpropagation into the encoding): each corner
receives its trilinear weight times the gradient of the feature it feeds;
corners of one point that share a table entry add up.

Adam (Kingma & Ba 2015) with bias correction, step t counted from 1, every
parameter updated each step (dense), no weight decay:
    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
    theta <- theta - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Learning rate (Sec. 3.4): the paper starts at 0.05 and lowers the rate
linearly over the first 200 steps to 0.001.  Reading: with f = min(t - 1,
D) / D, lr_t = (1 - f) lr0 + f lr1, i.e. lr0 at step 1 and lr1 from step
D + 1 on.
"""
from __future__ import annotations

import numpy as np

from . import hashgrid, mlp


def bce_loss(z: np.ndarray, y: np.ndarray):
    """Mean of softplus(z) - y z over all entries, and dL/dz."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    n = z.size
    loss = float(np.mean(np.logaddexp(0.0, z) - y * z))
    dz = (mlp.sigmoid(z) - y) / n
    return loss, dz


def l2_loss(z: np.ndarray, y: np.ndarray):
    """Mean of (sigmoid(z) - y)^2 over all entries, and dL/dz."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    v = mlp.sigmoid(z)
    n = z.size
    loss = float(np.mean((v - y) ** 2))
    dz = 2.0 * (v - y) * v * (1.0 - v) / n
    return loss, dz


def upstream_dz(z: np.ndarray, dvis: np.ndarray) -> np.ndarray:
    """dL/dz for a given dL/dv (chain rule through the sigmoid)."""
    v = mlp.sigmoid(np.asarray(z, np.float64))
    return np.asarray(dvis, np.float64) * v * (1.0 - v)


def table_gradient(d_enc: np.ndarray, corner_cache, shape) -> np.ndarray:
    """Scatter dL/d(encoding) [n, L*F] to the table shape [L,T,F] (FP64)."""
    L, T, F = shape
    g = np.zeros((L, T, F), np.float64)
    for l, (idx, w) in enumerate(corner_cache):
        contrib = w[:, :, None] * d_enc[:, None, l * F:(l + 1) * F]    # [n,8,F]
        np.add.at(g[l], idx.reshape(-1), contrib.reshape(-1, F))
    return g


def train_gradients(pos32, table, weights, base_res, growth, labels=None, dvis=None,
                    loss: str = "bce", act: str = "relu", slope: float = 0.01):
    """Loss and gradients of one training batch.

    Returns dict(loss, z, g_table [L,T,F], g_w list [out][in], d_enc).
    """
    enc, cache = hashgrid.encode(pos32, table, base_res, growth, return_corners=True)
    z, pre, inputs = mlp.forward(enc, weights, act, slope)
    if dvis is not None:
        lval, dz = None, upstream_dz(z, dvis)
    elif loss == "bce":
        lval, dz = bce_loss(z, labels)
    elif loss == "l2":
        lval, dz = l2_loss(z, labels)
    else:
        raise ValueError(loss)
    g_w, d_enc = mlp.backward(weights, pre, inputs, dz, act, slope)
    g_table = table_gradient(d_enc, cache, table.shape)
    return {"loss": lval, "z": z, "g_table": g_table, "g_w": g_w, "d_enc": d_enc}


def learning_rate(t: int, lr0: float, lr1: float | None = None, decay_steps: int = 0) -> float:
    """Rate of step t >= 1 (FP64): lr0, or the linear decay to lr1 over decay_steps steps (Sec. 3.4)."""
    if decay_steps <= 0 or lr1 is None:
        return float(lr0)
    f = min(t - 1, decay_steps) / decay_steps
    return (1.0 - f) * float(lr0) + f * float(lr1)


def adam_step(p, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.99, eps: float = 1e-8):
    """One Adam update (FP64).  Returns new (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
