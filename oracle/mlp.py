"""Visibility MLP: forward and hand-written backward, FP64.

Test infrastructure (see the package docstring).

Sec. 3.1: the encoding is fed to an MLP whose output layer has one neuron per
light, each the estimated visibility of that light.  Sec. 3.3: hidden layers
use (leaky) ReLU, the output a sigmoid; the network is trained by
backpropagation (Sec. 3.3, 3.4).  No biases (fully fused MLP style; the
paper is silent).  Weights are given per layer as [out][in] matrices, input
layer first.  The derivative of ReLU at 0 is taken as 0 (leaky: slope).
"""
from __future__ import annotations

import numpy as np


def act(x: np.ndarray, kind: str = "relu", slope: float = 0.01) -> np.ndarray:
    if kind == "relu":
        return np.where(x > 0.0, x, 0.0)
    if kind == "leaky":
        return np.where(x > 0.0, x, slope * x)
    raise ValueError(kind)


def act_grad(pre: np.ndarray, kind: str = "relu", slope: float = 0.01) -> np.ndarray:
    if kind == "relu":
        return (pre > 0.0).astype(np.float64)
    if kind == "leaky":
        return np.where(pre > 0.0, 1.0, slope)
    raise ValueError(kind)


def sigmoid(z: np.ndarray) -> np.ndarray:
    """1/(1+e^-z), evaluated without overflow for either sign of z."""
    z = np.asarray(z, np.float64)
    out = np.empty_like(z)
    pos = z >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-z[pos]))
    ez = np.exp(z[~pos])
    out[~pos] = ez / (1.0 + ez)
    return out


def forward(enc: np.ndarray, weights, kind: str = "relu", slope: float = 0.01):
    """Returns (z, pre, inputs): output logits [n,M], hidden pre-activations, and each layer's input."""
    h = np.asarray(enc, np.float64)
    pre, inputs = [], []
    for W in weights[:-1]:
        inputs.append(h)
        a = h @ np.asarray(W, np.float64).T
        pre.append(a)
        h = act(a, kind, slope)
    inputs.append(h)
    z = h @ np.asarray(weights[-1], np.float64).T
    return z, pre, inputs


def visibility(enc: np.ndarray, weights, kind: str = "relu", slope: float = 0.01) -> np.ndarray:
    """Predicted visibility sigma(z) in (0,1), one column per light."""
    return sigmoid(forward(enc, weights, kind, slope)[0])


def backward(weights, pre, inputs, dz: np.ndarray, kind: str = "relu", slope: float = 0.01):
    """Gradients given dL/dz.  Returns (dW list [out][in], dL/d(encoding) [n, n_in]).

    dW_k = delta_k^T h_{k-1};  delta_{k-1} = (delta_k W_k) * act'(pre_{k-1}).
    """
    n_layers = len(weights)
    dW = [None] * n_layers
    delta = np.asarray(dz, np.float64)
    d_enc = None
    for k in range(n_layers - 1, -1, -1):
        Wk = np.asarray(weights[k], np.float64)
        dW[k] = delta.T @ inputs[k]
        d_in = delta @ Wk
        if k > 0:
            delta = d_in * act_grad(pre[k - 1], kind, slope)
        else:
            d_enc = d_in
    return dW, d_enc
