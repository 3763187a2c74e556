"""Element-wise error bounds of a computed visibility and training gradient.

Test infrastructure (see the package docstring).

The kernels evaluate the cache's forward pass (Sec. 3.1, 3.3) and its
backpropagation (Sec. 3.3, 3.4) in floating point: weights, encodings,
hidden activations and back-propagated deltas are rounded to the
matrix-core format (unit roundoff u_io: 2^-24 FP32, 2^-11 FP16, 2^-8 BF16)
and every dot product is accumulated in FP32 (unit roundoff u = 2^-24).
This module bounds |computed - exact| for every visibility and every
gradient entry by a running error analysis: the standard dot-product bound
|fl(x.y) - x.y| <= gamma_n |x|.|y| (Higham, Accuracy and Stability of
Numerical Algorithms, 2nd ed., eq. 3.5) applied layer by layer, with the
errors already present in each operand carried forward as absolute bounds
E, next to the magnitudes A = |exact| + E of the computed operands:

  forward   E(W h)  <= |W| E(h) + c(n) |W| A(h),    c(n) = u_io + 2u (n + 1)
            (u_io: the weights' rounding; n + 1 rounded products and sums,
            each counted as 2u so that truncating accumulators are covered)
  ReLU      1-Lipschitz, so E passes through; leaky ReLU likewise
            (slope <= 1); the stored activation adds u_io A
  sigmoid   |sigma'| <= 1/4, |sigma''| <= 0.0963
  backward  E(W^T d) <= |W|^T E(d) + c(n) |W|^T A(d); the mask of a hidden
            neuron is taken from the computed pre-activation, which may have
            the other sign when |pre| <= E(pre) (+ the format's smallest
            subnormal, where rounding flushes to zero): there the error is
            the whole |d| (1 - slope), not a rounding
  sums      a gradient entry sums batch terms through a tree of at most
            `depth` additions per term, adding 2u depth sum|terms|

Second-order products of errors are kept (E_a A_b + |a| E_b >= |ab - a~b~|
with A = |a| + E), so the bounds are rigorous, not first-order estimates.
The table gradient's fixed-point partition sums round each record to
2^-45 of the largest record (at most), counted per entry.
"""
from __future__ import annotations

import numpy as np

from . import hashgrid, mlp

U32 = 2.0 ** -24
UNIT_ROUNDOFF = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
# Largest value rounding flushes to zero: half the smallest subnormal (FP16 2^-24, BF16 and FP32 below 1e-38).
FLUSH = {"f32": 2.0 ** -150, "f16": 2.0 ** -25, "bf16": 2.0 ** -134}
SIGMOID_REL = 8 * U32          # hardware exp2 and reciprocal: a few units of u relative
D2_SIGMOID_MAX = 0.0963        # max |sigma''| = 1/(6 sqrt(3))
FIXED_RES = 2.0 ** -45         # fixed-point partition sums: resolution relative to the largest record


def weight_sum_depth(batch: int, min_blocks: int = 256) -> int:
    """Additions a batch term of a weight-gradient entry can pass through in the kernels: a block sums
    64 samples per iteration into a matrix-core accumulator (taken as 64 sequential additions, whatever the
    hardware's internal order), over ceil(batch / (64 G)) iterations with G >= min_blocks resident blocks;
    then at most 64 blocks per slice and 64 slices."""
    iters = -(-batch // (64 * min_blocks))
    return 64 * max(iters, 1) + 128


def _c(n: int, u_io: float) -> float:
    return u_io + 2.0 * U32 * (n + 1)


def _forward(pos32, table, weights, base_res, growth, act, slope, u_io):
    """Exact forward (FP64) with error bounds of the computed values."""
    enc, corners = hashgrid.encode(pos32, table, base_res, growth, return_corners=True)
    L, T, F = table.shape
    # sum over the 8 corners of |w| |theta|: the encoding's own magnitude
    s_e = np.zeros_like(enc)
    for l, (idx, w) in enumerate(corners):
        vals = np.abs(table[l].astype(np.float64))[idx]                     # [n,8,F]
        s_e[:, l * F:(l + 1) * F] = np.einsum("nk,nkf->nf", np.abs(w), vals)
    # trilinear weight: three FP32 factors (1 - f may round) and two products (5u); eight products and
    # seven sums (15u); then rounding to the matrix-core format
    e_enc = 2.0 * 20 * U32 * s_e
    e_enc = e_enc + u_io * (np.abs(enc) + e_enc)
    h, e_h = enc, e_enc
    layers = []
    n_layers = len(weights)
    for k, W in enumerate(weights):
        W = np.asarray(W, np.float64)
        aW = np.abs(W)
        a_h = np.abs(h) + e_h
        pre = h @ W.T
        e_pre = e_h @ aW.T + _c(W.shape[1], u_io) * (a_h @ aW.T)
        layers.append({"h": h, "e_h": e_h, "pre": pre, "e_pre": e_pre})
        if k < n_layers - 1:
            h = mlp.act(pre, act, slope)
            e_h = e_pre + u_io * (np.abs(h) + e_pre)
    return enc, corners, layers


def visibility_error_bound(pos32, table, weights, base_res, growth, act="relu", slope=0.01, dtype="f32",
                           out_dtype=None):
    """Exact visibility v (FP64) and a bound on |v_computed - v| per entry for the given format."""
    u_io = UNIT_ROUNDOFF[dtype]
    _, _, layers = _forward(pos32, table, weights, base_res, growth, act, slope, u_io)
    z, e_z = layers[-1]["pre"], layers[-1]["e_pre"]
    v = mlp.sigmoid(z)
    e_v = 0.25 * e_z + SIGMOID_REL * (v + 0.25 * e_z)
    u_out = UNIT_ROUNDOFF[out_dtype or dtype]
    e_v = e_v + u_out * (v + e_v)
    return v, e_v


def gradient_error_bounds(pos32, table, weights, base_res, growth, labels=None, dvis=None, loss="bce",
                          act="relu", slope=0.01, dtype="f32", depth_w: int | None = None):
    """Exact gradients (FP64) and element-wise bounds on |computed - exact| for the given format.

    depth_w bounds how many additions a batch term of a weight-gradient entry passes through (the
    kernel's tree of matrix-core sums, persistent iterations and partial reductions).  Table entries
    are bounded for any order of their terms.  Returns dict(g_w, e_w (lists [out][in]), g_table,
    e_table ([L,T,F]), scale)."""
    u_io = UNIT_ROUNDOFF[dtype]
    eta = FLUSH[dtype]
    if depth_w is None:
        depth_w = weight_sum_depth(pos32.shape[0])
    slope_v = slope if act == "leaky" else 0.0
    enc, corners, layers = _forward(pos32, table, weights, base_res, growth, act, slope, u_io)
    n = pos32.shape[0]
    z, e_z = layers[-1]["pre"], layers[-1]["e_pre"]
    s = mlp.sigmoid(z)
    # output gradient, per sample and light, before the 1/(B M) of the mean
    if dvis is not None:
        d = np.asarray(dvis, np.float64)
        dz = d * s * (1.0 - s)
        e_dz = np.abs(d) * (D2_SIGMOID_MAX * e_z + 4 * SIGMOID_REL + 4 * U32)
        scale = 1.0
    else:
        y = np.asarray(labels, np.float64)
        if loss == "bce":
            dz = s - y
            e_dz = 0.25 * e_z + 2 * SIGMOID_REL
        elif loss == "l2":
            dz = 2.0 * (s - y) * s * (1.0 - s)
            # |d/dz 2 (s - y) s (1 - s)| <= 2 (1/16 + 0.0963) < 0.32; rounding of four operations
            e_dz = 0.32 * e_z + 2 * (4 * SIGMOID_REL + 4 * U32)
        else:
            raise ValueError(loss)
        scale = 1.0 / dz.size
    e_dz = e_dz + u_io * (np.abs(dz) + e_dz)
    delta, e_delta = dz, e_dz
    n_layers = len(weights)
    g_w, e_w = [None] * n_layers, [None] * n_layers
    for k in range(n_layers - 1, -1, -1):
        W = np.asarray(weights[k], np.float64)
        aW = np.abs(W)
        h, e_h = layers[k]["h"], layers[k]["e_h"]
        a_h = np.abs(h) + e_h
        a_d = np.abs(delta) + e_delta
        g = delta.T @ h
        e = e_delta.T @ a_h + np.abs(delta).T @ e_h + 2.0 * U32 * depth_w * (a_d.T @ a_h)
        g_w[k] = g * scale
        e_w[k] = (e + 4 * U32 * np.abs(g)) * scale
        dprev = delta @ W
        e_dprev = e_delta @ aW + _c(W.shape[0], u_io) * (a_d @ aW)
        if k > 0:
            pre, e_pre = layers[k - 1]["pre"], layers[k - 1]["e_pre"]
            ag = mlp.act_grad(pre, act, slope)
            amb = np.abs(pre) <= e_pre + eta
            delta = dprev * ag
            e_delta = np.where(amb, e_dprev + (1.0 - slope_v) * (np.abs(dprev) + e_dprev), e_dprev * ag)
            e_delta = e_delta + u_io * (np.abs(delta) + e_delta)
        else:
            d_enc, e_denc = dprev, e_dprev
    # table gradient: terms w * d_enc per corner; any order of additions; fixed-point resolution
    L, T, F = table.shape
    a_denc = np.abs(d_enc) + e_denc
    g_t = np.zeros((L, T, F))
    e_t = np.zeros((L, T, F))
    mag = np.zeros((L, T, F))
    cnt = np.zeros((L, T), np.float64)
    for l, (idx, w) in enumerate(corners):
        sl = slice(l * F, (l + 1) * F)
        aw = np.abs(w)[:, :, None]
        flat = idx.reshape(-1)
        np.add.at(g_t[l], flat, (w[:, :, None] * d_enc[:, None, sl]).reshape(-1, F))
        np.add.at(e_t[l], flat, (aw * e_denc[:, None, sl] + 12 * U32 * aw * a_denc[:, None, sl]).reshape(-1, F))
        np.add.at(mag[l], flat, (aw * a_denc[:, None, sl]).reshape(-1, F))
        np.add.at(cnt[l], flat, 1.0)
    m_glob = float(mag.max()) if mag.size else 0.0
    e_t = e_t + 2.0 * U32 * (cnt[:, :, None] + 4.0) * mag + cnt[:, :, None] * FIXED_RES * m_glob
    e_t = (e_t + 4 * U32 * np.abs(g_t)) * scale
    return {"g_w": g_w, "e_w": e_w, "g_table": g_t * scale, "e_table": e_t, "scale": scale}
