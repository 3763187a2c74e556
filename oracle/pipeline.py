"""One frame of the cache, composed from the oracle's steps (Sec. 3.1, Fig. "overview"; Sec. 3.4).

Test infrastructure (see the package docstring).

Inference: encode -> MLP -> visibility.  Sampling: light weights with the
clamped visibility, one WRS pick per pixel, neural DI.  Training: pick
pixels, label them with shadow rays, compute gradients, one Adam step.
"""
from __future__ import annotations

import numpy as np

from . import hashgrid, lighting, mlp, philox, shadow, training


def infer(pos_unit, table, weights, base_res, growth, act="relu", slope=0.01) -> np.ndarray:
    """Visibility [n,M] (FP64) of FP32 unit-cube positions."""
    enc = hashgrid.encode(pos_unit, table, base_res, growth)
    return mlp.visibility(enc, weights, act, slope)


def sample(vis, pos, nrm, lights, seed: int, frame: int, floor: float = lighting.VIS_FLOOR,
           first: int = 0):
    """WRS pick per pixel.  The pick is decided in FP32 from fl32(vis); pmf and W come from that
    FP32 pass, and `pmf64` / `di` are the FP64 values of the same quantities.
    """
    vis = np.asarray(vis)
    u = philox.wrs_uniforms(seed, frame, vis.shape[0], first)
    w32 = lighting.light_weights(pos, nrm, lights, vis.astype(np.float32), floor, np.float32)
    idx, pmf, W = lighting.wrs_pick(w32, u)
    f64 = lighting.unshadowed_weight(pos, nrm, lights, np.float64)
    w64 = f64 * lighting.clamp_visibility(vis, floor, np.float64)
    p64 = lighting.selection_pmf(w64)
    safe = np.where(idx >= 0, idx, 0)
    pmf64 = np.where(idx >= 0, np.take_along_axis(p64, safe[:, None].astype(np.int64), axis=1)[:, 0], 0.0)
    di = lighting.neural_di(vis, f64)
    return {"idx": idx, "pmf": pmf, "wsum": W, "u": u, "pmf64": pmf64, "wsum64": w64.sum(axis=1),
            "di": di, "w64": w64}


def train_step(pos_unit_pix, pos_pix, lights, spheres, table, weights, base_res, growth,
               seed: int, frame: int, batch: int, adam_state=None, lr=1e-2, beta1=0.9, beta2=0.99,
               eps=1e-8, loss="bce", act="relu", slope=0.01):
    """Pixel selection, shadow labels, gradients and one Adam step over all parameters."""
    n_pix = pos_unit_pix.shape[0]
    pix = philox.training_pixels(seed, frame, batch, n_pix)
    y = shadow.labels_fp32(pos_pix[pix], lights, spheres)
    grads = training.train_gradients(pos_unit_pix[pix], table, weights, base_res, growth,
                                     labels=y, loss=loss, act=act, slope=slope)
    params = [np.asarray(table, np.float64)] + [np.asarray(w, np.float64) for w in weights]
    gs = [grads["g_table"]] + grads["g_w"]
    if adam_state is None:
        adam_state = {"t": 0, "m": [np.zeros_like(p) for p in params], "v": [np.zeros_like(p) for p in params]}
    t = adam_state["t"] + 1
    new_p, new_m, new_v = [], [], []
    for p, g, m, v in zip(params, gs, adam_state["m"], adam_state["v"]):
        a, b, c = training.adam_step(p, g, m, v, t, lr, beta1, beta2, eps)
        new_p.append(a)
        new_m.append(b)
        new_v.append(c)
    return {"pix": pix, "labels": y, "loss": grads["loss"], "grads": grads,
            "table": new_p[0], "weights": new_p[1:], "adam": {"t": t, "m": new_m, "v": new_v}}
