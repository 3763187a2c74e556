"""Light weights, visibility clamp, weighted reservoir sampling and neural DI.

Test infrastructure (see the package docstring).

* Sec. 1 / Sec. 3.1: a light is picked with probability proportional to its
  weight, the unshadowed contribution times the visibility predicted by the
  cache, using weighted reservoir sampling (Chao 1982; Wyman 2021).
* Sec. 3.1 and Fig. "bias": predicted visibility is clamped from below by a
  small positive constant (0.001) so every light with non-zero unshadowed
  contribution keeps a non-zero probability (unbiasedness).
* Sec. 3.1 approximates BRDF x cosine with LTC; these synthetic scenes use
  Lambertian point lights instead: f_i = I_i * max(0, n . w_i) / d_i^2
  (no normal: f_i = I_i / d_i^2).  The squared distance is floored at 1e-6.
* Sec. 3.2: neural direct illumination uses the predicted visibility directly:
  sum_i v_i f_i * rho/pi with rho = 1 (raw, unclamped visibility).

Weighted reservoir sampling with a single uniform u per pixel is taken as its
equal-in-distribution inverse-CDF form over the lights in index order: with
C_i the running sum of weights and W = C_{M-1}, the pick is the first i with
C_i > u*W.  That pick is an integer decided by floating point, so
`wrs_pick` runs in the caller's dtype (FP32 for parity with the kernels)
with this exact operation order:

    d   = l - p                       (componentwise)
    d2  = max((dx*dx + dy*dy) + dz*dz, 1e-6)
    nd  = (nx*dx + ny*dy) + nz*dz     (with normals)
    f   = (I * max(nd, 0)) / (d2 * sqrt(d2))   or   I / d2 without normals
          (n . w / d^2 with w = d / |d|, i.e. I * cos / d^2)
    w   = f * max(v, floor)
    C_i = C_{i-1} + w_i  (sequential, light order);  t = u * W
"""
from __future__ import annotations

import math

import numpy as np

VIS_FLOOR = 1e-3


def unshadowed_weight(pos, nrm, lights, dtype=np.float64) -> np.ndarray:
    """f [n,M] for positions [n,3] (scene units), normals [n,3] or None, lights [M,4]."""
    dt = np.dtype(dtype).type
    p = np.asarray(pos).astype(dtype)
    L = np.asarray(lights).astype(dtype)
    dx = L[None, :, 0] - p[:, None, 0]
    dy = L[None, :, 1] - p[:, None, 1]
    dz = L[None, :, 2] - p[:, None, 2]
    d2 = np.fmax((dx * dx + dy * dy) + dz * dz, dt(1e-6))
    inten = L[None, :, 3]
    if nrm is None:
        return inten / d2
    n = np.asarray(nrm).astype(dtype)
    nd = (n[:, None, 0] * dx + n[:, None, 1] * dy) + n[:, None, 2] * dz
    return (inten * np.fmax(nd, dt(0.0))) / (d2 * np.sqrt(d2))


def clamp_visibility(vis, floor: float = VIS_FLOOR, dtype=np.float64) -> np.ndarray:
    """v_hat = max(v, floor) (NaN -> floor); floor = 0 gives the biased variant."""
    return np.fmax(np.asarray(vis).astype(dtype), np.dtype(dtype).type(floor))


def light_weights(pos, nrm, lights, vis, floor: float = VIS_FLOOR, dtype=np.float64) -> np.ndarray:
    """w = f * max(v, floor) [n,M]."""
    return unshadowed_weight(pos, nrm, lights, dtype) * clamp_visibility(vis, floor, dtype)


def wrs_pick(w: np.ndarray, u: np.ndarray):
    """Inverse-CDF pick in light order in w's dtype.

    Returns (idx int32 [n], pmf [n], wsum [n]); idx = -1 and pmf = 0 where W = 0.
    If no running sum exceeds u*W (only through rounding), the last light with
    positive weight is taken.
    """
    w = np.asarray(w)
    dt = w.dtype.type
    C = np.cumsum(w, axis=1, dtype=w.dtype)          # sequential accumulation
    W = C[:, -1]
    t = np.asarray(u).astype(w.dtype) * W
    above = C > t[:, None]
    has = above.any(axis=1)
    idx = np.where(has, above.argmax(axis=1), -1)
    pos_w = w > 0
    last_pos = np.where(pos_w.any(axis=1), w.shape[1] - 1 - pos_w[:, ::-1].argmax(axis=1), -1)
    idx = np.where(has, idx, last_pos)
    idx = np.where(W > 0, idx, -1).astype(np.int32)
    safe = np.where(idx >= 0, idx, 0)
    w_sel = np.take_along_axis(w, safe[:, None], axis=1)[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        pmf = np.where(idx >= 0, w_sel / np.where(W > 0, W, dt(1)), dt(0)).astype(w.dtype)
    return idx, pmf, W


def pick_reservoir(w, f, idx, W):
    """The pick as a one-candidate reservoir for the target f (Sec. 4.2: the cache's pick can seed ReSTIR):
    y = idx, M = 1, contribution weight W_r = W / w_idx (= 1 / pmf), w_sum = f_idx * W_r, in w's dtype;
    (-1, 0, 0, 0) without a pick."""
    w = np.asarray(w)
    dt = w.dtype.type
    safe = np.where(idx >= 0, idx, 0)
    wsel = np.take_along_axis(w, safe[:, None], axis=1)[:, 0]
    fsel = np.take_along_axis(np.asarray(f).astype(w.dtype), safe[:, None], axis=1)[:, 0]
    ok = idx >= 0
    with np.errstate(invalid="ignore", divide="ignore"):
        Wr = np.where(ok, np.asarray(W).astype(w.dtype) / np.where(ok, wsel, dt(1)), dt(0)).astype(w.dtype)
    return {"y": np.where(ok, idx, -1), "M": ok.astype(np.int32), "w_sum": np.where(ok, fsel * Wr, dt(0)),
            "W": Wr}


def selection_pmf(w: np.ndarray) -> np.ndarray:
    """Full selection distribution p_i = w_i / sum_j w_j (FP64), zero rows stay zero."""
    w = np.asarray(w, np.float64)
    W = w.sum(axis=1, keepdims=True)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(W > 0, w / np.where(W > 0, W, 1.0), 0.0)


def neural_di(vis, f) -> np.ndarray:
    """sum_i v_i f_i / pi (albedo 1), FP64."""
    return (np.asarray(vis, np.float64) * np.asarray(f, np.float64)).sum(axis=1) / math.pi
