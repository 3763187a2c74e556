"""Shadow-ray training labels against sphere occluders.

Test infrastructure (see the package docstring).

Sec. 3.4: each training example pairs a position with the visibility of every
light, obtained by casting one shadow ray from the position to each light;
with point lights the label is binary.  The paper traces its scenes with
hardware ray tracing; these synthetic scenes have sphere occluders only
(invisible to the camera), so a ray p -> l is occluded iff some sphere
(c, r) comes closer than r to the segment:

    t* = clamp(((c - p) . d) / (d . d), 0, 1),  d = l - p
    occluded  <=>  |p + t* d - c|^2 < r^2

A point or light inside a sphere is occluded; tangency counts as visible.
Label 1 = visible, 0 = occluded.

`labels` evaluates that definition in FP64.  The label is a bit decided by
floating point, so `labels_fp32` takes the decision in FP32 the way the
kernel does, from terms shared per (point, sphere):

    o  = c - p;   oo = (ox*ox + oy*oy) + oz*oz;   cc = oo - rr   (rr = fl32(r*r))
    d  = l - p;   dd = (dx*dx + dy*dy) + dz*dz
    b  = (ox*dx + oy*dy) + oz*dz
    b <= 0   : occluded iff cc < 0                      (closest point is p)
    b >= dd  : occluded iff ((ex*ex + ey*ey) + ez*ez) < rr,  e = c - l   (closest is l)
    else     : occluded iff cc*dd < b*b                 (|o|^2 - b^2/dd < r^2, times dd)
"""
from __future__ import annotations

import numpy as np


def labels(pos, lights, spheres, chunk: int = 4096) -> np.ndarray:
    """uint8 [n,M]: 1 if the segment pos->light misses every sphere (FP64 definition)."""
    p_all = np.asarray(pos, np.float64)
    L = np.asarray(lights, np.float64)[:, :3]
    c = np.asarray(spheres, np.float64)[:, :3]
    r2 = np.asarray(spheres, np.float64)[:, 3] ** 2
    out = np.empty((p_all.shape[0], L.shape[0]), np.uint8)
    for s in range(0, p_all.shape[0], chunk):
        p = p_all[s:s + chunk]
        d = L[None, :, :] - p[:, None, :]                          # [n,M,3]
        dd = np.einsum("nmk,nmk->nm", d, d)
        o = c[None, :, :] - p[:, None, :]                          # [n,S,3]
        b = np.einsum("nsk,nmk->nms", o, d)                        # [n,M,S]
        with np.errstate(invalid="ignore", divide="ignore"):
            t = np.clip(np.where(dd[..., None] > 0, b / dd[..., None], 0.0), 0.0, 1.0)
        q = p[:, None, None, :] + t[..., None] * d[:, :, None, :] - c[None, None, :, :]
        dist2 = np.einsum("nmsk,nmsk->nms", q, q)
        out[s:s + chunk] = (~(dist2 < r2[None, None, :]).any(axis=2)).astype(np.uint8)
    return out


def labels_fp32(pos, lights, spheres, chunk: int = 2048) -> np.ndarray:
    """uint8 [n,M], the same test decided in FP32 with the operation order in the module docstring."""
    f32 = np.float32
    p_all = np.asarray(pos, f32)
    L = np.asarray(lights, f32)
    S = np.asarray(spheres, f32)
    cx, cy, cz, r = S[:, 0], S[:, 1], S[:, 2], S[:, 3]
    rr = r * r
    ex = cx[None, :] - L[:, 0:1]
    ey = cy[None, :] - L[:, 1:2]
    ez = cz[None, :] - L[:, 2:3]
    light_inside = ((ex * ex + ey * ey) + ez * ez) < rr[None, :]   # [M,S]
    out = np.empty((p_all.shape[0], L.shape[0]), np.uint8)
    for s in range(0, p_all.shape[0], chunk):
        p = p_all[s:s + chunk]
        px, py, pz = p[:, 0:1], p[:, 1:2], p[:, 2:3]
        ox = cx[None, :] - px                                      # [n,S]
        oy = cy[None, :] - py
        oz = cz[None, :] - pz
        cc = ((ox * ox + oy * oy) + oz * oz) - rr[None, :]
        dx = L[None, :, 0] - px                                    # [n,M]
        dy = L[None, :, 1] - py
        dz = L[None, :, 2] - pz
        dd = (dx * dx + dy * dy) + dz * dz
        b = (ox[:, None, :] * dx[:, :, None] + oy[:, None, :] * dy[:, :, None]) + oz[:, None, :] * dz[:, :, None]
        ccb = cc[:, None, :]
        ddb = dd[:, :, None]
        mid = (ccb * ddb) < (b * b)
        occ = np.where(b <= f32(0), ccb < f32(0),
                       np.where(b >= ddb, light_inside[None, :, :], mid))
        out[s:s + chunk] = (~occ.any(axis=2)).astype(np.uint8)
    return out


def tangency_margin(pos, lights, spheres) -> np.ndarray:
    """min over spheres of |dist^2 - r^2| / r^2 (FP64), the distance of each label from flipping."""
    p = np.asarray(pos, np.float64)
    L = np.asarray(lights, np.float64)[:, :3]
    c = np.asarray(spheres, np.float64)[:, :3]
    r2 = np.asarray(spheres, np.float64)[:, 3] ** 2
    d = L[None, :, :] - p[:, None, :]
    dd = np.einsum("nmk,nmk->nm", d, d)
    o = c[None, :, :] - p[:, None, :]
    b = np.einsum("nsk,nmk->nms", o, d)
    with np.errstate(invalid="ignore", divide="ignore"):
        t = np.clip(np.where(dd[..., None] > 0, b / dd[..., None], 0.0), 0.0, 1.0)
    q = p[:, None, None, :] + t[..., None] * d[:, :, None, :] - c[None, None, :, :]
    dist2 = np.einsum("nmsk,nmsk->nms", q, q)
    return (np.abs(dist2 - r2[None, None, :]) / r2[None, None, :]).min(axis=2)
