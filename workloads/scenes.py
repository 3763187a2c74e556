"""Seeded scene, G-buffer and parameter generators (inputs only, no method arithmetic).

Every array is produced on the host with ``numpy.random.default_rng(seed)``
and handed, byte for byte, to both the HIP path and the oracle.

Scenes
------
* Unit-cube scene: query points, point lights and sphere occluders drawn
  uniformly in [0,1]^3.
* Box scene: a [0,10]^3 room (floor y=0, ceiling y=10, walls x=0 and z=0),
  axis-aligned boxes, point lights and sphere occluders.  A pinhole camera
  renders a G-buffer (closest hit position and face normal per pixel,
  row-major).  Spheres occlude shadow rays only and are invisible to the
  camera.  This stands in for the G-buffer pass of the paper's renderer
  (Sec. 4, pass 1), which is outside the cache itself.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .configs import GridCfg, MlpCfg

SCENE_EXTENT = 10.0


def _lights(rng, n, lo, hi):
    xyz = rng.uniform(lo, hi, size=(n, 3))
    inten = rng.uniform(0.5, 2.0, size=(n, 1))
    return np.concatenate([xyz, inten], axis=1).astype(np.float32)


def _spheres(rng, n, lo, hi, r_lo, r_hi):
    c = rng.uniform(lo, hi, size=(n, 3))
    r = rng.uniform(r_lo, r_hi, size=(n, 1))
    return np.concatenate([c, r], axis=1).astype(np.float32)


def unit_cube_scene(seed: int, n_points: int, n_lights: int, n_spheres: int,
                    n_train: int = 0, r_lo: float = 0.02, r_hi: float = 0.1) -> dict:
    """Points, lights [M,4] (x,y,z,intensity) and spheres [S,4] (x,y,z,radius) in the unit cube.

    Draw order: points, lights, spheres, training points.
    """
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(n_points, 3)).astype(np.float32)
    lights = _lights(rng, n_lights, 0.0, 1.0)
    spheres = _spheres(rng, n_spheres, 0.0, 1.0, r_lo, r_hi)
    train_pos = rng.uniform(0.0, 1.0, size=(n_train, 3)).astype(np.float32)
    return {"pos": pos, "nrm": None, "pos_unit": pos, "lights": lights, "spheres": spheres,
            "train_pos": train_pos, "extent": 1.0}


def _camera_rays(width: int, height: int, rows: slice, eye, target, vfov_deg: float):
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    tan_h = math.tan(math.radians(vfov_deg) * 0.5)
    aspect = width / height
    j = np.arange(rows.start, rows.stop, dtype=np.float64)
    i = np.arange(width, dtype=np.float64)
    u = (2.0 * (i + 0.5) / width - 1.0) * tan_h * aspect
    v = (1.0 - 2.0 * (j + 0.5) / height) * tan_h
    d = (fwd[None, None, :] + u[None, :, None] * right[None, None, :]
         + v[:, None, None] * up[None, None, :]).reshape(-1, 3)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return eye, d


def _cast(eye, d, boxes_lo, boxes_hi):
    """Closest hit of rays (eye, d) against the room planes and the boxes' outer faces."""
    n = d.shape[0]
    t_best = np.full(n, np.inf)
    nrm = np.zeros((n, 3))
    # Room planes: y=0 (normal +y), y=E (normal -y), x=0 (normal +x), z=0 (normal +z).
    planes = [(1, 0.0, (0, 1, 0)), (1, SCENE_EXTENT, (0, -1, 0)), (0, 0.0, (1, 0, 0)), (2, 0.0, (0, 0, 1))]
    with np.errstate(divide="ignore", invalid="ignore"):
        for axis, val, nn in planes:
            t = (val - eye[axis]) / d[:, axis]
            ok = (t > 1e-9) & (t < t_best)
            t_best = np.where(ok, t, t_best)
            nrm[ok] = nn
        inv = 1.0 / d
        t0 = (boxes_lo[None, :, :] - eye[None, None, :]) * inv[:, None, :]
        t1 = (boxes_hi[None, :, :] - eye[None, None, :]) * inv[:, None, :]
        tmin = np.minimum(t0, t1)
        t_far = np.maximum(t0, t1).min(axis=2)
        axis = tmin.argmax(axis=2)
        t_near = np.take_along_axis(tmin, axis[:, :, None], axis=2)[:, :, 0]
        # Entry hits only: a camera inside a box sees through it.
        ok = (t_near <= t_far) & (t_near > 1e-9)
        t_box = np.where(ok, t_near, np.inf)
        b = t_box.argmin(axis=1)
        tb = t_box[np.arange(n), b]
        hit = tb < t_best
        t_best = np.where(hit, tb, t_best)
        ax = axis[np.arange(n), b]
        nn = np.zeros((n, 3))
        nn[np.arange(n), ax] = -np.sign(d[np.arange(n), ax])
        nrm[hit] = nn[hit]
    return t_best, nrm


def morton_order(width: int, height: int) -> np.ndarray:
    """Row-major pixel indices listed in Z-order (Morton) of (x, y): any run of consecutive
    entries covers a compact 2D block of the image, as in tiled G-buffer layouts."""
    x = np.tile(np.arange(width, dtype=np.uint64), height)
    y = np.repeat(np.arange(height, dtype=np.uint64), width)

    def spread(v):
        v = (v | (v << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x3333333333333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x5555555555555555)
        return v

    key = spread(x) | (spread(y) << np.uint64(1))
    return np.argsort(key, kind="stable")


def box_scene(seed: int, width: int, height: int, n_boxes: int, n_lights: int, n_spheres: int,
              eye=(9.5, 5.0, 9.5), target=(0.0, 3.0, 0.0), vfov_deg: float = 50.0,
              chunk_rows: int = 16, order: str = "morton") -> dict:
    """Box room G-buffer: pos/nrm float32 [H*W, 3] in scene units.

    order='morton' (default) stores the pixels in Z-order of their (x, y) image
    coordinates; order='rows' keeps row-major order; order='shuffled' a seeded
    random permutation (no locality).  `pixel_xy` [H*W, 2] gives
    the image coordinates of every stored pixel.

    Draw order: box min corners U[0,9]^3, box extents U(0.3,1.5)^3 (clipped to
    the room), spheres (centres U[0,10]^3, radius U(0.1,0.8)), lights
    (U[0.5,9.5]^3, intensity U(0.5,2)).
    """
    rng = np.random.default_rng(seed)
    lo = rng.uniform(0.0, 9.0, size=(n_boxes, 3))
    ext = rng.uniform(0.3, 1.5, size=(n_boxes, 3))
    hi = np.minimum(lo + ext, SCENE_EXTENT)
    spheres = _spheres(rng, n_spheres, 0.0, SCENE_EXTENT, 0.1, 0.8)
    lights = _lights(rng, n_lights, 0.5, 9.5)
    pos = np.empty((width * height, 3), np.float32)
    nrm = np.empty((width * height, 3), np.float32)

    def render(r0):
        rows = slice(r0, min(height, r0 + chunk_rows))
        e, d = _camera_rays(width, height, rows, eye, target, vfov_deg)
        t, nn = _cast(e, d, lo, hi)
        if not np.all(np.isfinite(t)):
            raise RuntimeError("camera ray escaped the room")
        p = e[None, :] + t[:, None] * d
        s = r0 * width
        pos[s:s + p.shape[0]] = np.clip(p, 0.0, SCENE_EXTENT)
        nrm[s:s + p.shape[0]] = nn

    # Rows are independent and numpy releases the GIL, so a thread pool is deterministic and faster.
    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        list(ex.map(render, range(0, height, chunk_rows)))
    if order == "morton":
        perm = morton_order(width, height)
    elif order == "rows":
        perm = np.arange(width * height)
    elif order == "shuffled":              # no locality at all: the worst case for the table gathers
        perm = np.random.default_rng(seed + 1000).permutation(width * height)
    else:
        raise ValueError(order)
    pos = np.ascontiguousarray(pos[perm])
    nrm = np.ascontiguousarray(nrm[perm])
    xy = np.stack([perm % width, perm // width], axis=1).astype(np.int32)
    return {"pos": pos, "nrm": nrm, "pos_unit": pos_to_unit(pos, SCENE_EXTENT), "lights": lights,
            "spheres": spheres, "boxes": np.concatenate([lo, hi], axis=1).astype(np.float32),
            "extent": SCENE_EXTENT, "pixel_xy": xy, "order": order}


def pos_to_unit(pos: np.ndarray, extent: float = SCENE_EXTENT) -> np.ndarray:
    """Scene position -> unit cube, x / extent rounded once to FP32 (the caller's step before encoding)."""
    return (pos.astype(np.float64) / extent).astype(np.float32)


def init_params(seed: int, grid: GridCfg, mlp: MlpCfg, table_scale: float = 1e-4,
                init: str = "xavier", weight_gain: float = 1.0) -> dict:
    """Hash-table parameters U(-table_scale, table_scale) [L,T,F] float32 and MLP weights.

    Weights are FP32 row-major [out][in] per layer, input layer first,
    Xavier-uniform (bound sqrt(6/(fan_in+fan_out))) or He-uniform
    (bound sqrt(6/fan_in)), times weight_gain.  Draw order: table, then layers.
    """
    rng = np.random.default_rng(seed)
    table = rng.uniform(-table_scale, table_scale,
                        size=(grid.n_levels, grid.T, grid.n_feat)).astype(np.float32)
    weights = []
    for fo, fi in mlp.layer_shapes():
        if init == "xavier":
            bound = math.sqrt(6.0 / (fi + fo))
        elif init == "he":
            bound = math.sqrt(6.0 / fi)
        else:
            raise ValueError(init)
        weights.append((rng.uniform(-bound, bound, size=(fo, fi)) * weight_gain).astype(np.float32))
    return {"table": table, "weights": weights}


def moving_light(lights: np.ndarray, frame: int, n_frames: int = 60, radius: float = 3.0,
                 center_xz=(5.0, 5.0)) -> np.ndarray:
    """Light list for a frame of the loop: light 0 on a circle of the given radius in the xz-plane."""
    out = lights.copy()
    ang = 2.0 * math.pi * frame / n_frames
    out[0, 0] = np.float32(center_xz[0] + radius * math.cos(ang))
    out[0, 2] = np.float32(center_xz[1] + radius * math.sin(ang))
    return out


def moving_light_table(lights: np.ndarray, n_frames: int = 60, radius: float = 3.0, center_xz=(5.0, 5.0)) -> np.ndarray:
    """Row f = light 0 of `moving_light(lights, f, ...)`: float32 [n_frames][4]."""
    return np.stack([moving_light(lights, f, n_frames, radius, center_xz)[0] for f in range(n_frames)]).astype(np.float32)


class LightAnimation:
    """Per-frame scene update for a recorded frame: light 0 <- row (frame mod n_frames) of a table of
    its positions, the frame read from device counters at run time.  Every buffer is allocated here, so a
    call allocates nothing (it may be recorded into a graph).  table: device float32 [n_frames][4];
    lights: device float32 [m][4]; ctr: device int32 [2] (frame, step)."""

    def __init__(self, table, lights, ctr):
        import torch
        self.table, self.lights, self.ctr = table, lights, ctr
        self.idx = torch.zeros(1, dtype=torch.int64, device=table.device)
        self.row = torch.empty((1, 4), dtype=torch.float32, device=table.device)
        self.n = int(table.shape[0])

    def __call__(self, stream=None):
        import torch
        self.idx.copy_(self.ctr[0:1])
        torch.remainder(self.idx, self.n, out=self.idx)
        torch.index_select(self.table, 0, self.idx, out=self.row)
        self.lights[0:1].copy_(self.row)


def flatten_weights(weights) -> np.ndarray:
    """Concatenate per-layer [out][in] FP32 matrices into the flat master-weight buffer."""
    return np.concatenate([w.reshape(-1) for w in weights]).astype(np.float32)


def unflatten_weights(flat: np.ndarray, mlp: MlpCfg):
    out, off = [], 0
    for fo, fi in mlp.layer_shapes():
        out.append(flat[off:off + fo * fi].reshape(fo, fi))
        off += fo * fi
    return out


def random_visibility(seed: int, n: int, m: int, dtype=np.float16) -> np.ndarray:
    """Synthetic visibility values in [0,1] (exactly representable in dtype), with exact zeros and ones mixed in."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.0, 1.0, size=(n, m))
    kind = rng.integers(0, 8, size=(n, m))
    v = np.where(kind == 0, 0.0, np.where(kind == 1, 1.0, v))
    return v.astype(dtype)
