"""Shared helpers of the GPU parity tests: seeded inputs and a device cache.

Inputs come from `workloads` only; expected values come from `oracle` only.
"""
from __future__ import annotations

import numpy as np

from workloads import get_workload, init_params
from workloads.scenes import flatten_weights

# Parameter scale giving a realistic activation range (logit std ~1.5, visibility
# spanning (0.005, 1)) instead of the near-constant 0.5 of a fresh network.
TRAINED_SCALE = dict(table_scale=1.0, weight_gain=2.0)


def params(wl, seed=1, **kw):
    kw = {**TRAINED_SCALE, **kw}
    return init_params(seed, wl.grid, wl.mlp, **kw)


def make_cache(wl, p, dtype=None, device="cuda", **kw):
    from dataclasses import replace

    from paper_2506_05930_amd.cache import NVCache
    mlp = wl.mlp if dtype is None else replace(wl.mlp, dtype=dtype)
    return NVCache(wl.grid, mlp, p["table"], p["weights"], device=device, seed=wl.rng_key, lr=wl.lr,
                   beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps, loss=wl.loss, vis_floor=wl.vis_floor,
                   lr_end=wl.lr_end, lr_decay_steps=wl.lr_decay_steps, **kw)


def rand_pos(seed, n, adversarial=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    if adversarial and n >= 16:
        special = np.array([[0, 0, 0], [1, 1, 1], [0.5, 0.25, 0.75], [1, 0, 0.5],
                            [np.nextafter(np.float32(0.5), np.float32(0)), 0.5, np.nextafter(np.float32(1), np.float32(0))],
                            [-0.1, 1.2, 0.3], [1 / 3, 2 / 3, 0.999999], [0.0625, 0.125, 0.1875]], np.float32)
        pos[:len(special)] = special
    return pos


def tiny():
    return get_workload("tiny")


def p1080():
    return get_workload("frame_1080p")


__all__ = ["params", "make_cache", "rand_pos", "tiny", "p1080", "flatten_weights", "TRAINED_SCALE"]
