"""Philox4x32-10 counter-based generator, written from its published description.

Test infrastructure (see the package docstring).

Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3"
(SC 2011), Sec. 3: a 4x32-bit counter and a 2x32-bit key; each of the ten
rounds multiplies two counter words by fixed 32-bit constants, keeps both
halves of each 64-bit product and mixes the high halves with the other two
counter words and the round key; the key is advanced by two Weyl constants
between rounds.

The paper under study does not name a generator; the cache needs one uniform
per pixel for light selection and one pixel index per training sample.
Counter layout used here: (index low 32 bits, index high 32 bits, frame, tag),
key = (seed low 32 bits, seed high 32 bits); tag 0 = light selection,
tag 1 = training-pixel selection.
"""
from __future__ import annotations

import numpy as np

MUL0 = 0xD2511F53
MUL1 = 0xCD9E8D57
WEYL0 = 0x9E3779B9
WEYL1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

TAG_WRS = 0
TAG_TRAIN_PIXEL = 1
TAG_WORLD_POINT = 6


def philox4x32_10(ctr, key):
    """ctr: 4 arrays (or ints) of uint32 words; key: 2 words.  Returns 4 uint64 arrays holding uint32 values."""
    x = [np.asarray(c, dtype=np.uint64) & MASK32 for c in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK32
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK32
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + WEYL0) & MASK32
            k1 = (k1 + WEYL1) & MASK32
        p0 = x[0] * np.uint64(MUL0)          # < 2^64: both factors < 2^32
        p1 = x[2] * np.uint64(MUL1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        x = [hi1 ^ x[1] ^ k0, lo1, hi0 ^ x[3] ^ k1, lo0]
    return x


def _counter(index, frame, tag):
    index = np.asarray(index, dtype=np.uint64)
    return (index & np.uint64(MASK32), index >> np.uint64(32),
            np.full(index.shape, frame & MASK32, np.uint64), np.full(index.shape, tag, np.uint64))


def _key(seed):
    return (seed & MASK32, (seed >> 32) & MASK32)


def uniform24(word) -> np.ndarray:
    """Top 24 bits of a 32-bit word scaled by 2^-24: a uniform in [0, 1 - 2^-24], exact in FP32."""
    return ((np.asarray(word, np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def wrs_uniforms(seed: int, frame: int, n: int, first: int = 0) -> np.ndarray:
    """The light-selection uniform of pixels first..first+n-1 (tag 0)."""
    r = philox4x32_10(_counter(np.arange(first, first + n, dtype=np.uint64), frame, TAG_WRS), _key(seed))
    return uniform24(r[0])


def world_points(seed: int, frame: int, n: int, box, extent: float):
    """World-space training points (Sec. 3.4: samples at random scene positions, not only on the visible
    surfaces): point i is lo + u * (hi - lo) per axis with u = uniform24 of words 0, 1, 2 of counter
    (i, frame, 6), in FP32 (ext = hi - lo, then u * ext, then + lo); its unit-cube position is p / extent
    (FP32 division).  Returns (pos_scene [n,3], pos_unit [n,3]) float32."""
    r = philox4x32_10(_counter(np.arange(n, dtype=np.uint64), frame, TAG_WORLD_POINT), _key(seed))
    lo = np.asarray(box[:3], np.float32)
    hi = np.asarray(box[3:], np.float32)
    ext = hi - lo
    u = np.stack([uniform24(r[k]) for k in range(3)], axis=1)
    p = (u * ext[None, :]) + lo[None, :]
    return p.astype(np.float32), (p / np.float32(extent)).astype(np.float32)


def training_pixels(seed: int, frame: int, batch: int, n_pix: int) -> np.ndarray:
    """Training pixel of each of `batch` samples, uniform with replacement: floor(r0 * n_pix / 2^32)."""
    if not 0 < n_pix < (1 << 32):
        raise ValueError("n_pix out of range")
    r = philox4x32_10(_counter(np.arange(batch, dtype=np.uint64), frame, TAG_TRAIN_PIXEL), _key(seed))
    return ((r[0] * np.uint64(n_pix)) >> np.uint64(32)).astype(np.int64)
