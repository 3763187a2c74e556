"""Multi-resolution hash-grid encoding of a 3D position.

Test infrastructure (see the package docstring).

The cache encodes the query position with the multi-resolution hash grid of
Mueller et al. 2022 before the MLP (Sec. 3.1, Fig. "overview", step 1;
Sec. 3.3 gives levels, base resolution and features per level).  The paper
does not restate the encoding, so this follows the Instant-NGP paper:

* level l has resolution N_l = floor(N_min * b^l)                (its eq. 2)
* the position is scaled by N_l; the cell is the floor, the fractional part
  gives trilinear weights over the 8 cell corners                (its eq. 3, Sec. 3)
* a level whose (N_l+1)^3 vertices fit in the T table entries is indexed
  densely (one-to-one); otherwise the spatial hash
  h(x) = (x_1*pi_1 XOR x_2*pi_2 XOR x_3*pi_3) mod T with pi = 1, 2654435761,
  805459861 is used                                              (its eq. 4)
* the F features of the 8 corners are blended with the trilinear weights and
  the L levels are concatenated, level-major: feature j of level l lands in
  slot l*F + j.

Readings where both papers are silent: positions are clamped to [0,1]; the
scale has no half-cell offset; a position at 1.0 falls in the last cell with
fraction 1; corner delta = (dx, dy, dz) is corner number dx + 2*dy + 4*dz.
The cell is an integer decided by floating point, so it is computed in FP32
(s = fl32(x * N_l), one rounding) as the kernels do; weights and sums are FP64.
"""
from __future__ import annotations

import math

import numpy as np

PRIMES = (1, 2654435761, 805459861)


def level_resolutions(base_res: int, growth: float, n_levels: int) -> list[int]:
    """N_l = floor(base_res * growth**l), FP64 on the host."""
    return [int(math.floor(base_res * growth ** l)) for l in range(n_levels)]


def level_is_dense(res: int, T: int) -> bool:
    """A level is stored densely when all (N+1)^3 grid vertices fit in its T entries."""
    return (res + 1) ** 3 <= T


def clamp_unit(pos32: np.ndarray) -> np.ndarray:
    """min(max(x, 0), 1) in FP32 with NaN mapped to 0 (max first, NaN-ignoring)."""
    p = np.asarray(pos32, dtype=np.float32)
    return np.fmin(np.fmax(p, np.float32(0.0)), np.float32(1.0))


def cell_and_fraction(pos32: np.ndarray, res: int):
    """Cell c (int64, [n,3]) and fraction f (FP64, [n,3]) of each position at resolution res."""
    x = clamp_unit(pos32)
    s = x * np.float32(res)                       # FP32 product, one rounding
    c = np.minimum(np.floor(s), np.float32(res - 1)).astype(np.int64)
    f = s.astype(np.float64) - c                  # exact
    return c, f


def corner_offsets() -> np.ndarray:
    """[8,3] corner offsets, corner k = (k & 1, (k >> 1) & 1, (k >> 2) & 1)."""
    k = np.arange(8)
    return np.stack([k & 1, (k >> 1) & 1, (k >> 2) & 1], axis=1).astype(np.int64)


def spatial_hash(cx, cy, cz, T: int) -> np.ndarray:
    """(cx*1 XOR cy*2654435761 XOR cz*805459861) mod 2^32, then mod T (T a power of two)."""
    m32 = np.uint64(0xFFFFFFFF)
    hx = (np.asarray(cx, np.uint64) * np.uint64(PRIMES[0])) & m32
    hy = (np.asarray(cy, np.uint64) * np.uint64(PRIMES[1])) & m32
    hz = (np.asarray(cz, np.uint64) * np.uint64(PRIMES[2])) & m32
    return ((hx ^ hy ^ hz) & np.uint64(T - 1)).astype(np.int64)


def dense_index(cx, cy, cz, res: int) -> np.ndarray:
    """Row-major vertex index x + (N+1)*y + (N+1)^2*z of a dense level."""
    n1 = res + 1
    return np.asarray(cx, np.int64) + n1 * (np.asarray(cy, np.int64) + n1 * np.asarray(cz, np.int64))


def corners(pos32: np.ndarray, res: int, T: int):
    """Table index [n,8] and trilinear weight [n,8] (FP64) of the 8 corners of each position's cell."""
    c, f = cell_and_fraction(pos32, res)
    off = corner_offsets()
    cc = c[:, None, :] + off[None, :, :]                               # [n,8,3]
    if level_is_dense(res, T):
        idx = dense_index(cc[..., 0], cc[..., 1], cc[..., 2], res)
    else:
        idx = spatial_hash(cc[..., 0], cc[..., 1], cc[..., 2], T)
    w = np.ones(idx.shape, np.float64)
    for k in range(3):
        w = w * np.where(off[None, :, k] == 1, f[:, None, k], 1.0 - f[:, None, k])
    return idx, w


def encode(pos32: np.ndarray, table: np.ndarray, base_res: int, growth: float,
           return_corners: bool = False):
    """Encoding [n, L*F] (FP64) of FP32 unit-cube positions with FP32 table [L,T,F]."""
    L, T, F = table.shape
    res = level_resolutions(base_res, growth, L)
    n = pos32.shape[0]
    enc = np.zeros((n, L * F), np.float64)
    cache = []
    for l in range(L):
        idx, w = corners(pos32, res[l], T)
        vals = table[l].astype(np.float64)[idx]                          # [n,8,F]
        enc[:, l * F:(l + 1) * F] = np.einsum("nk,nkf->nf", w, vals)
        cache.append((idx, w))
    if return_corners:
        return enc, cache
    return enc
