"""Pins of the oracle's hash-grid encoding (Sec. 3.1 Fig. overview; Sec. 3.3; Mueller et al. 2022)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import hashgrid

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_spatial_hash_hand_values():
    for case in _load("spatial_hash_hand.json")["cases"]:
        cx, cy, cz = case["c"]
        h = hashgrid.spatial_hash(np.array([cx]), np.array([cy]), np.array([cz]), 1 << case["log2_T"])
        assert int(h[0]) == case["h"], case


def test_spatial_hash_matches_python_integers():
    # Independent evaluation with unbounded Python integers reduced mod 2^32 once at the end.
    rng = np.random.default_rng(7)
    c = rng.integers(0, 5000, size=(2000, 3))
    for log2_T in (10, 14, 19, 20, 24):
        T = 1 << log2_T
        h = hashgrid.spatial_hash(c[:, 0], c[:, 1], c[:, 2], T)
        ref = [((int(x) * 1) ^ (int(y) * 2654435761) ^ (int(z) * 805459861)) % (1 << 32) % T
               for x, y, z in c]
        assert np.array_equal(h, np.array(ref))


def test_level_resolutions_hand_and_exact():
    case = _load("level_resolutions.json")["cases"][0]
    res = hashgrid.level_resolutions(case["base"], case["growth"], case["levels"])
    assert res == case["res"]
    dense = [hashgrid.level_is_dense(r, 1 << case["log2_T"]) for r in res]
    assert dense == case["dense"]
    # growth 1.447: exact rational arithmetic, floor(16 * (1447/1000)^l).
    exact = [int((16 * Fraction(1447, 1000) ** l).__floor__()) for l in range(16)]
    assert hashgrid.level_resolutions(16, 1.447, 16) == exact
    # growth 1.447 at T = 2^19: the first five levels are dense.
    assert [hashgrid.level_is_dense(r, 1 << 19) for r in exact[:6]] == [True] * 5 + [False]


def test_dense_index_is_ravel_multi_index():
    rng = np.random.default_rng(1)
    N = 36
    c = rng.integers(0, N + 1, size=(500, 3))
    idx = hashgrid.dense_index(c[:, 0], c[:, 1], c[:, 2], N)
    ref = np.ravel_multi_index((c[:, 2], c[:, 1], c[:, 0]), (N + 1,) * 3)
    assert np.array_equal(idx, ref)


def test_cell_boundaries_and_clamp():
    pos = np.array([[0.0, 1.0, 0.5], [-0.25, 2.0, np.nan], [np.nextafter(np.float32(0.5), np.float32(0)), 0.5, 1.0]],
                   np.float32)
    c, f = hashgrid.cell_and_fraction(pos, 16)
    # x=0 -> cell 0 frac 0; x=1 -> last cell (15) frac 1; x=0.5 -> vertex 8 frac 0
    assert c[0].tolist() == [0, 15, 8] and f[0].tolist() == [0.0, 1.0, 0.0]
    # clamped: -0.25 -> 0, 2 -> 1, NaN -> 0
    assert c[1].tolist() == [0, 15, 0] and f[1].tolist() == [0.0, 1.0, 0.0]
    # just below 0.5: 16 * (0.5 - 2^-25) rounds to 8 - 2^-21 in FP32 -> cell 7, frac just below 1
    assert c[2, 0] == 7 and 0.999 < f[2, 0] < 1.0


def test_worked_vertex_example():
    # x = (0.5, 0.25, 0.75) at N = 36 scales to the vertex (18, 9, 27): fraction 0,
    # so the encoding equals the stored feature of that vertex exactly.
    T = 1 << 14
    rng = np.random.default_rng(3)
    table = rng.uniform(-1, 1, size=(1, T, 2)).astype(np.float32)
    # level 0 of base 36: one level only
    enc = hashgrid.encode(np.array([[0.5, 0.25, 0.75]], np.float32), table, 36, 1.0)
    h = ((18 * 1) ^ ((9 * 2654435761) % (1 << 32)) ^ ((27 * 805459861) % (1 << 32))) % T
    assert not hashgrid.level_is_dense(36, T)
    assert np.array_equal(enc[0], table[0, h].astype(np.float64))


def test_trilinear_weights_sum_to_one_and_nonnegative():
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 1, size=(5000, 3)).astype(np.float32)
    for res in (16, 101, 4084):
        _, w = hashgrid.corners(pos, res, 1 << 19)
        assert np.all(w >= 0)
        assert np.max(np.abs(w.sum(axis=1) - 1.0)) <= 4e-16


def test_linear_reproduction_on_dense_level():
    # theta(vertex) = a . vertex + b on a dense level -> encoding = a . s + b exactly (trilinear is exact on linear data).
    N = 16
    T = 1 << 14
    a = np.array([0.25, -0.5, 0.125])
    b0 = 0.75
    table = np.zeros((1, T, 2), np.float32)
    v = np.stack(np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij"), -1).reshape(-1, 3)
    idx = hashgrid.dense_index(v[:, 0], v[:, 1], v[:, 2], N)
    table[0, idx, 0] = (v @ a + b0).astype(np.float32)
    table[0, idx, 1] = v[:, 2].astype(np.float32)
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 1, size=(3000, 3)).astype(np.float32)
    enc = hashgrid.encode(pos, table, N, 1.0)
    s = pos.astype(np.float32) * np.float32(N)
    assert np.max(np.abs(enc[:, 0] - (s.astype(np.float64) @ a + b0))) < 1e-12
    assert np.max(np.abs(enc[:, 1] - s[:, 2])) < 1e-12


def test_matches_scipy_regular_grid_interpolator_on_dense_level():
    from scipy.interpolate import RegularGridInterpolator
    N = 24
    T = 1 << 15
    rng = np.random.default_rng(5)
    grid_vals = rng.normal(size=(N + 1, N + 1, N + 1, 2))
    table = np.zeros((1, T, 2), np.float32)
    v = np.stack(np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij"), -1).reshape(-1, 3)
    idx = hashgrid.dense_index(v[:, 0], v[:, 1], v[:, 2], N)
    table[0, idx] = grid_vals[v[:, 0], v[:, 1], v[:, 2]].astype(np.float32)
    pos = rng.uniform(0, 1, size=(2000, 3)).astype(np.float32)
    enc = hashgrid.encode(pos, table, N, 1.0)
    axes = [np.arange(N + 1, dtype=np.float64)] * 3
    for j in range(2):
        interp = RegularGridInterpolator(axes, grid_vals[..., j].astype(np.float32).astype(np.float64))
        ref = interp((pos.astype(np.float32) * np.float32(N)).astype(np.float64))
        assert np.max(np.abs(enc[:, j] - ref)) < 1e-12


def test_levels_concatenate_level_major():
    T = 1 << 14
    rng = np.random.default_rng(6)
    table = np.zeros((3, T, 2), np.float32)
    table[1, :, 1] = 1.0            # only level 1, feature 1 is non-zero, constant
    pos = rng.uniform(0, 1, size=(10, 3)).astype(np.float32)
    enc = hashgrid.encode(pos, table, 16, 1.5)
    expect = np.zeros((10, 6))
    expect[:, 1 * 2 + 1] = 1.0
    assert np.allclose(enc, expect, atol=1e-15)


@pytest.mark.parametrize("mutant", ["prime", "offset", "no_clamp_min"])
def test_pins_catch_planted_mistakes(monkeypatch, mutant):
    """A plausible mistake in the oracle makes one of the pins fail (mistake planted on the CPU)."""
    if mutant == "prime":
        monkeypatch.setattr(hashgrid, "PRIMES", (1, 2654435769, 805459861))
        orig = hashgrid.spatial_hash

        def bad(cx, cy, cz, T):
            m32 = np.uint64(0xFFFFFFFF)
            hx = np.asarray(cx, np.uint64) & m32
            hy = (np.asarray(cy, np.uint64) * np.uint64(hashgrid.PRIMES[1])) & m32
            hz = (np.asarray(cz, np.uint64) * np.uint64(hashgrid.PRIMES[2])) & m32
            return ((hx ^ hy ^ hz) & np.uint64(T - 1)).astype(np.int64)
        monkeypatch.setattr(hashgrid, "spatial_hash", bad)
        with pytest.raises(AssertionError):
            test_spatial_hash_hand_values()
        monkeypatch.setattr(hashgrid, "spatial_hash", orig)
    elif mutant == "offset":
        orig = hashgrid.cell_and_fraction

        def bad(pos32, res):
            x = hashgrid.clamp_unit(pos32)
            s = x * np.float32(res) + np.float32(0.5)      # half-cell offset
            c = np.minimum(np.floor(s), np.float32(res - 1)).astype(np.int64)
            return c, s.astype(np.float64) - c
        monkeypatch.setattr(hashgrid, "cell_and_fraction", bad)
        with pytest.raises(AssertionError):
            test_linear_reproduction_on_dense_level()
        monkeypatch.setattr(hashgrid, "cell_and_fraction", orig)
    else:
        orig = hashgrid.cell_and_fraction

        def bad(pos32, res):
            x = hashgrid.clamp_unit(pos32)
            s = x * np.float32(res)
            c = np.floor(s).astype(np.int64)                 # x = 1 leaves the grid
            return c, s.astype(np.float64) - c
        monkeypatch.setattr(hashgrid, "cell_and_fraction", bad)
        with pytest.raises(AssertionError):
            test_cell_boundaries_and_clamp()
        monkeypatch.setattr(hashgrid, "cell_and_fraction", orig)
