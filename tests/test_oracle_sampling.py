"""Pins of the oracle's light weights, WRS, generator, shadow labels and estimator moments."""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import estimator, lighting, philox, shadow

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- generator
def test_philox_known_answers():
    with open(os.path.join(GOLD, "philox4x32_10_kat.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        out = philox.philox4x32_10([int(x, 16) for x in c["ctr"]], [int(x, 16) for x in c["key"]])
        assert [int(v) for v in out] == [int(x, 16) for x in c["out"]]


def test_uniforms_are_exact_fp32_and_uniform():
    u = philox.wrs_uniforms(seed=2, frame=0, n=1 << 20)
    assert u.dtype == np.float32
    assert np.all(u >= 0) and np.all(u < 1)
    k = (u.astype(np.float64) * 2 ** 24)
    assert np.all(k == np.floor(k))                      # multiples of 2^-24
    counts = np.bincount((u * 64).astype(np.int64), minlength=64)
    assert stats.chisquare(counts).pvalue > 1e-3


def test_training_pixels_range_and_uniformity():
    pix = philox.training_pixels(seed=2, frame=3, batch=1 << 18, n_pix=1920 * 1080)
    assert pix.min() >= 0 and pix.max() < 1920 * 1080
    counts = np.bincount(pix * 50 // (1920 * 1080), minlength=50)
    assert stats.chisquare(counts).pvalue > 1e-3
    # distinct frames give different batches
    assert not np.array_equal(pix[:100], philox.training_pixels(2, 4, 100, 1920 * 1080))


# ------------------------------------------------------------- light weights
def test_unshadowed_weight_closed_forms():
    pos = np.zeros((1, 3))
    nrm = np.array([[0.0, 1.0, 0.0]])
    lights = np.array([[0, 2, 0, 3.0],       # straight above at distance 2: I/d^2 = 3/4
                       [2, 0, 0, 1.0],       # grazing: cos = 0
                       [0, -2, 0, 1.0],      # behind the surface: 0
                       [1, 1, 0, 2.0]])      # 45 degrees, d^2 = 2: 2 * (1/sqrt2) / 2
    f = lighting.unshadowed_weight(pos, nrm, lights)
    assert np.allclose(f[0], [0.75, 0.0, 0.0, 1 / math.sqrt(2)], rtol=1e-15, atol=0)
    f_nn = lighting.unshadowed_weight(pos, None, lights)
    assert np.allclose(f_nn[0], [0.75, 0.25, 0.25, 1.0], rtol=1e-15)


def test_unshadowed_weight_fp32_close_to_fp64():
    rng = np.random.default_rng(0)
    pos = rng.uniform(0, 10, size=(2000, 3)).astype(np.float32)
    nrm = rng.normal(size=(2000, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    lights = np.concatenate([rng.uniform(0.5, 9.5, size=(32, 3)), rng.uniform(0.5, 2, size=(32, 1))], 1).astype(np.float32)
    f32 = lighting.unshadowed_weight(pos, nrm, lights, np.float32)
    f64 = lighting.unshadowed_weight(pos, nrm, lights, np.float64)
    big = f64 > 1e-3
    assert np.max(np.abs(f32[big] - f64[big]) / f64[big]) < 1e-5


def test_clamp_floor():
    v = np.array([-1.0, 0.0, 5e-4, 1e-3, 0.5, np.nan])
    assert lighting.clamp_visibility(v).tolist() == [1e-3, 1e-3, 1e-3, 1e-3, 0.5, 1e-3]
    assert lighting.clamp_visibility(v, 0.0)[:2].tolist() == [0.0, 0.0]


# ------------------------------------------------------------------- WRS
def _dyadic_rows(rng, n, m):
    k = rng.integers(0, 65, size=(n, m))
    k[0] = 0
    k[1] = 0
    k[1, m // 2] = 64
    return k, (k / 64.0).astype(np.float32)


def test_wrs_exact_counts_on_dyadic_lattice():
    """Weights k_i/64 and u = j/4096: every sum and product is exact, so the
    number of lattice points u_j that pick light i is exactly 4096 * w_i / W
    when W is a power of two (brute force over all 4096 u values)."""
    rng = np.random.default_rng(1)
    m = 8
    for _ in range(20):
        k = rng.integers(0, 9, size=m)
        k[rng.integers(0, m)] += 64 - k.sum() if k.sum() < 64 else 0
        if k.sum() != 64:
            k = np.zeros(m, np.int64)
            k[:4] = 16
        w = np.tile((k / 64.0).astype(np.float32), (4096, 1))
        u = (np.arange(4096) / 4096.0).astype(np.float32)
        idx, pmf, W = lighting.wrs_pick(w, u)
        assert np.all(W == 1.0)
        counts = np.bincount(idx, minlength=m)
        assert counts.tolist() == (k * 64).tolist()
        assert np.all(pmf == w[0][idx])


def test_wrs_ties_go_to_the_next_light_and_zero_weights_never_picked():
    w = np.array([[0.25, 0.0, 0.25, 0.5]] * 4, np.float32)
    u = np.array([0.0, 0.25, 0.5, 0.75], np.float32)      # u*W hits C_0 = 0.25 exactly at u = 0.25
    idx, pmf, W = lighting.wrs_pick(w, u)
    assert idx.tolist() == [0, 2, 3, 3]
    assert pmf.tolist() == [0.25, 0.25, 0.5, 0.5]


def test_wrs_all_zero_row():
    idx, pmf, W = lighting.wrs_pick(np.zeros((2, 4), np.float32), np.array([0.1, 0.9], np.float32))
    assert idx.tolist() == [-1, -1] and pmf.tolist() == [0, 0] and W.tolist() == [0, 0]


def test_wrs_cumsum_is_sequential_fp32():
    rng = np.random.default_rng(2)
    w = rng.uniform(0, 1, size=(50, 32)).astype(np.float32) * (10.0 ** rng.integers(-3, 3, size=(50, 32))).astype(np.float32)
    C = np.cumsum(w, axis=1, dtype=np.float32)
    for r in range(50):
        acc = np.float32(0)
        for i in range(32):
            acc = np.float32(acc + w[r, i])
            assert C[r, i] == acc


@pytest.mark.parametrize("m", [8, 32])
def test_wrs_chi_square(m):
    rng = np.random.default_rng(3 + m)
    w_row = rng.uniform(0, 1, size=m).astype(np.float32)
    w_row[rng.integers(0, m)] = 0.0
    n = 1 << 20
    u = philox.wrs_uniforms(seed=9, frame=1, n=n)
    idx, _, W = lighting.wrs_pick(np.tile(w_row, (n, 1)), u)
    counts = np.bincount(idx, minlength=m)
    p = w_row.astype(np.float64) / w_row.astype(np.float64).sum()
    nz = p > 0
    assert counts[~nz].sum() == 0
    assert stats.chisquare(counts[nz], n * p[nz]).pvalue > 1e-3


def test_wrs_fp32_pick_agrees_with_fp64_away_from_boundaries():
    rng = np.random.default_rng(4)
    w = rng.uniform(0, 1, size=(20000, 32))
    u = philox.wrs_uniforms(5, 0, 20000)
    i32, _, _ = lighting.wrs_pick(w.astype(np.float32), u)
    i64, _, _ = lighting.wrs_pick(w.astype(np.float32).astype(np.float64), u)
    mism = np.nonzero(i32 != i64)[0]
    C = np.cumsum(w.astype(np.float32).astype(np.float64), axis=1)
    for r in mism:
        t = u[r] * C[r, -1]
        assert np.min(np.abs(C[r] - t)) <= 4 * np.spacing(np.float32(C[r, -1]))
    assert len(mism) <= 10


def test_selection_pmf_proportional_to_weights():
    rng = np.random.default_rng(6)
    w = rng.uniform(0, 1, size=(100, 8))
    p = lighting.selection_pmf(w)
    assert np.allclose(p.sum(1), 1.0, atol=1e-15)
    assert np.allclose(p * w.sum(1, keepdims=True), w, atol=1e-15)


def test_neural_di_with_true_visibility_is_brute_force_di():
    rng = np.random.default_rng(7)
    f = rng.uniform(0, 2, size=(10, 8))
    V = (rng.uniform(size=(10, 8)) > 0.5).astype(np.float64)
    assert np.allclose(lighting.neural_di(V, f), [sum(f[i, j] for j in range(8) if V[i, j]) / math.pi
                                                  for i in range(10)], atol=1e-15)


# ------------------------------------------------------------ shadow labels
def test_labels_analytic_cases():
    p = np.array([[0.0, 0.0, 0.0]])
    light = np.array([[4.0, 0.0, 0.0, 1.0]])
    cases = [
        ([2.0, 0.0, 0.0, 0.5], 0),     # centred on the segment
        ([2.0, 0.6, 0.0, 0.5], 1),     # off axis, distance 0.6 > 0.5
        ([2.0, 0.4, 0.0, 0.5], 0),     # off axis, distance 0.4 < 0.5
        ([6.0, 0.0, 0.0, 1.0], 1),     # behind the light
        ([-2.0, 0.0, 0.0, 1.0], 1),    # behind the point
        ([0.0, 0.0, 0.0, 0.25], 0),    # point inside
        ([4.0, 0.1, 0.0, 0.25], 0),    # light inside
        ([2.0, 0.5, 0.0, 0.5], 1),     # tangent: counts as visible
        ([4.5, 0.0, 0.0, 0.5], 1),     # touches the light only at distance 0.5: tangent
    ]
    for sph, expect in cases:
        s = np.array([sph])
        assert shadow.labels(p, light, s)[0, 0] == expect, sph
        assert shadow.labels_fp32(p, light, s)[0, 0] == expect, sph


def _labels_quadratic(p, l, spheres):
    """Brute force through the ray-sphere quadratic: occluded if a root lies in [0,1] or p is inside."""
    d = l - p
    out = 1
    for c, r in zip(spheres[:, :3], spheres[:, 3]):
        o = p - c
        a = d @ d
        b = 2 * (o @ d)
        cc = o @ o - r * r
        if cc < 0:
            return 0
        disc = b * b - 4 * a * cc
        if disc <= 0:
            continue
        sq = math.sqrt(disc)
        t0, t1 = (-b - sq) / (2 * a), (-b + sq) / (2 * a)
        if (0 <= t0 <= 1) or (0 <= t1 <= 1):
            out = 0
    return out


def test_labels_match_quadratic_brute_force_on_tiny_scene():
    rng = np.random.default_rng(8)
    pos = rng.uniform(0, 1, size=(300, 3))
    lights = np.concatenate([rng.uniform(0, 1, size=(8, 3)), np.ones((8, 1))], 1)
    spheres = np.concatenate([rng.uniform(0, 1, size=(16, 3)), rng.uniform(0.02, 0.1, size=(16, 1))], 1)
    lab = shadow.labels(pos, lights, spheres)
    ref = np.array([[_labels_quadratic(pos[i], lights[j, :3], spheres) for j in range(8)] for i in range(300)])
    assert np.array_equal(lab, ref)
    assert 0 < lab.mean() < 1


def test_labels_fp32_decision_agrees_with_fp64_away_from_tangency():
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, 10, size=(3000, 3)).astype(np.float32)
    lights = np.concatenate([rng.uniform(0.5, 9.5, size=(32, 3)), np.ones((32, 1))], 1).astype(np.float32)
    spheres = np.concatenate([rng.uniform(0, 10, size=(256, 3)), rng.uniform(0.1, 0.8, size=(256, 1))], 1).astype(np.float32)
    a = shadow.labels(pos, lights, spheres)
    b = shadow.labels_fp32(pos, lights, spheres)
    diff = a != b
    if diff.any():
        margin = shadow.tangency_margin(pos, lights, spheres)
        assert np.all(margin[diff] < 1e-4)
    assert diff.mean() < 1e-4
    assert 0.2 < a.mean() < 0.99


# ----------------------------------------------------------------- estimator
def test_estimator_zero_variance_for_ideal_pmf_and_bias_without_clamp():
    rng = np.random.default_rng(10)
    f = rng.uniform(0.1, 2, size=(50, 8))
    V = (rng.uniform(size=(50, 8)) > 0.3).astype(np.float64)
    V[:, 0] = 1.0
    ideal = lighting.selection_pmf(f * V)
    mu, E, var, waste = estimator.moments(f, V, ideal)
    assert np.allclose(E, mu) and np.max(np.abs(var)) < 1e-12 and np.all(waste == 0)
    # a cache that predicts 0 for a visible light, unclamped: biased (E < mu)
    vhat = V.copy()
    vhat[:, 0] = 0.0
    p_biased = lighting.selection_pmf(f * lighting.clamp_visibility(vhat, 0.0))
    _, E_b, _, _ = estimator.moments(f, V, p_biased)
    assert np.all(E_b < mu)
    # clamped: unbiased again
    p_clamped = lighting.selection_pmf(f * lighting.clamp_visibility(vhat, 1e-3))
    _, E_c, _, _ = estimator.moments(f, V, p_clamped)
    assert np.allclose(E_c, mu)


def test_estimator_variance_matches_monte_carlo():
    rng = np.random.default_rng(11)
    f = rng.uniform(0.1, 2, size=(1, 6))
    V = np.array([[1, 0, 1, 1, 0, 1]], np.float64)
    p = lighting.selection_pmf(f)
    mu, E, var, waste = estimator.moments(f, V, p)
    n = 400000
    pick = rng.choice(6, size=n, p=p[0])
    est = f[0, pick] * V[0, pick] / p[0, pick]
    assert abs(est.mean() - mu[0]) < 4 * math.sqrt(var[0] / n)
    assert abs(est.var() - var[0]) < 0.02 * var[0]
    assert abs((V[0, pick] == 0).mean() - waste[0]) < 0.005
