"""Pins of the clustered oracle (Sec. 3.6): k-means, cluster labels, two-step sampling."""
import numpy as np
import pytest

from oracle import clustered, lighting, shadow
from workloads import box_scene


def _lights(rng, n):
    return np.concatenate([rng.uniform(0.5, 9.5, (n, 3)), rng.uniform(0.5, 2, (n, 1))], 1).astype(np.float32)


def test_kmeans_recovers_separated_blobs():
    rng = np.random.default_rng(0)
    centres = rng.uniform(0, 100, (6, 3))
    centres[:, 0] = np.arange(6) * 40.0                       # far apart along x
    lab = rng.integers(0, 6, 600)
    pts = centres[lab] + rng.normal(0, 0.5, (600, 3))
    lights = np.concatenate([pts, np.ones((600, 1))], 1).astype(np.float32)
    off, mem = clustered.kmeans(lights, 6, iters=50)
    groups = [set(mem[off[j]:off[j + 1]].tolist()) for j in range(6)]
    truth = [set(np.nonzero(lab == b)[0].tolist()) for b in range(6)]
    assert sorted(map(sorted, groups)) == sorted(map(sorted, truth))


def test_kmeans_result_is_a_lloyd_fixed_point():
    rng = np.random.default_rng(1)
    lights = _lights(rng, 700)
    off, mem = clustered.kmeans(lights, 32, iters=200)
    assert off[0] == 0 and off[-1] == 700 and np.array_equal(np.sort(mem), np.arange(700))
    P = lights[:, :3].astype(np.float64)
    cent = np.array([P[mem[off[j]:off[j + 1]]].mean(0) for j in range(32) if off[j + 1] > off[j]])
    nonempty = [j for j in range(32) if off[j + 1] > off[j]]
    assign = np.empty(700, np.int64)
    for j in range(32):
        assign[mem[off[j]:off[j + 1]]] = j
        assert np.all(np.diff(mem[off[j]:off[j + 1]]) > 0)          # ascending light index
    d2 = ((P[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
    nearest = np.array(nonempty)[d2.argmin(1)]
    assert np.array_equal(nearest, assign)                           # every light at its nearest mean


def test_training_lights_uniform_in_their_cluster():
    off = np.array([0, 5, 5, 8])
    mem = np.array([10, 11, 12, 13, 14, 20, 21, 22])
    ch = clustered.training_lights(2, 3, 60000, off, mem)
    assert np.all(ch[:, 1] == -1)
    assert np.all(np.isin(ch[:, 0], mem[0:5])) and np.all(np.isin(ch[:, 2], mem[5:8]))
    cnt = np.array([(ch[:, 0] == l).sum() for l in mem[0:5]])
    chi2 = ((cnt - 12000.0) ** 2 / 12000.0).sum()
    assert chi2 < 18.5                                               # 4 dof, p ~ 1e-3


def test_singleton_clusters_reduce_to_the_plain_labels():
    sc = box_scene(0, 40, 24, 16, 12, 64)
    n = sc["pos"].shape[0]
    off, mem = np.arange(13), np.arange(12)
    ch = clustered.training_lights(2, 0, n, off, mem)
    assert np.array_equal(ch, np.tile(np.arange(12), (n, 1)))
    lab = clustered.labels(sc["pos"], sc["lights"], sc["spheres"], ch)
    assert np.array_equal(lab, shadow.labels_fp32(sc["pos"], sc["lights"], sc["spheres"]))


def _tiny_case(seed, sizes):
    rng = np.random.default_rng(seed)
    L = int(sum(sizes))
    f = rng.uniform(0.1, 2.0, L)
    f[rng.uniform(size=L) < 0.2] = 0.0
    V = (rng.uniform(size=L) > 0.3).astype(np.float64)
    vhat = np.maximum(rng.uniform(size=len(sizes)), 1e-3)
    perm = rng.permutation(L)
    members_of, o = [], 0
    for s in sizes:
        members_of.append(list(perm[o:o + s]))
        o += s
    return f, V, vhat, members_of


@pytest.mark.parametrize("n_cand", [1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_two_step_estimator_is_unbiased_exactly(n_cand, seed):
    f, V, vhat, members_of = _tiny_case(seed, [2, 3, 1, 3])
    E = clustered.expected_estimate(f, V, vhat, [len(m) for m in members_of], members_of, n_cand)
    assert abs(E - (f * V).sum()) <= 1e-12 * max(1.0, (f * V).sum())


def _point_scene(n_copies):
    rng = np.random.default_rng(7)
    lights = _lights(rng, 9)
    pos = np.tile(np.array([[4.0, 1.0, 5.0]], np.float32), (n_copies, 1))
    nrm = np.tile(np.array([[0.0, 1.0, 0.0]], np.float32), (n_copies, 1))
    off = np.array([0, 2, 2, 6, 9])
    mem = np.array([3, 7, 0, 1, 5, 8, 2, 4, 6])
    vis = np.tile(np.array([[0.9, 0.5, 0.2, 0.0]], np.float32), (n_copies, 1))
    return lights, pos, nrm, off, mem, vis


def test_sample_with_one_candidate_draws_p_and_weights_one_over_p():
    n = 200000
    lights, pos, nrm, off, mem, vis = _point_scene(n)
    out = clustered.sample(vis, pos, nrm, lights, off, mem, seed=5, frame=1, n_cand=1, dtype=np.float32)
    sizes = clustered.cluster_sizes(off)
    w = sizes * np.maximum(vis[0].astype(np.float64), 1e-3)
    P = w / w.sum()
    px = np.zeros(9)
    for j in range(4):
        for l in mem[off[j]:off[j + 1]]:
            px[l] = P[j] / sizes[j]
    f = lighting.unshadowed_weight(pos[:1], nrm[:1], lights)[0]
    ok = out["idx"] >= 0
    assert np.all(ok == (f[np.maximum(out["idx"], 0)] > 0) | ~ok)
    # frequencies of the lights that can be kept (f > 0), chi-square against p(x) renormalised
    keep = f > 0
    cnt = np.bincount(out["idx"][ok], minlength=9)[keep]
    exp_p = px[keep] / px[keep].sum() * ok.sum()
    chi2 = ((cnt - exp_p) ** 2 / exp_p).sum()
    assert chi2 < 30.0                                               # <= 8 dof, p < 1e-3
    # W = m_y / P(y) = 1 / p(x) (FP32, a few ulps)
    sel = out["idx"][ok]
    assert np.allclose(out["W"][ok], 1.0 / px[sel], rtol=5e-7)


@pytest.mark.parametrize("n_cand", [2, 8])
def test_sample_mean_matches_the_exact_sum(n_cand):
    n = 400000
    lights, pos, nrm, off, mem, vis = _point_scene(n)
    V = np.array([1, 0, 1, 1, 0, 1, 1, 0, 1], np.float64)
    out = clustered.sample(vis, pos, nrm, lights, off, mem, seed=9, frame=4, n_cand=n_cand, dtype=np.float64)
    f = lighting.unshadowed_weight(pos[:1], nrm[:1], lights)[0]
    est = np.where(out["idx"] >= 0, f[np.maximum(out["idx"], 0)] * V[np.maximum(out["idx"], 0)] * out["W"], 0.0)
    mu = (f * V).sum()
    se = est.std() / np.sqrt(n)
    assert abs(est.mean() - mu) <= 4.5 * se


def test_reservoirs_are_consistent():
    """Both picks as reservoirs (Sec. 4.2): W = w_sum / (M f_y), and W * P(pick) = 1 for the plain pick."""
    rng = np.random.default_rng(4)
    n, m = 3000, 32
    f = rng.uniform(0.0, 2.0, (n, m)).astype(np.float32)
    f[:, ::5] = 0
    v = rng.uniform(0, 1, (n, m)).astype(np.float32)
    w = f * np.maximum(v, np.float32(1e-3))
    u = rng.uniform(0, 1, n).astype(np.float32)
    idx, pmf, W = lighting.wrs_pick(w, u)
    r = lighting.pick_reservoir(w, f, idx, W)
    ok = idx >= 0
    assert np.all(r["M"][ok] == 1) and np.all(r["y"][ok] == idx[ok])
    assert np.allclose(r["W"][ok] * pmf[ok], 1.0, rtol=3e-7)
    fy = f[ok, idx[ok]]
    assert np.allclose(r["w_sum"][ok] / fy, r["W"][ok], rtol=2e-7)
    lights, pos, nrm, off, mem, vis = _point_scene(5000)
    out = clustered.sample(vis, pos, nrm, lights, off, mem, seed=1, frame=2, n_cand=8, dtype=np.float32)
    ok = out["idx"] >= 0
    fx = lighting.unshadowed_weight(pos[:1], nrm[:1], lights)[0][out["idx"][ok]].astype(np.float32)
    assert np.allclose(out["w_sum"][ok] / (8 * fx), out["W"][ok], rtol=5e-7)
