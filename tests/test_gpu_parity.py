"""Parity of the HIP path (through the C ABI) with the oracle, on seeded inputs.

Bars: bit-exact for integer work (grid cells via the encoding at vertices,
light picks, pixel picks, shadow labels) and for the FP32 quantities that
decide them (pmf, W); stated tolerances for floating point:
  encoding FP32           |err| <= 4e-6 * max|theta|   (3 roundings per weight, 8 fused terms)
  visibility FP32 path    |err| <= 2e-5
  visibility FP16 path    |err| <= 2e-3 (vs FP64 oracle and vs the GPU FP32 path)
  visibility BF16 path    |err| <= 3e-2 (reported, 8-bit mantissa)
  gradients FP32 path     relative L2 <= 1e-4
  gradients FP16 path     relative L2 <= 3e-2, BF16 <= 1e-1
  Adam                    |err| <= 1e-6 * (1 + |p|)
"""
import numpy as np
import pytest
import torch

from oracle import hashgrid, lighting, mlp as omlp, philox, pipeline, shadow, training
from tests.gpu_common import make_cache, p1080, params, rand_pos, tiny
from workloads import box_scene, get_workload, unit_cube_scene
from workloads.scenes import random_visibility

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


@pytest.fixture(scope="module")
def small_scene():
    # 1080p-style box room rendered at 160x90: same geometry class, cheap oracle.
    return box_scene(0, 160, 90, 64, 32, 256)


# ----------------------------------------------------------------- encoding
@pytest.mark.parametrize("wl_name", ["tiny", "frame_1080p"])
def test_encode_matches_oracle(wl_name):
    wl = get_workload(wl_name)
    p = params(wl)
    cache = make_cache(wl, p)
    pos = rand_pos(11, 3001)
    enc = cache.encode(t(pos)).cpu().numpy().astype(np.float64)
    ref = hashgrid.encode(pos, p["table"], wl.grid.base_res, wl.grid.growth)
    tol = 4e-6 * np.abs(p["table"]).max()
    err = np.abs(enc - ref)
    assert err.max() <= tol, f"max err {err.max():.3e} > {tol:.3e}"
    # at levels where the worked point (0.5, 0.25, 0.75) scales to a grid vertex the
    # encoding is the stored feature itself, bit for bit
    res = hashgrid.level_resolutions(wl.grid.base_res, wl.grid.growth, wl.grid.n_levels)
    F = wl.grid.n_feat
    vertex_levels = [l for l, r in enumerate(res) if all(float(c * r).is_integer() for c in (0.5, 0.25, 0.75))]
    assert vertex_levels and vertex_levels[0] == 0
    for l in vertex_levels:
        assert np.array_equal(enc[2, l * F:(l + 1) * F], ref[2, l * F:(l + 1) * F]), l


def test_encode_low_precision_outputs_round_the_fp32_encoding():
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p)
    pos = t(rand_pos(12, 777))
    e32 = cache.encode(pos, torch.float32)
    for dt in (torch.float16, torch.bfloat16):
        e = cache.encode(pos, dt)
        assert torch.equal(e, e32.to(dt))


# ----------------------------------------------------------------- inference
INFER_CASES = [
    ("tiny", "f32", 2e-5), ("tiny", "f16", 2e-3), ("tiny", "bf16", 3e-2),
    ("frame_1080p", "f32", 2e-5), ("frame_1080p", "f16", 2e-3), ("frame_1080p", "bf16", 3e-2),
    ("sweep_4k", "f32", 2e-5), ("sweep_4k", "f16", 2e-3), ("sweep_4k", "bf16", 3e-2),
    ("paper_1080p", "f32", 2e-5), ("paper_1080p", "f16", 2e-3), ("paper_1080p", "bf16", 3e-2),
    ("clustered_1080p", "f32", 2e-5), ("clustered_1080p", "f16", 2e-3), ("clustered_1080p", "bf16", 3e-2),
]


@pytest.mark.parametrize("wl_name,dtype,tol", INFER_CASES)
def test_infer_matches_oracle(wl_name, dtype, tol):
    wl = get_workload(wl_name)
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    pos = rand_pos(13, 2085)                           # several tiles and a ragged tail
    vis = cache.infer(t(pos), dtype=torch.float32).cpu().numpy()
    ref = pipeline.infer(pos, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, act=wl.mlp.act,
                         slope=wl.mlp.leaky_slope)
    err = np.abs(vis - ref)
    print(f"{wl_name} {dtype}: max|err| {err.max():.3e} mean {err.mean():.3e}")
    assert err.max() <= tol


def test_infer_f16_vs_f32_gpu_path():
    wl = p1080()
    p = params(wl)
    pos = t(rand_pos(14, 4099))
    v32 = make_cache(wl, p, dtype="f32").infer(pos, dtype=torch.float32)
    v16 = make_cache(wl, p, dtype="f16").infer(pos, dtype=torch.float32)
    err = (v16 - v32).abs().max().item()
    print(f"f16 vs f32 path: max|err| {err:.3e}")
    assert err <= 2e-3


def test_infer_paper_network_leaky_f4():
    """The paper's own network (Sec. 3.3): ten levels of four features, two hidden layers of 32, leaky ReLU."""
    from workloads import GridCfg, MlpCfg, init_params
    grid = GridCfg(n_levels=10, n_feat=4, log2_T=14, base_res=16, growth=1.5)
    for dt, tol in (("f32", 2e-5), ("f16", 2e-3)):
        m = MlpCfg(n_in=40, width=32, n_hidden=2, n_out=32, act="leaky", leaky_slope=0.01, dtype=dt)
        p = init_params(1, grid, m, table_scale=1.0, weight_gain=2.0, init="he")
        from paper_2506_05930_amd.cache import NVCache
        cache = NVCache(grid, m, p["table"], p["weights"], device=DEV)
        pos = rand_pos(15, 1000)
        vis = cache.infer(t(pos), dtype=torch.float32).cpu().numpy()
        ref = pipeline.infer(pos, p["table"], p["weights"], 16, 1.5, act="leaky", slope=0.01)
        assert np.abs(vis - ref).max() <= tol, dt


def test_infer_outputs_in_every_dtype_agree():
    wl = p1080()
    cache = make_cache(wl, params(wl), dtype="f16")
    pos = t(rand_pos(16, 1234))
    v32 = cache.infer(pos, dtype=torch.float32)
    for dt in (torch.float16, torch.bfloat16):
        assert torch.equal(cache.infer(pos, dtype=dt), v32.to(dt))


@pytest.mark.parametrize("wl_name,dtype", [(w, d) for w in ("tiny", "frame_1080p", "sweep_4k") for d in ("f32", "f16", "bf16")]
                         + [("paper", "f16"), ("paper", "bf16"), ("paper", "f32"), ("paper_1080p", "f16")])
def test_mlp_forward_on_encoding_equals_fused_inference(wl_name, dtype):
    """nvc_mlp_forward(nvc_encode(x)) reproduces nvc_infer(x) bit for bit, with the encoding stored
    in the network's dtype and in FP32 (both round to the same matrix-core inputs)."""
    from paper_2506_05930_amd import api
    if wl_name == "paper":                     # ten levels of four features, leaky ReLU (Sec. 3.3)
        from paper_2506_05930_amd.cache import NVCache
        from workloads import GridCfg, MlpCfg, init_params
        grid = GridCfg(n_levels=10, n_feat=4, log2_T=14, base_res=16, growth=1.5)
        m = MlpCfg(n_in=40, width=32, n_hidden=2, n_out=32, act="leaky", leaky_slope=0.01, dtype=dtype)
        p = init_params(1, grid, m, table_scale=1.0, weight_gain=2.0, init="he")
        cache = NVCache(grid, m, p["table"], p["weights"], device=DEV)
    else:
        wl = get_workload(wl_name)
        cache = make_cache(wl, params(wl), dtype=dtype)
    pos = t(rand_pos(17, 2085))
    ref = cache.infer(pos, dtype=torch.float32)
    for enc_dt in {api.torch_dtype(cache.mlp.dtype), torch.float32}:
        enc = cache.encode(pos, dtype=enc_dt)
        out = torch.empty_like(ref)
        api.nvc_mlp_forward(cache.mlp, cache.packed, enc, out)
        assert torch.equal(out, ref), (wl_name, dtype, enc_dt)


@pytest.mark.parametrize("wl_name,dtype,n", [("frame_1080p", "f16", 2085), ("frame_1080p", "bf16", 1000003),
                                             ("sweep_4k", "f16", 2085), ("sweep_4k", "f16", 200003),
                                             ("sweep_4k", "bf16", 200003), ("paper_1080p", "f16", 100003),
                                             ("tiny", "f16", 2085)])
def test_mlp_forward_16bit_output_equals_fused_inference(wl_name, dtype, n):
    """nvc_mlp_forward with the visibilities in the network's 16-bit dtype, from the encoding stored in that
    dtype (the branch-free kernel whose stores go through a per-tile buffer resource, the lanes past the last
    point dropped by its range check) and in FP32 (the general kernel), equals nvc_infer's 16-bit output bit
    for bit; n leaves a ragged last tile, and the larger n give every wave several tiles.  The rows of the
    output next to the buffer (a guard row on each side) stay untouched."""
    from paper_2506_05930_amd import api
    wl = get_workload(wl_name)
    cache = make_cache(wl, params(wl), dtype=dtype)
    tdt = api.torch_dtype(cache.mlp.dtype)
    pos = t(rand_pos(18, n))
    ref = cache.infer(pos, dtype=tdt)
    m = ref.shape[1]
    for enc_dt in (tdt, torch.float32):
        enc = cache.encode(pos, dtype=enc_dt)
        guard = torch.full((n + 2, m), 7.0, dtype=tdt, device=DEV)
        out = guard[1:n + 1]
        api.nvc_mlp_forward(cache.mlp, cache.packed, enc, out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (wl_name, dtype, n, enc_dt)
        assert torch.all(guard[0] == 7.0) and torch.all(guard[n + 1] == 7.0), (wl_name, dtype, n, enc_dt)


@pytest.mark.parametrize("wl_name,dtype", [("frame_1080p", "f16"), ("sweep_4k", "bf16")])
def test_mlp_forward_16bit_output_edge_cases(wl_name, dtype):
    """The 16-bit encoding-input kernel at sizes below and around one tile (1, 31, 33 points: the buffer
    resource of the only tile is clipped to the rows that exist) and with outputs the kernel cannot take
    (a row offset by one element, which breaks the 16-byte alignment, and an FP32 output): every case equals
    nvc_infer's output for the same points bit for bit, and nothing is written outside the output rows."""
    from paper_2506_05930_amd import api
    wl = get_workload(wl_name)
    cache = make_cache(wl, params(wl), dtype=dtype)
    tdt = api.torch_dtype(cache.mlp.dtype)
    m = cache.mlp.n_out
    for n in (1, 31, 33):
        pos = t(rand_pos(19 + n, n))
        enc = cache.encode(pos, dtype=tdt)
        ref = cache.infer(pos, dtype=tdt)
        guard = torch.full((n + 2, m), 7.0, dtype=tdt, device=DEV)
        api.nvc_mlp_forward(cache.mlp, cache.packed, enc, guard[1:n + 1])
        torch.cuda.synchronize()
        assert torch.equal(guard[1:n + 1], ref), (wl_name, n)
        assert torch.all(guard[0] == 7.0) and torch.all(guard[n + 1] == 7.0), (wl_name, n)
    n = 4099
    pos = t(rand_pos(23, n))
    enc = cache.encode(pos, dtype=tdt)
    ref = cache.infer(pos, dtype=tdt)
    flat = torch.full((n * m + 2,), 7.0, dtype=tdt, device=DEV)
    out = flat[1:n * m + 1].view(n, m)                     # 2-byte offset: not 16-byte aligned
    api.nvc_mlp_forward(cache.mlp, cache.packed, enc, out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    assert flat[0].item() == 7.0 and flat[-1].item() == 7.0
    out32 = torch.empty((n, m), dtype=torch.float32, device=DEV)
    api.nvc_mlp_forward(cache.mlp, cache.packed, enc, out32)
    assert torch.equal(out32, cache.infer(pos, dtype=torch.float32))


# ----------------------------------------------------------------- WRS
@pytest.mark.parametrize("m,with_n,floor", [(8, False, 1e-3), (32, True, 1e-3), (32, True, 0.0), (128, True, 1e-3),
                                            (20, True, 1e-3)])
def test_wrs_bit_exact_against_fp32_oracle(small_scene, m, with_n, floor):
    sc = small_scene
    n = sc["pos"].shape[0]
    rng = np.random.default_rng(m)
    lights = np.concatenate([rng.uniform(0.5, 9.5, (m, 3)), rng.uniform(0.5, 2, (m, 1))], 1).astype(np.float32)
    vis = random_visibility(17 + m, n, m, np.float16)
    nrm = sc["nrm"] if with_n else None
    out = {k: torch.empty(n, dtype=d, device=DEV) for k, d in
           (("idx", torch.int32), ("pmf", torch.float32), ("wsum", torch.float32), ("di", torch.float32))}
    from paper_2506_05930_amd import api
    api.nvc_sample_wrs(t(vis), t(sc["pos"]), None if nrm is None else t(nrm), t(lights), floor, 2, 5,
                       out["idx"], out["pmf"], out["wsum"], out["di"])
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = pipeline.sample(vis, sc["pos"], nrm, lights, seed=2, frame=5, floor=floor)
    assert np.array_equal(got["idx"], ref["idx"])
    assert np.array_equal(got["wsum"], ref["wsum"])
    assert np.array_equal(got["pmf"], ref["pmf"])
    assert np.allclose(got["di"], ref["di"], rtol=2e-5, atol=1e-6 * np.abs(ref["di"]).max())
    if floor == 0.0:
        # biased variant: occluded-by-prediction lights (v = 0) are never picked
        sel = got["idx"] >= 0
        assert np.all(vis[np.nonzero(sel)[0], got["idx"][sel]] > 0)


def test_wrs_dyadic_weights_distribution():
    """All pixels at the origin, lights at unit distance with intensity k/64, v = 1: weights are
    exactly k/64, so every pick is decided exactly; counts follow w_i / W (chi-square)."""
    from scipy import stats

    from paper_2506_05930_amd import api
    k = np.array([5, 0, 17, 9, 1, 30, 2, 0], np.float64)
    dirs = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 0, 0], [0, 1, 0]],
                    np.float64)
    lights = np.concatenate([dirs, (k / 64.0)[:, None]], 1).astype(np.float32)
    n = 1 << 20
    pos = np.zeros((n, 3), np.float32)
    vis = np.ones((n, 8), np.float32)
    idx = torch.empty(n, dtype=torch.int32, device=DEV)
    pmf = torch.empty(n, dtype=torch.float32, device=DEV)
    W = torch.empty(n, dtype=torch.float32, device=DEV)
    api.nvc_sample_wrs(t(vis), t(pos), None, t(lights), 1e-3, 7, 0, idx, pmf, W)
    idx = idx.cpu().numpy()
    u = philox.wrs_uniforms(7, 0, n)
    ref_idx, ref_pmf, _ = lighting.wrs_pick(np.tile((k / 64.0).astype(np.float32), (n, 1)), u)
    assert np.array_equal(idx, ref_idx)
    assert np.array_equal(pmf.cpu().numpy(), ref_pmf)
    counts = np.bincount(idx, minlength=8)
    p = k / k.sum()
    assert counts[p == 0].sum() == 0
    assert stats.chisquare(counts[p > 0], n * p[p > 0]).pvalue > 1e-3


def test_wrs_lights_with_zero_weight():
    """Lights a pixel cannot see weigh exactly zero: in its surface plane (n.d = 0), on the pixel itself
    (d^2 clamped), behind the surface, or of zero intensity; mixed with ordinary lights, on a floor whose
    waves see some lights from every pixel and others from none.  Bit for bit against the oracle."""
    from paper_2506_05930_amd import api
    n = 4096 + 17
    rng = np.random.default_rng(31)
    pos = np.zeros((n, 3), np.float32)
    pos[:, 0] = rng.uniform(0, 8, n)
    pos[:, 2] = rng.uniform(0, 8, n)
    pos[: n // 2] = np.round(pos[: n // 2] * 4) / 4          # repeated positions on a grid
    nrm = np.tile(np.array([[0, 1, 0]], np.float32), (n, 1))
    lights = np.array([[2, 0, 3, 1.0],                        # in the floor plane: n.d = 0 everywhere
                       [pos[5, 0], 0, pos[5, 2], 2.0],        # on a pixel
                       [4, -2, 4, 1.5],                       # below the floor
                       [3, 2, 3, 0.0],                        # zero intensity
                       [1, 3, 1, 1.0], [6, 1.5, 2, 0.7], [4, 5, 7, 1.2], [7, 0.5, 7, 0.9]], np.float32)
    vis = random_visibility(5, n, 8, np.float16)
    out = {k: torch.empty(n, dtype=d, device=DEV) for k, d in
           (("idx", torch.int32), ("pmf", torch.float32), ("wsum", torch.float32), ("di", torch.float32))}
    api.nvc_sample_wrs(t(vis), t(pos), t(nrm), t(lights), 1e-3, 2, 5, out["idx"], out["pmf"], out["wsum"],
                       out["di"])
    got = {k: v.cpu().numpy() for k, v in out.items()}
    ref = pipeline.sample(vis, pos, nrm, lights, seed=2, frame=5, floor=1e-3)
    assert np.array_equal(got["idx"], ref["idx"])
    assert np.array_equal(got["wsum"], ref["wsum"])
    assert np.array_equal(got["pmf"], ref["pmf"])
    assert np.allclose(got["di"], ref["di"], rtol=2e-5, atol=1e-6 * np.abs(ref["di"]).max())
    assert not np.isin(got["idx"], [0, 1, 2, 3]).any()      # zero-weight lights are never picked


def test_wrs_all_lights_behind_surface():
    from paper_2506_05930_amd import api
    pos = np.zeros((3, 3), np.float32)
    nrm = np.tile(np.array([[0, 1, 0]], np.float32), (3, 1))
    lights = np.array([[0, -1, 0, 1], [1, -1, 0, 1]], np.float32)
    out = [torch.empty(3, dtype=d, device=DEV) for d in (torch.int32, torch.float32, torch.float32, torch.float32)]
    api.nvc_sample_wrs(t(np.ones((3, 2), np.float16)), t(pos), t(nrm), t(lights), 1e-3, 1, 0, *out)
    assert out[0].cpu().tolist() == [-1, -1, -1]
    assert out[1].cpu().tolist() == [0, 0, 0] and out[2].cpu().tolist() == [0, 0, 0]


# ----------------------------------------------------------------- training inputs
def test_select_pixels_bit_exact():
    """The batch is the oracle's multiset of Philox pixel draws, returned sorted."""
    from paper_2506_05930_amd import api
    for n_pix, batch, frame in ((1920 * 1080, 1 << 18, 3), (1000, 5000, 0), (1, 7, 9), (4097, 300, 1)):
        pix = torch.empty(batch, dtype=torch.int32, device=DEV)
        ws = torch.empty(api.nvc_select_pixels_workspace_bytes(n_pix), dtype=torch.uint8, device=DEV)
        ws.fill_(0xAB)                             # stale contents must not matter
        api.nvc_select_pixels(2, frame, n_pix, pix, ws)
        assert np.array_equal(pix.cpu().numpy(), np.sort(philox.training_pixels(2, frame, batch, n_pix)))


@pytest.mark.parametrize("m", [8, 32, 128, 13])
def test_shadow_labels_bit_exact(small_scene, m):
    from paper_2506_05930_amd import api
    sc = small_scene
    rng = np.random.default_rng(m)
    lights = np.concatenate([rng.uniform(0.5, 9.5, (m, 3)), rng.uniform(0.5, 2, (m, 1))], 1).astype(np.float32)
    n_pix = sc["pos"].shape[0]
    batch = 3001
    pix = philox.training_pixels(2, 1, batch, n_pix).astype(np.int32)
    if m != 13:
        pix = np.sort(pix)                      # grouped samples: sphere culling active
    lab = torch.empty((batch, m), dtype=torch.uint8, device=DEV)
    api.nvc_shadow_labels(t(sc["pos"]), t(pix), t(lights), t(sc["spheres"]), lab)
    ref = shadow.labels_fp32(sc["pos"][pix], lights, sc["spheres"])
    got = lab.cpu().numpy()
    assert np.array_equal(got, ref)
    assert 0.05 < got.mean() < 0.999


@pytest.mark.parametrize("batch,m", [(8192, 32), (1 << 18, 32), (1 << 17, 13)])
def test_shadow_labels_large_batches_sampled(small_scene, batch, m):
    """Batches large enough for eight lights per block (and the small-batch split of the lights over more
    blocks at 8192): every label of a random subset of samples against the oracle."""
    from paper_2506_05930_amd import api
    sc = small_scene
    rng = np.random.default_rng(100 + m)
    lights = np.concatenate([rng.uniform(0.5, 9.5, (m, 3)), rng.uniform(0.5, 2, (m, 1))], 1).astype(np.float32)
    pix = np.sort(philox.training_pixels(2, 3, batch, sc["pos"].shape[0]).astype(np.int32))
    lab = torch.empty((batch, m), dtype=torch.uint8, device=DEV)
    api.nvc_shadow_labels(t(sc["pos"]), t(pix), t(lights), t(sc["spheres"]), lab)
    sub = rng.choice(batch, 2048, replace=False)
    ref = shadow.labels_fp32(sc["pos"][pix[sub]], lights, sc["spheres"])
    assert np.array_equal(lab.cpu().numpy()[sub], ref)


@pytest.mark.parametrize("n_spheres", [1, 63, 1024, 1025, 4096])
def test_shadow_labels_sphere_counts(n_spheres):
    """Up to 1024 spheres the block shares its exact tests through a survivor list in LDS; above, each wave
    tests its own survivors.  Both against the oracle, on a batch with a ragged last block."""
    from paper_2506_05930_amd import api
    sc = box_scene(0, 160, 90, 64, 8, n_spheres)
    batch = 2 * 1024 + 333
    pix = np.sort(philox.training_pixels(2, 5, batch, sc["pos"].shape[0]).astype(np.int32))
    lab = torch.empty((batch, 8), dtype=torch.uint8, device=DEV)
    api.nvc_shadow_labels(t(sc["pos"]), t(pix), t(sc["lights"]), t(sc["spheres"]), lab)
    ref = shadow.labels_fp32(sc["pos"][pix], sc["lights"], sc["spheres"])
    assert np.array_equal(lab.cpu().numpy(), ref)


def test_shadow_labels_unit_cube_without_indirection():
    from paper_2506_05930_amd import api
    sc = unit_cube_scene(0, 4096, 8, 16, n_train=1024)
    lab = torch.empty((1024, 8), dtype=torch.uint8, device=DEV)
    api.nvc_shadow_labels(t(sc["train_pos"]), None, t(sc["lights"]), t(sc["spheres"]), lab)
    assert np.array_equal(lab.cpu().numpy(), shadow.labels_fp32(sc["train_pos"], sc["lights"], sc["spheres"]))
    # no spheres: everything visible
    api.nvc_shadow_labels(t(sc["train_pos"]), None, t(sc["lights"]), torch.empty((0, 4), device=DEV), lab)
    assert lab.min().item() == 1


# ----------------------------------------------------------------- gradients
def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))


GRAD_CASES = [("tiny", "f32", 1e-4, 1000), ("tiny", "f16", 3e-2, 1000), ("frame_1080p", "f32", 1e-4, 2085),
              ("frame_1080p", "f16", 3e-2, 2085), ("frame_1080p", "bf16", 1e-1, 2085),
              ("sweep_4k", "f32", 1e-4, 700), ("sweep_4k", "f16", 3e-2, 700), ("sweep_4k", "bf16", 1e-1, 700),
              ("paper_1080p", "f32", 1e-4, 1500), ("paper_1080p", "f16", 3e-2, 1500),
              ("paper_1080p", "bf16", 1e-1, 1500), ("clustered_1080p", "f32", 1e-4, 1700),
              ("clustered_1080p", "f16", 3e-2, 1700)]


@pytest.mark.parametrize("wl_name,dtype,tol,batch", GRAD_CASES)
@pytest.mark.parametrize("loss", ["bce", "l2"])
def test_train_gradients_match_oracle(wl_name, dtype, tol, batch, loss):
    wl = get_workload(wl_name, loss=loss)
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    pos = rand_pos(21, batch)
    rng = np.random.default_rng(22)
    y = (rng.uniform(size=(batch, wl.mlp.n_out)) > 0.4).astype(np.uint8)
    cache.gradients(t(pos), labels=t(y))
    ref = training.train_gradients(pos, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, labels=y,
                                   loss=loss, act=wl.mlp.act, slope=wl.mlp.leaky_slope)
    g_w = cache.g_w.cpu().numpy()
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    g_t = cache.g_table.cpu().numpy()
    e_w, e_t = _rel_l2(g_w, ref_w), _rel_l2(g_t, ref["g_table"])
    e_l = abs(cache.loss_buf.item() - ref["loss"]) / abs(ref["loss"])
    print(f"{wl_name} {dtype} {loss}: relL2 g_w {e_w:.2e} g_table {e_t:.2e} loss {e_l:.2e}")
    assert e_w <= tol and e_t <= tol and e_l <= max(tol, 1e-5)
    # untouched table entries stay exactly zero
    assert np.all(g_t[ref["g_table"] == 0] == 0)


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 3e-2)])
def test_train_gradients_2pow14_samples(dtype, tol):
    """The 1080p network's gradient pass on 2^14 samples (many samples per table partition; 256 block
    iterations of 64 samples, at most one per resident training block) against the oracle.  The production
    batch, with several persistent iterations per block, is in test_gpu_fullsize.py."""
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    n = 1 << 14
    pos = rand_pos(31, n)
    y = (np.random.default_rng(32).uniform(size=(n, wl.mlp.n_out)) > 0.4).astype(np.uint8)
    cache.gradients(t(pos), labels=t(y))
    ref = training.train_gradients(pos, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, labels=y)
    e_w = _rel_l2(cache.g_w.cpu().numpy(), np.concatenate([g.ravel() for g in ref["g_w"]]))
    e_t = _rel_l2(cache.g_table.cpu().numpy(), ref["g_table"])
    print(f"2^14 samples {dtype}: relL2 g_w {e_w:.2e} g_table {e_t:.2e}")
    assert e_w <= tol and e_t <= tol
    assert abs(cache.loss_buf.item() - ref["loss"]) <= max(tol, 1e-5) * abs(ref["loss"])


def test_gradients_accumulate_and_indirection():
    wl = tiny()
    p = params(wl)
    cache = make_cache(wl, p)
    pos = rand_pos(23, 600)
    pix = np.random.default_rng(24).integers(0, 600, 300).astype(np.int32)
    y = (np.random.default_rng(25).uniform(size=(300, 8)) > 0.5).astype(np.uint8)
    cache.gradients(t(pos), labels=t(y), pix=t(pix))
    cache.gradients(t(pos), labels=t(y), pix=t(pix))
    ref = training.train_gradients(pos[pix], p["table"], p["weights"], 16, 1.5, labels=y)
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    assert _rel_l2(cache.g_w.cpu().numpy(), 2 * ref_w) <= 1e-4
    assert _rel_l2(cache.g_table.cpu().numpy(), 2 * ref["g_table"]) <= 1e-4


# A random upstream gradient makes the weight gradient a sum of terms of random
# sign, so its FP16 relative error is larger than with loss gradients (5e-2).
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 5e-2)])
def test_autograd_function_backward(dtype, tol):
    from paper_2506_05930_amd.cache import NVCFunction
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    pos = rand_pos(26, 1500)
    table = cache.table.clone().requires_grad_(True)
    w = cache.w.clone().requires_grad_(True)
    dvis = np.random.default_rng(27).normal(size=(1500, 32)).astype(np.float32) * 1e-3
    # loss scaling: bring the upstream gradient to O(1) before the low-precision backward
    vis = NVCFunction.apply(t(pos), table, w, cache, float(1.0 / np.sqrt(np.mean(dvis ** 2))))
    vis.backward(t(dvis))
    ref = training.train_gradients(pos, p["table"], p["weights"], 16, 1.447, dvis=dvis)
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    assert _rel_l2(w.grad.cpu().numpy(), ref_w) <= tol
    assert _rel_l2(table.grad.cpu().numpy(), ref["g_table"]) <= tol


def test_adam_matches_oracle():
    from paper_2506_05930_amd import api
    rng = np.random.default_rng(28)
    n = 100003                                  # not a multiple of 4: vector body + scalar tail
    p0, g0 = rng.normal(size=n).astype(np.float32), (rng.normal(size=n) * 1e-2).astype(np.float32)
    g0[::5] = 0
    m0, v0 = (rng.normal(size=n) * 1e-3).astype(np.float32), (rng.uniform(size=n) * 1e-4).astype(np.float32)
    P, G, M, V = t(p0), t(g0), t(m0), t(v0)
    api.nvc_adam(P, G, M, V, 3, 1e-2, 0.9, 0.99, 1e-8, zero_grad=True)
    rp, rm, rv = training.adam_step(p0, g0, m0, v0, 3, 1e-2, 0.9, 0.99, 1e-8)
    assert np.abs(P.cpu().numpy() - rp).max() <= 1e-6 * (1 + np.abs(rp).max())
    assert np.abs(M.cpu().numpy() - rm).max() <= 1e-7
    assert np.abs(V.cpu().numpy() - rv).max() <= 1e-9
    assert G.abs().max().item() == 0.0


@pytest.mark.parametrize("step", [1, 2, 57, 200, 201, 350])
def test_adam_learning_rate_schedule_matches_oracle(step):
    """nvc_adam with the linear decay of Sec. 3.4 (0.05 -> 0.001 over 200 steps), step from the host and from
    the device counter."""
    from paper_2506_05930_amd import api
    rng = np.random.default_rng(29)
    n = 4099
    p0, g0 = rng.normal(size=n).astype(np.float32), (rng.normal(size=n) * 1e-2).astype(np.float32)
    m0, v0 = (rng.normal(size=n) * 1e-3).astype(np.float32), (rng.uniform(size=n) * 1e-4).astype(np.float32)
    lr = training.learning_rate(step, 0.05, 0.001, 200)
    rp, rm, rv = training.adam_step(p0, g0, m0, v0, step, lr, 0.9, 0.99, 1e-8)
    for ctr in (None, api.new_counters(frame=0, step=step, device=DEV)):
        P, G, M, V = t(p0), t(g0), t(m0), t(v0)
        api.nvc_adam(P, G, M, V, step if ctr is None else 1, 0.05, 0.9, 0.99, 1e-8, ctr=ctr, lr_end=0.001,
                     lr_decay_steps=200)
        assert np.abs(P.cpu().numpy() - rp).max() <= 1e-6 * (1 + np.abs(rp).max())
        assert np.abs(M.cpu().numpy() - rm).max() <= 1e-7


def _straddling_points():
    """Vertices-centred points whose (dy, dz) = (0, 0) corner pair straddles a 4096-entry partition
    on the dense level of resolution 48 (1080p grid, level 3): e0 = cx + 49 cy + 49^2 cz = 4095 (mod 4096)."""
    pts = []
    for cz in range(0, 20):
        for cy in range(0, 48):
            cx = (4095 + 4096 * 8 - 49 * cy - 2401 * cz) % 4096
            if cx < 48 and (cx + 49 * cy + 2401 * cz) % 4096 == 4095:
                pts.append([(cx + 0.5) / 48, (cy + 0.5) / 48, (cz + 0.5) / 48])
    return np.array(pts, np.float32)


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 3e-2)])
def test_train_routed_scatter_edge_cases(dtype, tol):
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    strad = _straddling_points()
    assert len(strad) >= 5
    same = np.tile(np.array([[0.3, 0.6, 0.2]], np.float32), (300, 1))     # one cell: heavy bucket
    pos = np.concatenate([strad, same, rand_pos(31, 777)]).astype(np.float32)  # ragged batch
    y = (np.random.default_rng(32).uniform(size=(len(pos), 32)) > 0.5).astype(np.uint8)
    cache.gradients(t(pos), labels=t(y))
    ref = training.train_gradients(pos, p["table"], p["weights"], 16, 1.447, labels=y)
    assert _rel_l2(cache.g_table.cpu().numpy(), ref["g_table"]) <= tol
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    assert _rel_l2(cache.g_w.cpu().numpy(), ref_w) <= tol


def test_train_direct_atomic_fallback_for_fine_hashed_levels():
    """Growth 2.0 gives hashed levels finer than 2^14 cells per axis, which the routed scatter
    does not partition; the training step falls back to direct atomics and stays exact."""
    from dataclasses import replace

    from paper_2506_05930_amd.cache import NVCache
    wl = p1080()
    grid = replace(wl.grid, growth=2.0)
    p = params(wl)
    cache = NVCache(grid, replace(wl.mlp, dtype="f32"), p["table"], p["weights"], device=DEV)
    pos = rand_pos(33, 1000)
    y = (np.random.default_rng(34).uniform(size=(1000, 32)) > 0.5).astype(np.uint8)
    cache.gradients(t(pos), labels=t(y))
    ref = training.train_gradients(pos, p["table"], p["weights"], 16, 2.0, labels=y)
    assert _rel_l2(cache.g_table.cpu().numpy(), ref["g_table"]) <= 1e-4
