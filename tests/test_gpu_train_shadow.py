"""The training pass with its shadow labels computed inside the training kernel (Sec. 3.4).

nvc_train_step_shadow labels each training sample against every light with
the FP32 segment-sphere decision of the separate label kernel (the spheres
first culled against the bundle of the wave's 16 segments to each light), then
runs the labelled gradient pass on those labels.  Compared:
  * one training step on small scenes (tiny: 8 lights, 16 spheres, random
    points in the unit cube; the 1080p network on a 160x90 render of the
    1080p box scene: 32 lights, 256 spheres, FP32 and FP16), with batches that
    leave a ragged last tile, against the oracle's composed step: pixels and
    labels bit for bit, every gradient entry within its element-wise rounding
    bound, and the loss;
  * the production batch (2^18 seeded pixels of the 1920x1080 G-buffer, the
    frame's FP16 network): every label bit for bit against the oracle's FP32
    labels, every gradient entry within its element-wise rounding bound, the
    loss;
  * degenerate occluder sets against the oracle's labels: no spheres (every
    label 1), a sphere around a light, and a wave whose samples sit at one
    point (a bundle of zero width).
"""
import numpy as np
import pytest
import torch

from oracle import bounds, pipeline, shadow, training
from tests.gpu_common import make_cache, params
from workloads import box_scene, get_workload, unit_cube_scene

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


def _case(name):
    if name == "tiny":
        wl = get_workload("tiny")
        sc = unit_cube_scene(wl.scene_seed, wl.n_points, wl.n_lights, wl.n_spheres)
        return wl, sc, 1000                              # 15 tiles of 64 and a tail of 40
    wl = get_workload("frame_1080p", mlp_dtype=name.split("_")[1])
    sc = box_scene(0, 160, 90, 64, 32, 256)
    return wl, sc, 4096 + 37


@pytest.mark.parametrize("name", ["tiny", "1080p_f32", "1080p_f16"])
def test_fused_step_matches_the_oracle(name):
    wl, sc, batch = _case(name)
    p = params(wl)
    cache = make_cache(wl, p, fused_labels=True)
    print(f"fused-label step {name}: batch {batch}, {sc['pos'].shape[0]} pixels", flush=True)
    bufs = cache.train_gradients(t(sc["pos_unit"]), t(sc["pos"]), t(sc["lights"]), t(sc["spheres"]), frame=0,
                                 batch=batch)
    g_t = cache.g_table.cpu().numpy().astype(np.float64)
    g_w = cache.g_w.cpu().numpy().astype(np.float64)
    loss = cache.loss_buf.item()
    ref = pipeline.train_step(sc["pos_unit"], sc["pos"], sc["lights"], sc["spheres"], p["table"], p["weights"],
                              wl.grid.base_res, wl.grid.growth, seed=wl.rng_key, frame=0, batch=batch, lr=wl.lr,
                              beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps, loss=wl.loss)
    order = np.argsort(ref["pix"], kind="stable")
    assert np.array_equal(bufs["pix"].cpu().numpy(), ref["pix"][order])
    lab = bufs["labels"].cpu().numpy()
    assert np.array_equal(lab, ref["labels"][order])
    print(f"  labels: {lab.size} bit for bit, {lab.mean():.3f} visible")
    assert abs(loss - ref["loss"]) <= (1e-5 if wl.mlp.dtype == "f32" else 3e-2) * abs(ref["loss"])
    b = bounds.gradient_error_bounds(sc["pos_unit"][ref["pix"]], p["table"], p["weights"], wl.grid.base_res,
                                     wl.grid.growth, labels=ref["labels"], loss=wl.loss, act=wl.mlp.act,
                                     slope=wl.mlp.leaky_slope, dtype=wl.mlp.dtype)
    ref_gw = np.concatenate([g.ravel() for g in ref["grads"]["g_w"]])
    e_gw = np.concatenate([e.ravel() for e in b["e_w"]])
    for nm, got, r, e in (("g_table", g_t, ref["grads"]["g_table"], b["e_table"]), ("g_w", g_w, ref_gw, e_gw)):
        err = np.abs(got - r)
        print(f"  {nm}: max|err| {err.max():.3e}, largest err/bound {np.max(err / np.maximum(e, 1e-300)):.3f}")
        assert np.all(err <= e), nm


def test_fused_production_batch_against_oracle():
    """2^18 seeded pixels of the 1920x1080 G-buffer through the fused pass, in the frame's FP16 configuration."""
    wl = get_workload("train_1080p")
    sc = box_scene(wl.scene_seed, wl.width, wl.height, wl.n_boxes, wl.n_lights, wl.n_spheres)
    n, b = sc["pos"].shape[0], wl.train_batch
    pix = np.sort(np.random.default_rng(43).integers(0, n, b)).astype(np.int32)   # sorted, as the pixel pick
    p = params(wl)
    cache = make_cache(wl, p)
    print(f"fused production batch: {b} samples, {wl.n_lights} lights, {wl.n_spheres} spheres", flush=True)
    lab_t = torch.empty((b, wl.n_lights), dtype=torch.uint8, device=DEV)
    cache.gradients_shadow(t(sc["pos_unit"]), t(sc["pos"]), t(sc["lights"]), t(sc["spheres"]), pix=t(pix), batch=b,
                           labels_out=lab_t)
    lab = lab_t.cpu().numpy()
    y = shadow.labels_fp32(sc["pos"][pix], sc["lights"], sc["spheres"])
    assert np.array_equal(lab, y)
    print(f"  labels bit for bit with the oracle on every sample ({y.mean():.3f} visible)", flush=True)
    pos = sc["pos_unit"][pix]
    ref = bounds.gradient_error_bounds(pos, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, labels=y,
                                       dtype=wl.mlp.dtype)
    g_w = cache.g_w.cpu().numpy().astype(np.float64)
    g_t = cache.g_table.cpu().numpy().astype(np.float64)
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    e_w = np.concatenate([e.ravel() for e in ref["e_w"]])
    for nm, got, r, e in (("g_table", g_t, ref["g_table"], ref["e_table"]), ("g_w", g_w, ref_w, e_w)):
        err = np.abs(got - r)
        print(f"  {nm}: max|err| {err.max():.3e} (max|g| {np.abs(r).max():.3e}), "
              f"largest err/bound {np.max(err / np.maximum(e, 1e-300)):.3f}")
        assert np.all(err <= e), nm
    assert np.all(g_t[ref["g_table"] == 0] == 0)                   # untouched entries stay exactly zero
    full = training.train_gradients(pos, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, labels=y)
    loss = cache.loss_buf.item()
    print(f"  loss {loss:.7f} oracle {full['loss']:.7f}")
    assert abs(loss - full["loss"]) <= 3e-2 * abs(full["loss"])


def _labels_only(wl, pos_scene, lights, spheres):
    """Labels from the fused pass (gradients discarded), on the tiny network with one output per light."""
    p = params(wl)
    cache = make_cache(wl, p)
    n = pos_scene.shape[0]
    unit = np.clip(pos_scene / 10.0, 0, 1).astype(np.float32)
    lab = torch.empty((n, lights.shape[0]), dtype=torch.uint8, device=DEV)
    sph = torch.empty((0, 4), dtype=torch.float32, device=DEV) if spheres.shape[0] == 0 else t(spheres)
    cache.gradients_shadow(t(unit), t(pos_scene), t(lights), sph, batch=n, labels_out=lab)
    return lab.cpu().numpy()


def test_fused_labels_on_degenerate_occluders():
    wl = get_workload("tiny")                                       # 8 outputs: 8 lights
    rng = np.random.default_rng(45)
    pos = rng.uniform(0, 10, size=(777, 3)).astype(np.float32)
    lights = np.concatenate([rng.uniform(0, 10, size=(8, 3)), np.ones((8, 1))], 1).astype(np.float32)
    # no spheres: every ray reaches its light
    lab = _labels_only(wl, pos, lights, np.zeros((0, 4), np.float32))
    assert np.all(lab == 1)
    # a sphere around light 3 (radius 0.5), a sphere through the middle of the box, and small ones
    spheres = np.concatenate([np.r_[lights[3, :3], 0.5][None], [[5.0, 5.0, 5.0, 2.0]],
                              np.c_[rng.uniform(0, 10, size=(40, 3)), rng.uniform(0.1, 0.8, 40)]]).astype(np.float32)
    lab = _labels_only(wl, pos, lights, spheres)
    y = shadow.labels_fp32(pos, lights, spheres)
    assert np.array_equal(lab, y)
    outside = np.linalg.norm(pos - lights[3, :3], axis=1) > 0.5
    assert np.all(lab[outside, 3] == 0)
    # a wave's samples at one point (zero-width bundle), beside scattered ones
    pos1 = pos.copy()
    pos1[64:160] = pos1[64]
    lab = _labels_only(wl, pos1, lights, spheres)
    assert np.array_equal(lab, shadow.labels_fp32(pos1, lights, spheres))
