"""One whole training step of the cache (Sec. 3.4) on the GPU against the oracle's composed step.

The step is the library's: training pixels (Philox draws), shadow labels,
the gradient pass, Adam on the table and on the master weights, and the
repack of the weights the inference kernel reads.  The oracle's
`pipeline.train_step` composes its own pinned steps.  Compared:
  * pixels and labels bit for bit (as multisets of (pixel, labels) rows);
  * every gradient entry within its element-wise rounding bound;
  * every parameter after Adam: the kernel's update against the first Adam
    step's closed form p - lr g / (|g| + eps) evaluated here in FP64 on the
    gradient the kernel used (1e-6 (1 + |p|)), and against the oracle's
    parameters, within that plus what the gradient's bound allows the first
    step to move (lr g / (|g| + eps) is monotone in g with slope
    lr eps / (|g| + eps)^2; a gradient whose interval holds zero may take the
    full step of either sign);
  * inference after the step, through the weights the step repacked, against
    a fresh pack of the same updated master weights (bit for bit).
The oracle only ever receives the workload's inputs: the GPU's pixels, labels,
gradients and parameters are compared with its results, never fed to it.
A ten-step trajectory on the tiny workload then checks that the two sides do
not drift apart: the loss of every step within 1e-5 relative, and the
visibility after ten steps within 1e-4.
"""
import numpy as np
import pytest
import torch

from oracle import bounds, pipeline
from tests.gpu_common import make_cache, params
from workloads import box_scene, get_workload, unit_cube_scene
from workloads.scenes import unflatten_weights

pytestmark = pytest.mark.gpu

DEV = "cuda"
ADAM_TOL = 1e-6


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


def _case(name):
    if name == "tiny":
        wl = get_workload("tiny")
        sc = unit_cube_scene(wl.scene_seed, wl.n_points, wl.n_lights, wl.n_spheres)
        return wl, sc, wl.train_batch
    wl = get_workload("frame_1080p", mlp_dtype=name.split("_")[1])
    sc = box_scene(0, 160, 90, 64, 32, 256)
    return wl, sc, 4096


def _first_step_move_bound(g_ref, e_g, lr, eps):
    """sup |lr x/(|x|+eps) - lr g/(|g|+eps)| over |x - g| <= e (Adam's first step from zero moments)."""
    a = np.abs(g_ref)
    d = a - e_g
    flip = d <= 0
    smooth = lr * e_g * eps / (np.maximum(d, 0) + eps) ** 2
    full = lr * (a / (a + eps) + e_g / (e_g + eps))
    return np.where(flip, full, smooth)


@pytest.mark.parametrize("name", ["tiny", "1080p_f32", "1080p_f16"])
def test_one_training_step_matches_the_oracle(name):
    wl, sc, batch = _case(name)
    p = params(wl)
    cache = make_cache(wl, p)
    pos_unit, pos = t(sc["pos_unit"]), t(sc["pos"])
    lights, spheres = t(sc["lights"]), t(sc["spheres"])
    print(f"one step {name}: batch {batch}, {sc['pos'].shape[0]} pixels", flush=True)
    bufs = cache.train_gradients(pos_unit, pos, lights, spheres, frame=0, batch=batch)
    g_t = cache.g_table.cpu().numpy().astype(np.float64)
    g_w = cache.g_w.cpu().numpy().astype(np.float64)
    loss = cache.loss_buf.item()
    cache.adam()
    new_t = cache.table.cpu().numpy().astype(np.float64)
    new_w = cache.w.cpu().numpy().astype(np.float64)

    ref = pipeline.train_step(sc["pos_unit"], sc["pos"], sc["lights"], sc["spheres"], p["table"], p["weights"],
                              wl.grid.base_res, wl.grid.growth, seed=wl.rng_key, frame=0, batch=batch, lr=wl.lr,
                              beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps, loss=wl.loss)
    # pixels and their labels, bit for bit (the library returns the multiset sorted)
    gpu_pix = bufs["pix"].cpu().numpy()
    order = np.argsort(ref["pix"], kind="stable")
    assert np.array_equal(gpu_pix, ref["pix"][order])
    gpu_lab = bufs["labels"].cpu().numpy()
    assert np.array_equal(gpu_lab, ref["labels"][order])
    assert abs(loss - ref["loss"]) <= (1e-5 if wl.mlp.dtype == "f32" else 3e-2) * abs(ref["loss"])

    # gradients entry by entry within their rounding bounds (on the oracle's own pixels and labels, equal to
    # the GPU's as checked above)
    b = bounds.gradient_error_bounds(sc["pos_unit"][ref["pix"]], p["table"], p["weights"], wl.grid.base_res,
                                     wl.grid.growth, labels=ref["labels"], loss=wl.loss, act=wl.mlp.act,
                                     slope=wl.mlp.leaky_slope, dtype=wl.mlp.dtype)
    ref_gw = np.concatenate([g.ravel() for g in ref["grads"]["g_w"]])
    e_gw = np.concatenate([e.ravel() for e in b["e_w"]])
    assert np.allclose(b["g_table"], ref["grads"]["g_table"], rtol=1e-10, atol=1e-12 * np.abs(b["g_table"]).max())
    for nm, got, r, e in (("g_table", g_t, ref["grads"]["g_table"], b["e_table"]), ("g_w", g_w, ref_gw, e_gw)):
        err = np.abs(got - r)
        print(f"  {nm}: max|err| {err.max():.3e}, largest err/bound {np.max(err / np.maximum(e, 1e-300)):.3f}")
        assert np.all(err <= e), nm

    # Adam: the kernel's arithmetic on the gradient it used (the first step's closed form: m^ = g, v^ = g^2),
    # then end to end against the oracle
    p0 = [p["table"].astype(np.float64).ravel(), np.concatenate([w.ravel() for w in p["weights"]]).astype(np.float64)]
    for nm, got, g, p_ref, r_g, e_g in (
            ("table", new_t.ravel(), g_t.ravel(), ref["table"].ravel(), ref["grads"]["g_table"].ravel(),
             b["e_table"].ravel()),
            ("weights", new_w, g_w, np.concatenate([w.ravel() for w in ref["weights"]]), ref_gw, e_gw)):
        base = p0[0] if nm == "table" else p0[1]
        own = base - wl.lr * g / (np.abs(g) + wl.adam_eps)
        tol = ADAM_TOL * (1 + np.abs(own))
        assert np.all(np.abs(got - own) <= tol), nm
        move = _first_step_move_bound(r_g, e_g, wl.lr, wl.adam_eps)
        err = np.abs(got - p_ref)
        flips = int(np.count_nonzero(err > tol + _first_step_move_bound(r_g, 0 * e_g, wl.lr, wl.adam_eps)))
        print(f"  {nm} after Adam: max|err| {err.max():.3e}; entries whose gradient bound allows a sign "
              f"change: {int(np.count_nonzero(np.abs(r_g) <= e_g))}, entries beyond the exact-gradient step: {flips}")
        assert np.all(err <= tol + move), nm

    # inference after the step reads the weights the step repacked: the same as a fresh pack of them
    probe = t(sc["pos_unit"][:: max(1, sc["pos_unit"].shape[0] // 2000)])
    vis = cache.infer(probe, dtype=torch.float32)
    fresh = make_cache(wl, {"table": new_t.astype(np.float32).reshape(p["table"].shape),
                            "weights": unflatten_weights(new_w.astype(np.float32), wl.mlp)})
    assert torch.equal(vis, fresh.infer(probe, dtype=torch.float32))


def test_ten_step_trajectory_stays_with_the_oracle():
    """Ten frames of training on the tiny workload (FP32), GPU against the oracle's FP64 trajectory."""
    wl, sc, batch = _case("tiny")
    p = params(wl)
    cache = make_cache(wl, p)
    pos_unit, pos = t(sc["pos_unit"]), t(sc["pos"])
    lights, spheres = t(sc["lights"]), t(sc["spheres"])
    state, cur_t, cur_w = None, p["table"], p["weights"]
    for f in range(10):
        cache.train_gradients(pos_unit, pos, lights, spheres, frame=f, batch=batch)
        loss = cache.loss_buf.item()
        cache.adam()
        out = pipeline.train_step(sc["pos_unit"], sc["pos"], sc["lights"], sc["spheres"], cur_t, cur_w,
                                  wl.grid.base_res, wl.grid.growth, seed=wl.rng_key, frame=f, batch=batch,
                                  adam_state=state, lr=wl.lr, beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps)
        state, cur_t, cur_w = out["adam"], out["table"], out["weights"]
        rel = abs(loss - out["loss"]) / abs(out["loss"])
        print(f"  frame {f}: loss gpu {loss:.7f} oracle {out['loss']:.7f} rel {rel:.2e}")
        assert rel <= 1e-5
    dt = np.abs(cache.table.cpu().numpy() - cur_t)
    dw = np.abs(cache.w.cpu().numpy() - np.concatenate([w.ravel() for w in cur_w]))
    print(f"  after 10 steps: table max|dp| {dt.max():.3e} (99.9% {np.quantile(dt, 0.999):.3e}), "
          f"weights max|dp| {dw.max():.3e}")
    vis = cache.infer(pos_unit, dtype=torch.float32).cpu().numpy()
    ref = pipeline.infer(sc["pos_unit"], cur_t, cur_w, wl.grid.base_res, wl.grid.growth)
    err = np.abs(vis - ref).max()
    print(f"  visibility after 10 steps: max|err| {err:.3e}")
    assert err <= 1e-4
