"""Precision of the 128-light, 128-wide network in FP32 / FP16 / BF16 (the 4K precision sweep).

Two trained versions of the 4K workload's network (32 -> 128 x3 -> 128, grid
T = 2^20, 128 lights), so that activations have a realistic range instead of
the near-constant 0.5 of a fresh network:

* trained for 200 steps on the FP32 path by the library; the same FP32 master
  parameters then run in each format on a fixed 65,536-point subset of a
  box-room render (the 4K scene class at 640x360) and are compared with the
  GPU's FP32 path (these parameters never reach the oracle: its inputs do not
  come from the HIP path);
* trained by the oracle itself (its composed FP64 training step, 20 steps of
  2048 samples on a 160x90 render), rounded to FP32 for both sides; each format
  is compared with the oracle's FP64 forward on the same subset, with the
  agreement of the light pick with the oracle's pick on the same uniforms and
  the error of the pick's pmf against the exact FP64 pmf of the same light.

The sweep is a report; its bounds are set to catch a broken format, not to
restate the 1080p target (FP16 within 2e-3 of the FP32 path, checked on the
64-wide network after training by test_gpu_trained_precision).  With four
128-wide layers and a trained network whose logits reach tens, FP16 rounding
of the inputs, weights and three hidden activations (unit roundoff 2^-11)
moves a logit by up to a few 1e-2 in the worst of 8.4M outputs, and the
sigmoid's slope (at most 1/4) turns that into a visibility error of about
1e-2; the mean error stays near 1e-4.  BF16 (unit roundoff 2^-8) is eight
times coarser.  Bounds: FP32 1e-4 max; FP16 2.5e-2 max and 2e-4 mean; BF16
0.2 max and 2e-3 mean; the FP32 pick agrees with the oracle's on more than
99.9% of the points, FP16 on more than 99%.  If NVC_REPORT_DIR is set the
report is also written there as JSON.
"""
import json
import os

import numpy as np
import pytest
import torch

from oracle import lighting, pipeline
from tests.gpu_common import make_cache
from workloads import box_scene, get_workload, init_params

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


def test_precision_sweep_128_lights():
    wl = get_workload("sweep_4k")
    sc = box_scene(0, 640, 360, wl.n_boxes, wl.n_lights, wl.n_spheres)
    n = sc["pos"].shape[0]
    from workloads.scenes import unflatten_weights
    sub = np.sort(np.random.default_rng(3).choice(n, 65536, replace=False))
    pu, ps, pn = sc["pos_unit"][sub], sc["pos"][sub], sc["nrm"][sub]
    lights = t(sc["lights"])

    # library-trained: formats against the GPU's FP32 path
    p = init_params(1, wl.grid, wl.mlp)
    c32 = make_cache(wl, p, dtype="f32")
    pos_unit, pos = t(sc["pos_unit"]), t(sc["pos"])
    spheres = t(sc["spheres"])
    for frame in range(200):
        c32.train_step(pos_unit, pos, lights, spheres, frame, 1 << 16)
    gpu_trained = {"table": c32.table.cpu().numpy(), "weights": unflatten_weights(c32.w.cpu().numpy(), wl.mlp)}
    report = {"subset": 65536, "library_trained": {"train_steps": 200, "loss_fp32_path": c32.loss_buf.item(),
                                                   "formats": {}},
              "oracle_trained": {"train_steps": 20, "batch": 2048, "formats": {}}}
    v_ref = c32.infer(t(pu)).float().cpu().numpy().astype(np.float64)
    for fmt in ("f16", "bf16"):
        v = make_cache(wl, gpu_trained, dtype=fmt).infer(t(pu)).float().cpu().numpy().astype(np.float64)
        e = np.abs(v - v_ref)
        report["library_trained"]["formats"][fmt] = {"vis_max_abs_err_vs_gpu_fp32": float(e.max()),
                                                     "vis_mean_abs_err_vs_gpu_fp32": float(e.mean())}

    # oracle-trained: formats against the FP64 oracle
    small = box_scene(0, 160, 90, wl.n_boxes, wl.n_lights, wl.n_spheres)
    state, tab, ws = None, p["table"], p["weights"]
    for f in range(20):
        out = pipeline.train_step(small["pos_unit"], small["pos"], small["lights"], small["spheres"], tab, ws,
                                  wl.grid.base_res, wl.grid.growth, seed=wl.rng_key, frame=f, batch=2048,
                                  adam_state=state, lr=wl.lr, beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps)
        state, tab, ws = out["adam"], out["table"], out["weights"]
    report["oracle_trained"]["loss"] = out["loss"]
    table, weights = tab.astype(np.float32), [w.astype(np.float32) for w in ws]
    v64 = pipeline.infer(pu, table, weights, wl.grid.base_res, wl.grid.growth)
    ref = pipeline.sample(v64, ps, pn, sc["lights"], wl.rng_key, 0, wl.vis_floor)
    p64 = ref["w64"] / ref["w64"].sum(axis=1, keepdims=True)
    v_fp32_gpu = None
    for fmt in ("f32", "f16", "bf16"):
        cache = make_cache(wl, {"table": table, "weights": weights}, dtype=fmt)
        vis = cache.infer(t(pu))                                   # the format's own output dtype
        v = vis.float().cpu().numpy().astype(np.float64)
        if fmt == "f32":
            v_fp32_gpu = v
        out = cache.sample(vis, t(ps), t(pn), lights, 0)
        idx = out["idx"].cpu().numpy()
        pmf = out["pmf"].cpu().numpy().astype(np.float64)
        safe = np.maximum(idx, 0)
        exact = np.take_along_axis(p64, safe[:, None], axis=1)[:, 0]
        e = np.abs(v - v64)
        report["oracle_trained"]["formats"][fmt] = {
            "vis_max_abs_err_vs_fp64": float(e.max()), "vis_mean_abs_err_vs_fp64": float(e.mean()),
            "vis_p999_abs_err_vs_fp64": float(np.quantile(e, 0.999)),
            "vis_max_abs_err_vs_gpu_fp32": float(np.abs(v - v_fp32_gpu).max()),
            "pick_agreement_vs_fp64": float((idx == ref["idx"]).mean()),
            "pmf_max_abs_err_vs_fp64": float(np.abs(pmf - exact)[idx >= 0].max()),
            "pmf_mean_abs_err_vs_fp64": float(np.abs(pmf - exact)[idx >= 0].mean()),
        }
    print(json.dumps(report, indent=1))
    if os.environ.get("NVC_REPORT_DIR"):
        with open(os.path.join(os.environ["NVC_REPORT_DIR"], "precision_sweep_128.json"), "w") as f:
            json.dump(report, f, indent=1)
    lt = report["library_trained"]["formats"]
    assert lt["f16"]["vis_max_abs_err_vs_gpu_fp32"] <= 2.5e-2 and lt["f16"]["vis_mean_abs_err_vs_gpu_fp32"] <= 2e-4
    assert lt["bf16"]["vis_max_abs_err_vs_gpu_fp32"] <= 0.2 and lt["bf16"]["vis_mean_abs_err_vs_gpu_fp32"] <= 2e-3
    r = report["oracle_trained"]["formats"]
    assert r["f32"]["vis_max_abs_err_vs_fp64"] <= 1e-4
    assert r["f16"]["vis_max_abs_err_vs_gpu_fp32"] <= 2.5e-2 and r["f16"]["vis_mean_abs_err_vs_fp64"] <= 2e-4
    assert r["bf16"]["vis_max_abs_err_vs_gpu_fp32"] <= 0.2 and r["bf16"]["vis_mean_abs_err_vs_fp64"] <= 2e-3
    assert r["f32"]["pick_agreement_vs_fp64"] > 0.999 and r["f16"]["pick_agreement_vs_fp64"] > 0.99
    assert np.std(v64) > 0.1          # trained: visibility far from the constant 0.5
