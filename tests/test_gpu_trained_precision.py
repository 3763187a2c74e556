"""Visibility precision of the 1080p network (32 -> 64 x3 -> 32, FP16 matrix cores) on trained weights.

A fresh network outputs about 0.5 everywhere, which hides rounding; these
checks use trained parameters.

* GPU-trained: 200 training steps of 2^18 samples on the FP32 path (the 1080p
  training workload); the same FP32 master parameters are then packed for FP16
  and BF16 and every pixel of the 1920x1080 frame is compared with the FP32
  path.  Nothing here goes through the oracle: its inputs never come from the
  HIP path.  The precision target (FP16 within 2e-3 of the FP32 path) is NOT
  met on this network and is kept as an expected failure: after 200 steps
  (BCE 0.004) the output logits are sums of terms whose magnitudes add up to
  ~250 while the logit itself is near 0, so rounding the encoding, the
  weights and the hidden activations to FP16 (unit roundoff 2^-11) moves such
  a logit by up to ~0.07, i.e. the visibility by up to ~0.02.  An emulation of
  the same network with every operand rounded to FP16 and FP32 sums
  reproduces the kernel's largest error to 4 digits; every rounding site
  contributes (encoding 7e-3, weights 8e-3, hidden activations 1.5e-2 alone),
  and only a three-product split (hi and lo FP16 parts of both operands)
  brings it under 2e-3.  What FP16 does deliver there is gated: mean error
  below 1e-4 and max below u16 * 250 / 4 ~ 3e-2.
* Oracle-trained: 30 steps of 4096 samples trained by the oracle itself (FP64,
  its composed training step on a 320x180 render of the scene); those
  parameters, rounded to FP32, feed both sides.  Every format is compared with
  the oracle's FP64 forward on a 65,536-pixel subset of the 1080p G-buffer,
  with the light pick and its pmf.  Gates: FP32 within 2e-5, FP16 within 2e-3
  of the FP64 visibility.
Both print the max, mean and 99.9th-percentile errors per format.
"""
import numpy as np
import pytest
import torch

from oracle import pipeline
from tests.gpu_common import make_cache
from workloads import box_scene, get_workload, init_params
from workloads.scenes import unflatten_weights

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).to(DEV)


def _frame(wl):
    return box_scene(wl.scene_seed, wl.width, wl.height, wl.n_boxes, wl.n_lights, wl.n_spheres)


def _stats(e):
    return f"max {e.max():.3e} mean {e.mean():.3e} 99.9% {np.quantile(e, 0.999):.3e}"


_TRAINED = {}


def _gpu_trained():
    """The 1080p network after 200 training steps on the FP32 path, and its FP32 and FP16 / BF16 outputs."""
    if not _TRAINED:
        wl = get_workload("train_1080p")
        sc = _frame(wl)
        p = init_params(wl.init_seed, wl.grid, wl.mlp)               # the workload's own initialisation
        c32 = make_cache(wl, p, dtype="f32")
        pos_unit, pos = t(sc["pos_unit"]), t(sc["pos"])
        lights, spheres = t(sc["lights"]), t(sc["spheres"])
        print("training 200 steps on the FP32 path", flush=True)
        for frame in range(200):
            c32.train_step(pos_unit, pos, lights, spheres, frame, wl.train_batch)
        trained = {"table": c32.table.cpu().numpy(), "weights": unflatten_weights(c32.w.cpu().numpy(), wl.mlp)}
        v32 = c32.infer(pos_unit)
        z = torch.logit(v32.double().clamp(1e-12, 1 - 1e-12))
        print(f"  loss after 200 steps {c32.loss_buf.item():.4f}; visibility std {v32.std().item():.3f}, "
              f"|logit| 99th percentile {torch.quantile(z.abs().flatten()[::97], 0.99).item():.1f}")
        _TRAINED["v32"] = v32
        for fmt in ("f16", "bf16"):
            v = make_cache(wl, trained, dtype=fmt).infer(pos_unit, dtype=torch.float32)
            e = (v - v32).abs().flatten()
            _TRAINED[fmt] = (e.max().item(), e.mean().item())
            print(f"  {fmt} vs FP32 path, {sc['pos'].shape[0]} pixels x 32 lights: max {e.max().item():.3e} "
                  f"mean {e.mean().item():.3e}")
    return _TRAINED


def test_low_precision_paths_on_gpu_trained_network():
    r = _gpu_trained()
    assert r["v32"].std().item() > 0.1
    assert r["f16"][1] <= 1e-4 and r["f16"][0] <= 3e-2
    assert r["bf16"][1] <= 1e-3 and r["bf16"][0] <= 0.25


@pytest.mark.xfail(strict=True, reason="FP16 rounding of a well-trained network exceeds the 2e-3 target "
                                       "(cancellation in the output logits); see the module docstring")
def test_f16_within_target_of_f32_path_after_200_gpu_training_steps():
    assert _gpu_trained()["f16"][0] <= 2e-3


def test_formats_against_fp64_on_oracle_trained_weights():
    wl = get_workload("train_1080p")
    small = box_scene(wl.scene_seed, 320, 180, wl.n_boxes, wl.n_lights, wl.n_spheres)
    p = init_params(wl.init_seed, wl.grid, wl.mlp)
    state, tab, ws = None, p["table"], p["weights"]
    print("oracle training: 30 steps of 4096 samples", flush=True)
    for f in range(30):
        out = pipeline.train_step(small["pos_unit"], small["pos"], small["lights"], small["spheres"], tab, ws,
                                  wl.grid.base_res, wl.grid.growth, seed=wl.rng_key, frame=f, batch=4096,
                                  adam_state=state, lr=wl.lr, beta1=wl.beta1, beta2=wl.beta2, eps=wl.adam_eps)
        state, tab, ws = out["adam"], out["table"], out["weights"]
    trained = {"table": tab.astype(np.float32), "weights": [w.astype(np.float32) for w in ws]}
    print(f"  oracle loss after 30 steps {out['loss']:.4f}", flush=True)

    sc = _frame(wl)
    n = sc["pos"].shape[0]
    sub = np.sort(np.random.default_rng(3).choice(n, 65536, replace=False))
    pu, ps, pn = sc["pos_unit"][sub], sc["pos"][sub], sc["nrm"][sub]
    v64 = pipeline.infer(pu, trained["table"], trained["weights"], wl.grid.base_res, wl.grid.growth)
    assert v64.std() > 0.1
    ref = pipeline.sample(v64, ps, pn, sc["lights"], wl.rng_key, 0, wl.vis_floor)
    p64 = ref["w64"] / ref["w64"].sum(axis=1, keepdims=True)
    err = {}
    for fmt in ("f32", "f16", "bf16"):
        cache = make_cache(wl, trained, dtype=fmt)
        vis = cache.infer(t(pu))                                    # the format's own output dtype
        v = vis.float().cpu().numpy().astype(np.float64)
        e = np.abs(v - v64)
        err[fmt] = e.max()
        out = cache.sample(vis, t(ps), t(pn), t(sc["lights"]), 0)
        idx = out["idx"].cpu().numpy()
        pmf = out["pmf"].cpu().numpy().astype(np.float64)
        exact = np.take_along_axis(p64, np.maximum(idx, 0)[:, None], axis=1)[:, 0]
        pe = np.abs(pmf - exact)[idx >= 0]
        print(f"  {fmt}: visibility vs FP64 {_stats(e)}; pick agreement {np.mean(idx == ref['idx']):.5f}; "
              f"pmf vs FP64 max {pe.max():.3e} mean {pe.mean():.3e}")
    assert err["f32"] <= 2e-5
    assert err["f16"] <= 2e-3
    assert err["bf16"] <= 3e-2
