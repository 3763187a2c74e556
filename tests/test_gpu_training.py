"""What training the cache on the GPU gains (Sec. 1, Sec. 3.1, Sec. 3.4).

The network is trained online by the library's own kernels (pixel picks,
shadow-ray labels, forward + backward, Adam) on a static 1080p-class scene
rendered at 320x180.  The gain is measured with the exact moments of the
one-sample light estimator (no Monte Carlo noise), with the true visibility
from the oracle's shadow rays: sampling by the unshadowed weight times the
trained cache's clamped visibility must have clearly lower variance and pick
occluded lights less often than sampling by the unshadowed weight alone, and
must stay unbiased (every light with f V > 0 keeps a positive probability).
An untrained network gains nothing (its prediction is about 0.5 everywhere).
"""
import numpy as np
import pytest
import torch

from oracle import estimator, lighting, shadow
from tests.gpu_common import make_cache
from workloads import box_scene, get_workload, init_params

pytestmark = pytest.mark.gpu

DEV = "cuda"


def t(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to(DEV)


def test_trained_cache_reduces_estimator_variance():
    wl = get_workload("frame_1080p")
    sc = box_scene(0, 320, 180, 64, 32, 256)
    n = sc["pos"].shape[0]
    p = init_params(1, wl.grid, wl.mlp)          # the workload's own initialisation
    cache = make_cache(wl, p)
    pos_unit, pos, nrm = t(sc["pos_unit"]), t(sc["pos"]), t(sc["nrm"])
    lights, spheres = t(sc["lights"]), t(sc["spheres"])
    sub = np.random.default_rng(5).choice(n, 4096, replace=False)
    V = shadow.labels_fp32(sc["pos"][sub], sc["lights"], sc["spheres"]).astype(np.float64)
    f = lighting.unshadowed_weight(sc["pos"][sub], sc["nrm"][sub], sc["lights"])
    sub_t = t(sc["pos_unit"][sub])

    def stats():
        v = cache.infer(sub_t, dtype=torch.float32).cpu().numpy().astype(np.float64)
        w = f * np.maximum(v, wl.vis_floor)
        pc = w / w.sum(1, keepdims=True)
        pn = f / f.sum(1, keepdims=True)
        ok = (f * V).sum(1) > 0
        mu, Ec, var_c, waste_c = estimator.moments(f[ok], V[ok], pc[ok])
        _, En, var_n, waste_n = estimator.moments(f[ok], V[ok], pn[ok])
        assert np.allclose(Ec, mu, rtol=1e-12) and np.allclose(En, mu, rtol=1e-12)   # unbiased
        return var_c.mean() / var_n.mean(), waste_c.mean(), waste_n.mean(), np.abs(v - V).mean()

    r0, wc0, wn0, mae0 = stats()
    for frame in range(150):
        cache.train_step(pos_unit, pos, lights, spheres, frame, 1 << 14)
    r1, wc1, wn1, mae1 = stats()
    print(f"variance ratio cache/none: untrained {r0:.3f} trained {r1:.3f}; occluded picks {wn1:.3f} -> {wc1:.3f}; "
          f"visibility MAE {mae0:.3f} -> {mae1:.3f}; loss {cache.loss_buf.item():.4f}")
    assert 0.8 < r0 < 1.25 and abs(wc0 - wn0) < 0.05
    assert r1 < 0.7
    assert wc1 < wn1 - 0.1
    assert mae1 < 0.5 * mae0
