"""The autograd wrapper's backward against central finite differences.

L(theta) = sum_{b,i} r_bi * vis_bi(theta) for a fixed random upstream
gradient r, with vis from the library's FP32 forward (nvc_infer) on 256
points.  Its gradient from NVCFunction.backward (the training kernel in
upstream-gradient mode) is projected on unit directions d and compared with
(L(theta + h d) - L(theta - h d)) / 2h, the two sums taken in FP64 on the
GPU.  Directions: the table part of the gradient and the weight part, each
scaled entrywise by random factors in [0.5, 1.5] (so they differ from the
gradient but keep a projection far above the noise), and the gradient's own
direction.

Error budget: each FP32 visibility carries an error of a few 1e-7 (hardware
exp2 and reciprocal in the sigmoid), so L carries about
sqrt(256 * 32) * 3e-7 / 2 = 1.4e-5 and the difference quotient 1.4e-5 / h.
With h = 1e-2 that is 1.4e-3; the O(h^2) term (a parameter moves by about
1e-4) and a rare ReLU kink inside +-h add less.
Bound: |FD - <g, d>| <= 1e-2 |<g, d>| + 2e-3.
"""
import numpy as np
import pytest
import torch

from paper_2506_05930_amd.cache import NVCFunction
from tests.gpu_common import make_cache, p1080, params, rand_pos

pytestmark = pytest.mark.gpu

DEV = "cuda"


def test_backward_matches_central_differences():
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p, dtype="f32")
    n = 256
    pos = torch.as_tensor(rand_pos(31, n)).to(DEV)
    r = torch.as_tensor(np.random.default_rng(32).normal(size=(n, wl.mlp.n_out)).astype(np.float32)).to(DEV)
    table = cache.table.clone().requires_grad_(True)
    w = cache.w.clone().requires_grad_(True)
    vis = NVCFunction.apply(pos, table, w, cache, 0.0)
    vis.backward(r)
    g_t, g_w = table.grad.detach(), w.grad.detach()

    def L(tab, ww):
        with torch.no_grad():
            v = NVCFunction.apply(pos, tab.contiguous(), ww.contiguous(), cache, 0.0)
        return (v.double() * r.double()).sum().item()

    rng = np.random.default_rng(33)
    touched = (g_t != 0)
    d_t = g_t * torch.as_tensor(rng.uniform(0.5, 1.5, size=tuple(table.shape)).astype(np.float32)).to(DEV)
    d_t /= d_t.norm()
    d_w = g_w * torch.as_tensor(rng.uniform(0.5, 1.5, size=tuple(w.shape)).astype(np.float32)).to(DEV)
    d_w /= d_w.norm()
    gn = torch.sqrt((g_t.double() ** 2).sum() + (g_w.double() ** 2).sum())
    dirs = [("table", d_t, torch.zeros_like(d_w)), ("weights", torch.zeros_like(d_t), d_w),
            ("gradient", (g_t.double() / gn).float(), (g_w.double() / gn).float())]
    h = 1e-2
    base_t, base_w = table.detach(), w.detach()
    for name, dt, dw in dirs:
        fd = (L(base_t + h * dt, base_w + h * dw) - L(base_t - h * dt, base_w - h * dw)) / (2 * h)
        an = ((g_t.double() * dt.double()).sum() + (g_w.double() * dw.double()).sum()).item()
        print(f"{name}: FD {fd:.6e} analytic {an:.6e}")
        assert abs(fd - an) <= 1e-2 * abs(an) + 2e-3, (name, fd, an)
        assert abs(an) > 0.05
    assert touched.sum().item() > 1000
