"""The autograd wrappers' gradients against central finite differences of an FP64 forward pass.

The 1080p network on 256 points.  The finite differences use the library's
FP64 forward pass (nvc_forward_f64: FP64 encoding, network and loss on the
GPU, the cell decided in FP32 as everywhere else), step h = 1e-3:

  * every MLP weight (12,288 coordinates), 512 table entries touched by the
    points, and 8 random directions over the weights and the touched entries,
    of the BCE loss L(theta) over 256 points x 32 lights, compared with the
    gradient `NVCLossFunction` (the training kernel in labelled mode) returns;
  * 2048 weights and 512 touched table entries of L(theta) = sum r_bi
    v_bi(theta) for a fixed upstream gradient r, compared with the gradient
    `NVCFunction.backward` (the training kernel in upstream-gradient mode)
    returns.

A coordinate whose perturbation changes any ReLU branch of any point (the
kernel reports every hidden pre-activation's sign) is skipped.

Error budget of a difference quotient D(h) = (L(theta + h e) - L(theta - h e)) / 2h:
  * truncation.  With the branches fixed, the logits are linear in a single
    weight or table entry, z(t) = z + t a with a = (z(h) - z(-h)) / 2h
    computed from the two passes' logits, so for BCE
      |D(h) - L'| <= h^2 / 6 max|sigma''| sum |a|^3 / (B M),  max|sigma''| = 0.0963,
    and for sum r v, h^2 / 6 max|sigma'''| sum |r| |a|^3 with max|sigma'''| = 1/8.
    Along a direction that moves several layers at once the logits are
    polynomial in t; there the truncation is estimated as 2 |D(h) - D(h/2)|.
  * rounding.  Each FP64 logit carries at most a few hundred unit roundoffs
    (2^-53) of its magnitude (<= 1e-12 here), each loss term as much, so L is
    known to 2e-13 (1 + L) and the quotient to 2e-13 (1 + L) / h.
The kernel's own gradient carries its rounding error, bounded entry by entry
by oracle/bounds.py for its format.  Checks:
  |D(h) - g_oracle| <= truncation + rounding     (pins the FP64 pass and the differences)
  |D(h) - g_kernel| <= truncation + rounding + bound(g_kernel)
"""
import numpy as np
import pytest
import torch

from oracle import bounds, hashgrid, mlp as omlp, training
from paper_2506_05930_amd import api
from paper_2506_05930_amd.cache import NVCFunction, NVCLossFunction
from tests.gpu_common import make_cache, p1080, params, rand_pos

pytestmark = pytest.mark.gpu

DEV = "cuda"
H = 1e-3
N = 256
SIG2 = 0.0963


class F64Pass:
    """FP64 parameters on the device and one buffer set per evaluation."""

    def __init__(self, cache, p, pos, labels=None):
        self.cache = cache
        self.t64 = torch.as_tensor(p["table"].astype(np.float64)).to(DEV)
        self.w64 = torch.as_tensor(np.concatenate([w.ravel() for w in p["weights"]]).astype(np.float64)).to(DEV)
        self.pos = pos
        self.labels = labels
        m = cache.mlp
        self.z = torch.empty((N, m.n_out), dtype=torch.float64, device=DEV)
        self.masks = torch.empty((N, m.n_hidden, (m.width + 7) // 8), dtype=torch.uint8, device=DEV)
        self.lo = torch.empty(N + 1, dtype=torch.float64, device=DEV)

    def run(self, z=None, masks=None):
        api.nvc_forward_f64(self.cache.grid, self.cache.mlp, self.t64, self.w64, self.pos, labels=self.labels,
                            loss=self.cache.loss, z=self.z if z is None else z,
                            masks=self.masks if masks is None else masks, loss_out=self.lo if self.labels is not None else None)


def _setup(dtype):
    wl = p1080()
    p = params(wl)
    cache = make_cache(wl, p, dtype=dtype)
    pos_np = rand_pos(31, N, adversarial=False)
    lab_np = (np.random.default_rng(32).uniform(size=(N, wl.mlp.n_out)) > 0.4).astype(np.uint8)
    return wl, p, cache, pos_np, lab_np


def _fd_coordinates(f, coords, mode, r64=None):
    """Central differences of every coordinate: (D(h), truncation bound, branch changed) per coordinate.
    mode "loss": L = the kernel's mean loss (BCE); mode "upstream": L = sum r sigmoid(z), computed here in
    FP64 from the pass's logits."""
    n_out = f.cache.mlp.n_out
    m0 = f.masks.clone()
    lp = torch.empty(len(coords), dtype=torch.float64, device=DEV)
    lm, trunc = torch.empty_like(lp), torch.empty_like(lp)
    flip = torch.empty(len(coords), dtype=torch.bool, device=DEV)
    zp, zm = torch.empty_like(f.z), torch.empty_like(f.z)
    mp, mm = torch.empty_like(m0), torch.empty_like(m0)
    flat_t = f.t64.view(-1)
    for c, (kind, i) in enumerate(coords):
        vec = f.w64 if kind == "w" else flat_t
        x0 = vec[i].clone()
        for sgn, z, mk, out in ((1, zp, mp, lp), (-1, zm, mm, lm)):
            vec[i] = x0 + sgn * H
            f.run(z, mk)
            out[c] = f.lo[N] if mode == "loss" else (torch.sigmoid(z) * r64).sum()
        vec[i] = x0
        flip[c] = (mp != m0).any() | (mm != m0).any()
        a = ((zp - zm) / (2 * H)).abs().pow(3)
        if mode == "loss":         # third derivative <= max|sigma''| sum |a|^3 / (B M)
            trunc[c] = (H * H / 6) * SIG2 * a.sum() / (N * n_out)
        else:                      # third derivative <= max|sigma'''| sum |r| |a|^3, max|sigma'''| = 1/8
            trunc[c] = (H * H / 6) * 0.125 * (r64.abs() * a).sum()
    return ((lp - lm) / (2 * H)).cpu().numpy(), trunc.cpu().numpy(), flip.cpu().numpy()


def _check(fd, tr, fl, rnd, coords, g_w, g_t, ref_w, ref_t, e_w, e_t, min_share):
    got = np.array([g_w[i] if k == "w" else g_t[i] for k, i in coords])
    exact = np.array([ref_w[i] if k == "w" else ref_t[i] for k, i in coords])
    e_path = np.array([e_w[i] if k == "w" else e_t[i] for k, i in coords])
    ok = ~fl
    print(f"  {len(coords)} coordinates, skipped for a branch change: {int(fl.sum())}; largest truncation "
          f"bound {tr[ok].max():.2e}, rounding {rnd:.2e}")
    assert ok.sum() >= min_share * len(coords)
    d_or = np.abs(fd - exact)[ok]
    assert np.all(d_or <= tr[ok] + rnd), f"FD vs oracle: worst {np.max(d_or / (tr[ok] + rnd)):.3f} of the budget"
    d_k = np.abs(fd - got)[ok]
    budget = tr[ok] + rnd + e_path[ok]
    print(f"  FD vs oracle gradient: max {d_or.max():.2e}; FD vs kernel gradient: max {d_k.max():.2e} "
          f"(largest share of its budget {np.max(d_k / budget):.3f}); max|g| {np.abs(exact).max():.2e}")
    assert np.all(d_k <= budget)


# A perturbation of 1e-3 moves a first-layer pre-activation by up to 1e-3 |e| at every one of the 256
# points, so about a sixth of the weights change some point's ReLU branch and are skipped.
MIN_CHECKED = 0.7


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_loss_gradient_against_fp64_central_differences(dtype):
    wl, p, cache, pos_np, lab_np = _setup(dtype)
    pos, lab = torch.as_tensor(pos_np).to(DEV), torch.as_tensor(lab_np).to(DEV)
    table = cache.table.clone().requires_grad_(True)
    w = cache.w.clone().requires_grad_(True)
    loss = NVCLossFunction.apply(pos, table, w, lab, cache)
    loss.backward()
    g_t = table.grad.double().cpu().numpy().ravel()
    g_w = w.grad.double().cpu().numpy()

    f = F64Pass(cache, p, pos, lab)
    f.run()
    z0 = f.z.clone()
    L0 = f.lo[N].item()
    # the FP64 pass against the oracle's forward pass and loss
    enc = hashgrid.encode(pos_np, p["table"], wl.grid.base_res, wl.grid.growth)
    z_ref = omlp.forward(enc, p["weights"])[0]
    assert np.abs(z0.cpu().numpy() - z_ref).max() <= 1e-12 * (1 + np.abs(z_ref).max())
    ref = training.train_gradients(pos_np, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth, labels=lab_np)
    assert abs(L0 - ref["loss"]) <= 1e-13 * (1 + ref["loss"])
    assert abs(loss.item() - ref["loss"]) <= (1e-5 if dtype == "f32" else 3e-2) * ref["loss"]
    eb = bounds.gradient_error_bounds(pos_np, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth,
                                      labels=lab_np, dtype=dtype)
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    e_w = np.concatenate([e.ravel() for e in eb["e_w"]])
    ref_t, e_t = ref["g_table"].ravel(), eb["e_table"].ravel()

    touched = np.flatnonzero(ref_t != 0)
    rng = np.random.default_rng(33)
    t_idx = np.sort(rng.choice(touched, 512, replace=False))
    coords = [("w", i) for i in range(f.w64.numel())] + [("t", int(i)) for i in t_idx]
    print(f"FD {dtype}: every weight and 512 touched table entries", flush=True)
    fd, tr, fl = _fd_coordinates(f, coords, "loss")
    rnd = 2e-13 * (1 + L0) / H
    _check(fd, tr, fl, rnd, coords, g_w, g_t, ref_w, ref_t, e_w, e_t, MIN_CHECKED)

    # eight random directions over the weights and the touched table entries
    flat_t = f.t64.view(-1)
    m0 = f.masks.clone()
    checked = 0
    for j in range(8):
        dw = torch.as_tensor(rng.normal(size=f.w64.numel())).to(DEV)
        dt = torch.zeros_like(flat_t)
        dt[torch.as_tensor(touched).to(DEV)] = torch.as_tensor(rng.normal(size=len(touched))).to(DEV)
        nrm = torch.sqrt((dw * dw).sum() + (dt * dt).sum())
        dw /= nrm
        dt /= nrm
        w_base, t_base = f.w64.clone(), flat_t.clone()
        vals = {}
        for hh in (H, H / 2):
            for sgn in (1, -1):
                f.w64.copy_(w_base + sgn * hh * dw)
                flat_t.copy_(t_base + sgn * hh * dt)
                f.run()
                vals[(hh, sgn)] = (f.lo[N].item(), bool((f.masks != m0).any().item()))
        f.w64.copy_(w_base)
        flat_t.copy_(t_base)
        if any(v[1] for v in vals.values()):
            print(f"  direction {j}: a branch changed, skipped")
            continue
        checked += 1
        d1 = (vals[(H, 1)][0] - vals[(H, -1)][0]) / (2 * H)
        d2 = (vals[(H / 2, 1)][0] - vals[(H / 2, -1)][0]) / H
        dwn, dtn = dw.cpu().numpy(), dt.cpu().numpy()
        an_exact = float(ref_w @ dwn + ref_t @ dtn)
        an_kernel = float(g_w @ dwn + g_t @ dtn)
        e_dir = float(e_w @ np.abs(dwn) + e_t @ np.abs(dtn))
        est = 2 * abs(d1 - d2) + 2 * rnd
        print(f"  direction {j}: FD {d1:.9e} oracle {an_exact:.9e} kernel {an_kernel:.9e} (est. FD error {est:.1e})")
        assert abs(d1 - an_exact) <= est
        assert abs(d1 - an_kernel) <= est + e_dir
    assert checked >= 4


def test_upstream_gradient_against_fp64_central_differences():
    """NVCFunction (inference forward, training kernel in upstream-gradient mode as backward), FP32 path:
    L = sum r v for a fixed upstream gradient r, on 2048 weights and 512 touched table entries."""
    wl, p, cache, pos_np, _ = _setup("f32")
    pos = torch.as_tensor(pos_np).to(DEV)
    r32 = np.random.default_rng(34).normal(size=(N, wl.mlp.n_out)).astype(np.float32)
    r = torch.as_tensor(r32).to(DEV)
    table = cache.table.clone().requires_grad_(True)
    w = cache.w.clone().requires_grad_(True)
    vis = NVCFunction.apply(pos, table, w, cache, 0.0)
    vis.backward(r)
    g_t = table.grad.double().cpu().numpy().ravel()
    g_w = w.grad.double().cpu().numpy()
    r64 = r.double()
    ref = training.train_gradients(pos_np, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth,
                                   dvis=r32.astype(np.float64))
    eb = bounds.gradient_error_bounds(pos_np, p["table"], p["weights"], wl.grid.base_res, wl.grid.growth,
                                      dvis=r32.astype(np.float64), dtype="f32")
    ref_w = np.concatenate([g.ravel() for g in ref["g_w"]])
    e_w = np.concatenate([e.ravel() for e in eb["e_w"]])
    ref_t, e_t = ref["g_table"].ravel(), eb["e_table"].ravel()

    f = F64Pass(cache, p, pos)
    f.run()
    L0 = float((torch.sigmoid(f.z) * r64).sum().item())
    rng = np.random.default_rng(35)
    touched = np.flatnonzero(ref_t != 0)
    coords = [("w", int(i)) for i in np.sort(rng.choice(f.w64.numel(), 2048, replace=False))] + \
             [("t", int(i)) for i in np.sort(rng.choice(touched, 512, replace=False))]
    print("FD upstream: 2048 weights and 512 touched table entries", flush=True)
    fd, tr, fl = _fd_coordinates(f, coords, "upstream", r64)
    rnd = 2e-13 * (np.abs(r32).sum() + abs(L0)) / H
    _check(fd, tr, fl, rnd, coords, g_w, g_t, ref_w, ref_t, e_w, e_t, MIN_CHECKED)
