"""Pins of the oracle's MLP, losses, gradients and Adam (Sec. 3.3, Sec. 3.4)."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import hashgrid, mlp, training

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _hand():
    with open(os.path.join(GOLD, "mlp_two_layer_hand.json")) as f:
        return json.load(f)


def test_two_layer_hand_example_forward_and_backward():
    g = _hand()
    W = [np.array(g["W1"]), np.array(g["W2"])]
    enc = np.array([g["enc"]])
    z, pre, inputs = mlp.forward(enc, W)
    assert z[0, 0] == g["z"]
    assert abs(mlp.sigmoid(z)[0, 0] - g["v"]) < 1e-17
    loss, dz = training.bce_loss(z, np.array([[g["label"]]]))
    assert abs(loss - g["loss"]) < 1e-14
    assert abs(dz[0, 0] - g["dz"]) < 1e-16
    dW, d_enc = mlp.backward(W, pre, inputs, dz)
    assert np.allclose(dW[0], g["dW1"], rtol=0, atol=1e-15)
    assert np.allclose(dW[1], g["dW2"], rtol=0, atol=1e-15)
    assert np.allclose(d_enc[0], g["d_enc"], rtol=0, atol=1e-15)


def test_sigmoid_special_values():
    z = np.array([0.0, 1000.0, -1000.0, 3.0, -3.0])
    s = mlp.sigmoid(z)
    assert s[0] == 0.5 and s[1] == 1.0 and s[2] == 0.0
    assert abs(s[3] + s[4] - 1.0) <= 2.3e-16
    assert np.all(np.isfinite(s))


def _torch_net(weights, kind, slope):
    layers = []
    for k, W in enumerate(weights):
        lin = torch.nn.Linear(W.shape[1], W.shape[0], bias=False).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(np.asarray(W, np.float64)))
        layers.append(lin)
        if k < len(weights) - 1:
            layers.append(torch.nn.ReLU() if kind == "relu" else torch.nn.LeakyReLU(slope))
    return torch.nn.Sequential(*layers)


@pytest.mark.parametrize("kind", ["relu", "leaky"])
def test_forward_backward_match_torch_autograd(kind):
    rng = np.random.default_rng(0)
    shapes = [(64, 32), (64, 64), (64, 64), (32, 64)]
    weights = [rng.normal(scale=1 / math.sqrt(i), size=(o, i)) for o, i in shapes]
    enc = rng.normal(size=(300, 32))
    y = (rng.uniform(size=(300, 32)) > 0.4).astype(np.float64)
    z, pre, inputs = mlp.forward(enc, weights, kind)
    loss, dz = training.bce_loss(z, y)
    dW, d_enc = mlp.backward(weights, pre, inputs, dz, kind)

    net = _torch_net(weights, kind, 0.01)
    x = torch.from_numpy(enc).requires_grad_(True)
    zt = net(x)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.from_numpy(y))
    lt.backward()
    assert np.max(np.abs(zt.detach().numpy() - z)) < 1e-12
    assert abs(lt.item() - loss) < 1e-13
    lin = [m for m in net if isinstance(m, torch.nn.Linear)]
    for k in range(len(weights)):
        ref = lin[k].weight.grad.numpy()
        assert np.max(np.abs(ref - dW[k])) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(x.grad.numpy() - d_enc)) < 1e-13


def test_l2_loss_matches_torch():
    rng = np.random.default_rng(1)
    z = rng.normal(size=(50, 8))
    y = (rng.uniform(size=(50, 8)) > 0.5).astype(np.float64)
    loss, dz = training.l2_loss(z, y)
    zt = torch.from_numpy(z).requires_grad_(True)
    lt = torch.nn.functional.mse_loss(torch.sigmoid(zt), torch.from_numpy(y))
    lt.backward()
    assert abs(lt.item() - loss) < 1e-14
    assert np.max(np.abs(zt.grad.numpy() - dz)) < 1e-16


def test_bce_closed_forms():
    # z = 0: loss log 2 whatever the label, gradient (1/2 - y)/n.
    z = np.zeros((4, 2))
    y = np.array([[0, 1], [1, 0], [1, 1], [0, 0]], np.float64)
    loss, dz = training.bce_loss(z, y)
    assert abs(loss - math.log(2.0)) < 1e-15
    assert np.allclose(dz, (0.5 - y) / 8, atol=0)
    # large |z| stays finite
    loss, dz = training.bce_loss(np.array([[800.0, -800.0]]), np.array([[0.0, 1.0]]))
    assert abs(loss - 800.0) < 1e-9 and np.all(np.isfinite(dz))


def test_full_gradient_matches_torch_autograd_through_the_encoding():
    """Table and weight gradients of the whole path against torch FP64 autograd.

    torch gathers the 8 corners (indices and trilinear weights from the pinned
    hash-grid oracle) and differentiates the gather, so the scatter of
    `training.table_gradient` is checked by an independent route.
    """
    rng = np.random.default_rng(3)
    L, T, F = 8, 1 << 10, 2
    base, growth = 4, 1.5
    table = rng.uniform(-0.5, 0.5, size=(L, T, F)).astype(np.float32)
    shapes = [(32, 16), (32, 32), (8, 32)]
    weights = [rng.normal(scale=0.5, size=s).astype(np.float32) for s in shapes]
    pos = rng.uniform(0, 1, size=(256, 3)).astype(np.float32)
    y = (rng.uniform(size=(256, 8)) > 0.5).astype(np.float64)
    out = training.train_gradients(pos, table, weights, base, growth, labels=y, loss="bce")

    tt = torch.from_numpy(table.astype(np.float64)).requires_grad_(True)
    ws = [torch.from_numpy(w.astype(np.float64)).requires_grad_(True) for w in weights]
    res = hashgrid.level_resolutions(base, growth, L)
    feats = []
    for l in range(L):
        idx, w = hashgrid.corners(pos, res[l], T)
        vals = tt[l][torch.from_numpy(idx)]                       # [n,8,F]
        feats.append((torch.from_numpy(w)[:, :, None] * vals).sum(1))
    h = torch.cat(feats, 1)
    for k, W in enumerate(ws):
        h = h @ W.T
        if k < len(ws) - 1:
            h = torch.relu(h)
    lt = torch.nn.functional.binary_cross_entropy_with_logits(h, torch.from_numpy(y))
    lt.backward()
    assert abs(lt.item() - out["loss"]) < 1e-13
    assert np.max(np.abs(tt.grad.numpy() - out["g_table"])) < 1e-15
    for k in range(len(ws)):
        assert np.max(np.abs(ws[k].grad.numpy() - out["g_w"][k])) < 1e-14


def test_central_finite_differences():
    """Central differences (h = 1e-3, FP64) on weights, touched table entries and random directions.

    The trilinear encoding is linear in the table, so those differences are
    exact up to rounding; for weights, perturbations that flip a ReLU mask are
    skipped (detected by comparing masks).
    """
    rng = np.random.default_rng(11)
    L, T, F = 4, 1 << 8, 2
    base, growth = 4, 1.5
    table = rng.uniform(-0.5, 0.5, size=(L, T, F))
    shapes = [(16, 8), (16, 16), (4, 16)]
    weights = [rng.normal(scale=0.6, size=s) for s in shapes]
    pos = rng.uniform(0, 1, size=(64, 3)).astype(np.float32)
    y = (rng.uniform(size=(64, 4)) > 0.5).astype(np.float64)
    out = training.train_gradients(pos, table, weights, base, growth, labels=y)

    def loss_and_masks(tab, ws):
        enc = hashgrid.encode(pos, tab, base, growth)
        z, pre, _ = mlp.forward(enc, ws)
        return training.bce_loss(z, y)[0], [p > 0 for p in pre]

    _, masks0 = loss_and_masks(table, weights)
    h = 1e-3
    checked = 0
    for k, W in enumerate(weights):
        for _ in range(12):
            i, j = rng.integers(0, W.shape[0]), rng.integers(0, W.shape[1])
            wp = [w.copy() for w in weights]
            wm = [w.copy() for w in weights]
            wp[k][i, j] += h
            wm[k][i, j] -= h
            lp, mp = loss_and_masks(table, wp)
            lm, mm = loss_and_masks(table, wm)
            if any((a != b).any() for a, b in zip(mp, masks0)) or any((a != b).any() for a, b in zip(mm, masks0)):
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(fd - out["g_w"][k][i, j]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9
            checked += 1
    touched = np.argwhere(np.abs(out["g_table"]) > 0)
    for l, t, f in touched[rng.choice(len(touched), 40, replace=False)]:
        tp, tm = table.copy(), table.copy()
        tp[l, t, f] += h
        tm[l, t, f] -= h
        lp, mp = loss_and_masks(tp, weights)
        lm, mm = loss_and_masks(tm, weights)
        if any((a != b).any() for a, b in zip(mp, masks0)) or any((a != b).any() for a, b in zip(mm, masks0)):
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(fd - out["g_table"][l, t, f]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10
        checked += 1
    assert checked > 40


def test_adam_matches_torch_optim_adam_ten_steps():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=1000)
    grads = [rng.normal(size=1000) * (0.1 ** rng.integers(0, 4)) for _ in range(10)]
    grads[3][::7] = 0.0
    pt = torch.from_numpy(p0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.99), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    for t, g in enumerate(grads, start=1):
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = training.adam_step(p, g, m, v, t, 1e-2, 0.9, 0.99, 1e-8)
        assert np.max(np.abs(pt.detach().numpy() - p)) <= 1e-12 * np.max(np.abs(p))


def test_learning_rate_schedule_points():
    """Sec. 3.4: start at 0.05, lowered linearly over the first 200 steps to 0.001, constant after."""
    lr = [training.learning_rate(t, 0.05, 0.001, 200) for t in range(1, 400)]
    assert lr[0] == 0.05 and lr[200] == 0.001 and lr[-1] == 0.001
    assert abs(lr[100] - 0.0255) <= 1e-15                    # halfway: the mean of the two rates
    steps = np.diff(lr[:201])
    assert np.all(steps < 0) and np.allclose(steps, -0.049 / 200, rtol=1e-9, atol=0)
    assert training.learning_rate(7, 0.01) == 0.01 and training.learning_rate(7, 0.01, 0.5, 0) == 0.01


def test_adam_with_schedule_matches_torch_linear_lr():
    """The schedule equals torch's LinearLR (factor 1 -> lr1/lr0 over D scheduler steps) driving torch Adam."""
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=300)
    pt = torch.from_numpy(p0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=0.05, betas=(0.9, 0.99), eps=1e-8)
    sched = torch.optim.lr_scheduler.LinearLR(opt, start_factor=1.0, end_factor=0.001 / 0.05, total_iters=200)
    p, m, v = p0.copy(), np.zeros(300), np.zeros(300)
    for t in range(1, 231):
        g = rng.normal(size=300) * 0.1
        pt.grad = torch.from_numpy(g.copy())
        assert abs(opt.param_groups[0]["lr"] - training.learning_rate(t, 0.05, 0.001, 200)) <= 1e-15
        opt.step()
        sched.step()
        p, m, v = training.adam_step(p, g, m, v, t, training.learning_rate(t, 0.05, 0.001, 200), 0.9, 0.99, 1e-8)
    assert np.max(np.abs(pt.detach().numpy() - p)) <= 1e-11 * np.max(np.abs(p))


def test_adam_first_step_closed_form():
    # t = 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps).
    g = np.array([1.0, -2.0, 1e-3, 0.0])
    p, m, v = training.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.5, 0.9, 0.99, 1e-8)
    assert np.allclose(p, -0.5 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.01 * g * g)


def test_world_points_uniform_in_the_box():
    """World-space samples (Sec. 3.4): inside the box, uniform per axis, unit positions = p / extent."""
    from oracle import philox
    box = (0.5, 1.0, 2.0, 9.5, 4.0, 8.0)
    p, u = philox.world_points(2, 3, 200000, box, 10.0)
    lo, hi = np.array(box[:3]), np.array(box[3:])
    assert np.all(p >= lo) and np.all(p < hi)
    for k in range(3):
        cnt, _ = np.histogram(p[:, k], bins=20, range=(lo[k], hi[k]))
        chi2 = ((cnt - 10000.0) ** 2 / 10000.0).sum()
        assert chi2 < 45.0                                       # 19 dof, p ~ 1e-3
    assert np.array_equal(u, (p.astype(np.float64) / 10.0).astype(np.float32))
    # the first coordinate is the uniform of the first Philox word of counter (i, frame, 6)
    w = philox.philox4x32_10(philox._counter(np.arange(5, dtype=np.uint64), 3, 6), philox._key(2))[0]
    assert np.allclose(p[:5, 0], lo[0] + philox.uniform24(w).astype(np.float64) * 9.0, rtol=1e-6)


def test_pipeline_train_step_matches_torch_autograd_and_adam():
    """The composed training step (Sec. 3.4: pick pixels, label them with shadow rays, backpropagate,
    one Adam step on every parameter) against an independent route: torch FP64 autograd through the
    corner gather and torch.optim.Adam on [table, W_1, ...], three steps with the optimiser state
    carried.  The pixel draws and shadow labels it consumes are pinned on their own (Random123 known
    answers; analytic and brute-force label cases); this checks how the step wires them together:
    which positions are trained, which gradient reaches which parameter, and the Adam state."""
    from oracle import philox, pipeline, shadow
    from workloads import unit_cube_scene
    sc = unit_cube_scene(4, 300, 8, 12)
    rng = np.random.default_rng(8)
    L, T, F = 4, 1 << 9, 2
    base, growth = 4, 1.5
    table = rng.uniform(-0.5, 0.5, size=(L, T, F)).astype(np.float32)
    weights = [rng.normal(scale=0.5, size=s).astype(np.float32) for s in [(16, 8), (16, 16), (8, 16)]]
    res = hashgrid.level_resolutions(base, growth, L)
    tt = torch.from_numpy(table.astype(np.float64)).requires_grad_(True)
    ws = [torch.from_numpy(w.astype(np.float64)).requires_grad_(True) for w in weights]
    opt = torch.optim.Adam([tt, *ws], lr=0.02, betas=(0.9, 0.99), eps=1e-8)
    state, cur_t, cur_w = None, table, weights
    batch = 200
    for frame in range(3):
        out = pipeline.train_step(sc["pos"], sc["pos"], sc["lights"], sc["spheres"], cur_t, cur_w, base, growth,
                                  seed=5, frame=frame, batch=batch, adam_state=state, lr=0.02)
        pix = philox.training_pixels(5, frame, batch, sc["pos"].shape[0])
        assert np.array_equal(out["pix"], pix)
        y = shadow.labels_fp32(sc["pos"][pix], sc["lights"], sc["spheres"])
        assert np.array_equal(out["labels"], y) and 0.05 < y.mean() < 0.99
        p = sc["pos"][pix]
        opt.zero_grad()
        feats = []
        for l in range(L):
            idx, w = hashgrid.corners(p, res[l], T)
            feats.append((torch.from_numpy(w)[:, :, None] * tt[l][torch.from_numpy(idx)]).sum(1))
        h = torch.cat(feats, 1)
        for k, W in enumerate(ws):
            h = h @ W.T
            if k < len(ws) - 1:
                h = torch.relu(h)
        lt = torch.nn.functional.binary_cross_entropy_with_logits(h, torch.from_numpy(y.astype(np.float64)))
        lt.backward()
        opt.step()
        assert abs(lt.item() - out["loss"]) <= 1e-13
        assert np.max(np.abs(tt.detach().numpy() - out["table"])) <= 1e-12
        for k in range(len(ws)):
            assert np.max(np.abs(ws[k].detach().numpy() - out["weights"][k])) <= 1e-12
        assert out["adam"]["t"] == frame + 1
        # the next step starts from the updated parameters (FP64 carried, as torch does)
        state, cur_t, cur_w = out["adam"], out["table"], out["weights"]
    # entries no sample touched moved only by their earlier steps' moments: at step 1 an untouched
    # entry has g = 0 and stays put
    first = pipeline.train_step(sc["pos"], sc["pos"], sc["lights"], sc["spheres"], table, weights, base, growth,
                                seed=5, frame=0, batch=batch, lr=0.02)
    untouched = first["grads"]["g_table"] == 0
    assert untouched.any() and np.array_equal(first["table"][untouched], table.astype(np.float64)[untouched])


def test_l2_loss_leaves_confident_misses_bce_does_not():
    """Why the paper's L2 loss can raise the mean variance of the light estimator (Sec. 3.1 Fig. "bias":
    fireflies) while BCE lowers it, on the oracle alone.  The paper's network and schedule (ten levels of
    four features, 40-32-32-32 leaky ReLU, rate 0.05 decaying) trained for 25 steps of 2048 screen samples
    with each loss.  With L2 the gradient 2 (v - y) v (1 - v) vanishes on a visible light predicted near
    zero, so such confident misses persist; clamped to 0.001 they get a tiny pick probability and their
    1/p term dominates the second moment.  With BCE (gradient v - y) they are rare."""
    from oracle import estimator, lighting, pipeline, shadow
    from workloads import box_scene, get_workload, init_params
    sc = box_scene(0, 96, 54, 64, 32, 256)
    n = sc["pos"].shape[0]
    sub = np.random.default_rng(5).choice(n, 1024, replace=False)
    V = shadow.labels_fp32(sc["pos"][sub], sc["lights"], sc["spheres"]).astype(np.float64)
    f = lighting.unshadowed_weight(sc["pos"][sub], sc["nrm"][sub], sc["lights"])
    ok = (f * V).sum(1) > 0
    out = {}
    for loss in ("l2", "bce"):
        wl = get_workload("paper_1080p", loss=loss)
        p = init_params(wl.init_seed, wl.grid, wl.mlp, init=wl.init)
        state, tab, ws = None, p["table"], p["weights"]
        for s in range(25):
            lr = training.learning_rate(s + 1, wl.lr, wl.lr_end, wl.lr_decay_steps)
            r = pipeline.train_step(sc["pos_unit"], sc["pos"], sc["lights"], sc["spheres"], tab, ws,
                                    wl.grid.base_res, wl.grid.growth, seed=2, frame=s, batch=2048, adam_state=state,
                                    lr=lr, loss=loss, act="leaky", slope=0.01)
            state, tab, ws = r["adam"], r["table"], r["weights"]
        v = pipeline.infer(sc["pos_unit"][sub], tab.astype(np.float32), [w.astype(np.float32) for w in ws],
                           wl.grid.base_res, wl.grid.growth, act="leaky", slope=0.01)
        w = f * np.maximum(v, 1e-3)
        pc = w / w.sum(1, keepdims=True)
        pn = f / f.sum(1, keepdims=True)
        _, Ec, vc, _ = estimator.moments(f[ok], V[ok], pc[ok])
        mu, _, vn, _ = estimator.moments(f[ok], V[ok], pn[ok])
        assert np.allclose(Ec, mu, rtol=1e-12)                     # the clamp keeps it unbiased
        miss = (V[ok] == 1) & (v[ok] < 0.01) & (f[ok] > 0)
        c = f[ok] * V[ok]
        second = np.where(pc[ok] > 0, c * c / np.where(pc[ok] > 0, pc[ok], 1.0), 0.0)
        out[loss] = {"miss": miss.mean(), "miss_share": (second * miss).sum() / second.sum(),
                     "ratio": vc.mean() / vn.mean(), "median": np.median(vc[vn > 0] / vn[vn > 0])}
    l2, bce = out["l2"], out["bce"]
    assert l2["miss"] > 10 * bce["miss"] and l2["miss_share"] > 0.5
    assert l2["ratio"] > 1.0 > bce["ratio"]
    assert l2["median"] < 0.5 and bce["median"] < 0.5               # the typical pixel gains with either loss
