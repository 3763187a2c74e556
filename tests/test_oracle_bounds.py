"""Pins of the oracle's element-wise error bounds (oracle/bounds.py).

The bounds are checked against an independent emulation of the arithmetic
they describe: the encoding, the network and its backpropagation evaluated
with every operand rounded to FP32, FP16 or BF16 and every dot product
accumulated in FP32 one addition at a time, in a random order, as a
kernel may do.  Whatever the order, the emulated result must stay within
the bound, at every visibility and every gradient entry, on networks built
so that some hidden pre-activations sit near zero (the masks the
low-precision pass may flip).  In exact arithmetic (every unit roundoff
set to zero) the bound must vanish.  And the bound must not be vacuous:
on the worst entry the emulated error reaches a stated share of it.
"""
import numpy as np
import pytest

from oracle import bounds, hashgrid, mlp, training

GRID = dict(L=4, F=2, T=1 << 10, base=4, growth=2.0)


def round_to(x, fmt):
    """Round FP64 values to the format (nearest, ties to even)."""
    x = np.asarray(x, np.float64)
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    if fmt == "f16":
        return x.astype(np.float16).astype(np.float64)
    if fmt == "bf16":
        b = x.astype(np.float32).view(np.uint32).astype(np.uint64)
        b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
        return b.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(fmt)


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def seq_sum(terms, axis, rng):
    """FP32 sum of `terms` along `axis`, one rounded addition at a time, in a random order."""
    t = np.moveaxis(np.asarray(terms, np.float64), axis, 0)
    order = rng.permutation(t.shape[0])
    acc = np.zeros(t.shape[1:])
    for i in order:
        acc = f32(acc + t[i])
    return acc


def emulate(pos, table, weights, labels, fmt, act, slope, loss, rng):
    """Visibility and gradients computed with the rounding the bounds describe."""
    L, T, F = table.shape
    res = hashgrid.level_resolutions(GRID["base"], GRID["growth"], L)
    n = pos.shape[0]
    enc = np.zeros((n, L * F))
    corners = []
    for l in range(L):
        idx, _ = hashgrid.corners(pos, res[l], T)
        _, fr = hashgrid.cell_and_fraction(pos, res[l])
        off = hashgrid.corner_offsets()
        w = np.ones((n, 8))
        for k in range(3):
            fk = fr[:, None, k]
            factor = np.where(off[None, :, k] == 1, fk, f32(1.0 - fk))
            w = f32(w * factor)
        vals = table[l].astype(np.float64)[idx]                    # [n,8,F]
        enc[:, l * F:(l + 1) * F] = seq_sum(f32(w[:, :, None] * vals), 1, rng)
        corners.append((idx, w))
    h = round_to(enc, fmt)
    Wr = [round_to(W, fmt) for W in weights]
    hs, pres = [], []
    for k, W in enumerate(Wr):
        hs.append(h)
        prod = f32(h[:, None, :] * W[None, :, :]) if fmt == "f32" else h[:, None, :] * W[None, :, :]
        pre = seq_sum(prod, 2, rng)
        pres.append(pre)
        if k < len(Wr) - 1:
            h = round_to(mlp.act(pre, act, slope), fmt)
    z = pres[-1]
    s = f32(mlp.sigmoid(z))
    if loss == "bce":
        dz = round_to(f32(s - labels), fmt)
    else:
        dz = round_to(f32(f32(f32(2.0 * f32(s - labels)) * s) * f32(1.0 - s)), fmt)
    delta = dz
    gw = [None] * len(Wr)
    for k in range(len(Wr) - 1, -1, -1):
        W, hk = Wr[k], hs[k]
        prod = delta[:, :, None] * hk[:, None, :]
        gw[k] = seq_sum(f32(prod) if fmt == "f32" else prod, 0, rng) / labels.size
        dprod = delta[:, :, None] * W[None, :, :]
        d = seq_sum(f32(dprod) if fmt == "f32" else dprod, 1, rng)
        if k > 0:
            mask = pres[k - 1] > 0
            delta = round_to(np.where(mask, d, f32(slope * d) if act == "leaky" else 0.0), fmt)
        else:
            d_enc = d
    gt = np.zeros_like(table, dtype=np.float64)
    for l, (idx, w) in enumerate(corners):
        terms = f32(w[:, :, None] * d_enc[:, None, l * F:(l + 1) * F]).reshape(-1, F)
        flat = idx.reshape(-1)
        for i in rng.permutation(flat.shape[0]):
            gt[l, flat[i]] = f32(gt[l, flat[i]] + terms[i])
    return f32(mlp.sigmoid(z)), gw, gt / labels.size


def make_case(seed, n=96, near_zero=True):
    rng = np.random.default_rng(seed)
    L, F, T = GRID["L"], GRID["F"], GRID["T"]
    table = rng.uniform(-1, 1, (L, T, F)).astype(np.float32)
    dims = [L * F, 16, 16, 6]
    weights = [(rng.normal(size=(o, i)) * 1.5 / np.sqrt(i)).astype(np.float32) for i, o in zip(dims[:-1], dims[1:])]
    pos = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    if near_zero:
        # make hidden neuron 0 of layer 1 nearly cancel for every sample: its pre-activation sits within
        # a few FP16 ulps of zero, so the low-precision masks flip there
        enc = hashgrid.encode(pos, table, GRID["base"], GRID["growth"])
        w0 = weights[0][0].astype(np.float64)
        j = int(np.argmax(np.abs(w0)))
        pre = enc @ w0
        shift = np.median(pre / enc[:, j])
        weights[0][0, j] = np.float32(w0[j] - shift)
    y = (rng.uniform(size=(n, 6)) > 0.5).astype(np.float64)
    return pos, table, weights, y


CASES = [(s, fmt, act, loss) for s, (fmt, act, loss) in enumerate(
    [("f16", "relu", "bce"), ("f16", "leaky", "l2"), ("bf16", "relu", "bce"), ("f32", "relu", "bce"),
     ("f32", "leaky", "bce"), ("f16", "relu", "l2")])]


@pytest.mark.parametrize("seed,fmt,act,loss", CASES)
def test_emulated_arithmetic_stays_within_the_bounds(seed, fmt, act, loss):
    pos, table, weights, y = make_case(seed)
    slope = 0.01
    b = bounds.gradient_error_bounds(pos, table, weights, GRID["base"], GRID["growth"], labels=y, loss=loss, act=act,
                                     slope=slope, dtype=fmt)
    v_ref, e_v = bounds.visibility_error_bound(pos, table, weights, GRID["base"], GRID["growth"], act=act,
                                               slope=slope, dtype=fmt, out_dtype="f32")
    exact = training.train_gradients(pos, table, weights, GRID["base"], GRID["growth"], labels=y, loss=loss, act=act,
                                     slope=slope)
    for a, r in zip(b["g_w"], exact["g_w"]):            # the bound module's exact values are the oracle's
        assert np.allclose(a, r, rtol=1e-12, atol=1e-15)
    assert np.allclose(b["g_table"], exact["g_table"], rtol=1e-12, atol=1e-15)
    worst = []
    for rep in range(3):                                # three random summation orders
        rng = np.random.default_rng(1000 * seed + rep)
        v, gw, gt = emulate(pos, table, weights, y, fmt, act, slope, loss, rng)
        assert np.all(np.abs(v - v_ref) <= e_v)
        for k, (g, r, e) in enumerate(zip(gw, b["g_w"], b["e_w"])):
            err = np.abs(g - r)
            assert np.all(err <= e), (fmt, k, float((err / e).max()))
            worst.append(float((err / np.maximum(e, 1e-300)).max()))
        err = np.abs(gt - b["g_table"])
        assert np.all(err <= b["e_table"])
        worst.append(float((err / np.maximum(b["e_table"], 1e-300)).max()))
    # not vacuous: the worst entry uses a stated share of its bound
    assert max(worst) > (1e-2 if fmt != "f32" else 1e-3), max(worst)


def test_bounds_vanish_in_exact_arithmetic(monkeypatch):
    pos, table, weights, y = make_case(7, near_zero=False)
    monkeypatch.setattr(bounds, "U32", 0.0)
    monkeypatch.setattr(bounds, "SIGMOID_REL", 0.0)
    monkeypatch.setattr(bounds, "FIXED_RES", 0.0)
    monkeypatch.setitem(bounds.UNIT_ROUNDOFF, "f16", 0.0)
    monkeypatch.setitem(bounds.FLUSH, "f16", 0.0)
    b = bounds.gradient_error_bounds(pos, table, weights, GRID["base"], GRID["growth"], labels=y, dtype="f16")
    assert all(np.all(e == 0) for e in b["e_w"]) and np.all(b["e_table"] == 0)
    _, e_v = bounds.visibility_error_bound(pos, table, weights, GRID["base"], GRID["growth"], dtype="f16")
    assert np.all(e_v == 0)


def test_flipped_masks_are_charged_in_full():
    """A hidden neuron whose exact pre-activation is zero may take either branch in any arithmetic: the bound
    of the gradients below it then includes the whole back-propagated value, not a rounding of it."""
    pos, table, weights, y = make_case(3, near_zero=False)
    w = [x.copy() for x in weights]
    w[0][0] = 0.0                                        # neuron 0 of layer 1: pre-activation exactly 0
    b = bounds.gradient_error_bounds(pos, table, w, GRID["base"], GRID["growth"], labels=y, dtype="f32")
    exact = training.train_gradients(pos, table, w, GRID["base"], GRID["growth"], labels=y, act="relu")
    # with the mask open, row 0 of the first layer's gradient would be delta_0^T enc; the bound covers it
    enc = hashgrid.encode(pos, table, GRID["base"], GRID["growth"])
    z, pre, inputs = mlp.forward(enc, [x.astype(np.float64) for x in w])
    dz = (mlp.sigmoid(z) - y) / y.size
    d1 = dz @ w[2].astype(np.float64) * (pre[1] > 0)
    d0 = d1 @ w[1].astype(np.float64)
    row_open = d0[:, 0] @ enc
    assert np.all(np.abs(row_open - exact["g_w"][0][0]) <= b["e_w"][0][0])
    assert b["e_w"][0][0].max() > 1e-3 * np.abs(row_open).max()
