"""Pins for the oracle's model step (forward, Eq. 1 mixer, softmax, Eq. 2
loss, hand-written backward) and optimisers.

Independent references:
  * torch FP64 on the CPU: F.embedding / F.linear / F.relu / softmax and
    torch.autograd for every gradient (the oracle's backward is hand-written);
  * central finite differences of the oracle's own loss on sampled
    coordinates of every tensor;
  * closed forms: zero weights give the uniform distribution and loss ln V;
    SGD w - lr*g; Adam's first step is -lr*g/(|g| + eps);
  * SplitMix64's published outputs for the initial weights.
"""
import os

import numpy as np
import pytest
import torch

from synth.workloads import model_small

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")

SHAPES = [
    dict(k=3, t=32, E=16, hidden=[32], bs=64),          # cfg1/3/5 model
    dict(k=2, t=5, E=3, hidden=[7], bs=6),
    dict(k=3, t=4, E=4, hidden=[8, 6], bs=5),           # two hidden layers, like cfg4
    dict(k=1, t=3, E=2, hidden=[], bs=4),               # no hidden layer
]


def _cfg(sh, **kw):
    return model_small(s=1, **sh, **kw)


def _torch_step(cfg, w, ctx, tgt, ws=None, a_alpha=0.0):
    V = 4 ** cfg["k"]
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [V]

    def mlp(flat):
        off = 0
        emb = flat[off:off + V * cfg["E"]].view(V, cfg["E"])
        off += V * cfg["E"]
        h = torch.nn.functional.embedding(torch.as_tensor(ctx, dtype=torch.long), emb).reshape(len(ctx), -1)
        for l in range(len(dims) - 1):
            W = flat[off:off + dims[l] * dims[l + 1]].view(dims[l], dims[l + 1])
            off += dims[l] * dims[l + 1]
            b = flat[off:off + dims[l + 1]]
            off += dims[l + 1]
            h = torch.nn.functional.linear(h, W.t(), b)
            if l < len(dims) - 2:
                h = torch.relu(h)
        return h

    wt = torch.tensor(w, dtype=torch.float64, requires_grad=True)
    at = torch.tensor(a_alpha, dtype=torch.float64, requires_grad=True)
    lm = mlp(wt)
    if ws is not None:
        lu = mlp(torch.tensor(ws, dtype=torch.float64))
        al = torch.sigmoid(at)
        z = al * lu + (1 - al) * lm
    else:
        z = lm
    P = torch.softmax(z, dim=1)
    loss = torch.nn.functional.cross_entropy(z, torch.as_tensor(tgt, dtype=torch.long))  # mean over rows
    loss.backward()
    ga = at.grad.item() if at.grad is not None else 0.0
    return P.detach().numpy(), wt.grad.numpy(), ga, loss.item()


def _data(cfg, rng):
    V = 4 ** cfg["k"]
    ctx = rng.integers(0, V, size=(cfg["bs"], cfg["t"]), dtype=np.uint8)
    tgt = rng.integers(0, V, size=cfg["bs"], dtype=np.uint8)
    return ctx, tgt


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("static", [False, True])
def test_step_matches_torch_autograd(orc, shape, static):
    cfg = _cfg(shape)
    rng = np.random.default_rng(11)
    w = orc.init_params(cfg) + rng.normal(0, 0.05, orc.param_count(cfg))  # break ReLU ties at 0
    ws = orc.init_params(cfg, seed=99) if static else None
    a = 0.3 if static else 0.0
    ctx, tgt = _data(cfg, rng)
    P, g, ga, loss = orc.step(cfg, w, ctx, tgt, ws=ws, a_alpha=a)
    Pt, gt, gat, losst = _torch_step(cfg, w, ctx, tgt, ws=ws, a_alpha=a)
    assert np.max(np.abs(P - Pt)) <= 1e-12
    assert abs(loss - losst) <= 1e-12
    assert np.max(np.abs(g - gt)) <= 1e-12 * max(1.0, np.max(np.abs(gt)))
    assert abs(ga - gat) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES[1:])
def test_step_gradient_central_differences(orc, shape):
    cfg = _cfg(shape)
    rng = np.random.default_rng(5)
    w = orc.init_params(cfg) + rng.normal(0, 0.05, orc.param_count(cfg))
    ws = orc.init_params(cfg, seed=7)
    ctx, tgt = _data(cfg, rng)
    a = -0.4
    _, g, ga, _ = orc.step(cfg, w, ctx, tgt, ws=ws, a_alpha=a)
    h = 1e-6
    idx = rng.choice(len(w), size=min(400, len(w)), replace=False)
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp = orc.step(cfg, wp, ctx, tgt, ws=ws, a_alpha=a, grad=False)[3]
        lm = orc.step(cfg, wm, ctx, tgt, ws=ws, a_alpha=a, grad=False)[3]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])
    lp = orc.step(cfg, w, ctx, tgt, ws=ws, a_alpha=a + h, grad=False)[3]
    lm = orc.step(cfg, w, ctx, tgt, ws=ws, a_alpha=a - h, grad=False)[3]
    assert abs((lp - lm) / (2 * h) - ga) <= 1e-7


def test_zero_model_is_uniform(orc):
    cfg = _cfg(SHAPES[0])
    w = np.zeros(orc.param_count(cfg))
    ctx, tgt = _data(cfg, np.random.default_rng(0))
    P, g, _, loss = orc.step(cfg, w, ctx, tgt)
    V = 64
    assert np.allclose(P, 1.0 / V, atol=0, rtol=1e-15)
    assert abs(loss - np.log(V)) < 1e-14
    # with all weights zero only the output bias gets a gradient: mean(P - onehot)
    sl = orc.param_slices(cfg)
    off, shp = sl["b1"]
    onehot = np.zeros((len(tgt), V))
    onehot[np.arange(len(tgt)), tgt] = 1
    assert np.allclose(g[off:off + V], (1.0 / V - onehot).mean(0), atol=1e-15)
    mask = np.ones_like(g, dtype=bool)
    mask[off:off + V] = False
    assert np.all(g[mask] == 0)


def test_output_bias_only_model(orc):
    # only the output bias non-zero: P = softmax(b) for every row, whatever the context
    cfg = _cfg(SHAPES[1])
    w = np.zeros(orc.param_count(cfg))
    off, shp = orc.param_slices(cfg)["b1"]
    b = np.random.default_rng(1).normal(size=shp)
    w[off:off + shp[0]] = b
    ctx, tgt = _data(cfg, np.random.default_rng(2))
    P = orc.step(cfg, w, ctx, tgt)[0]
    sm = np.exp(b - b.max()) / np.exp(b - b.max()).sum()
    assert np.max(np.abs(P - sm[None, :])) < 1e-15


def test_init_params_follow_splitmix64(orc):
    vals = [int(x, 16) for x in open(GOLD) if x.strip() and not x.startswith("#")]
    cfg = _cfg(SHAPES[0], seed=0)
    w = orc.init_params(cfg, seed=0)
    for i, x in enumerate(vals):  # first parameters are embedding entries (a = 1)
        u = (x >> 40) / float(1 << 24)
        assert w[i] == float(np.float32(2 * u - 1))
    # every value is an FP32 number inside +-a of its tensor
    assert np.all(w.astype(np.float32).astype(np.float64) == w)
    for name, (off, shp) in orc.param_slices(cfg).items():
        a = 1.0 if name == "emb" else 1.0 / np.sqrt(
            orc.param_slices(cfg)["W" + name[1:]][1][0] if name[0] == "b" else shp[0])
        seg = w[off:off + int(np.prod(shp))]
        assert np.all(np.abs(seg) <= a + 1e-7)
        assert np.abs(seg).max() > 0.8 * a


def test_sgd_closed_form(orc):
    rng = np.random.default_rng(3)
    w, g = rng.normal(size=50), rng.normal(size=50)
    w0 = w.copy()
    z = np.zeros(50)
    orc.opt_step(0, 1e-3, 0.9, 0.999, 1e-8, w, g, z.copy(), z.copy(), 1)
    assert np.array_equal(w, w0 - 1e-3 * g)


def test_adam_closed_form(orc):
    rng = np.random.default_rng(4)
    w, g = rng.normal(size=50), rng.normal(size=50)
    w0 = w.copy()
    m, v = np.zeros(50), np.zeros(50)
    lr, eps = 1e-3, 1e-8
    orc.opt_step(1, lr, 0.9, 0.999, eps, w, g, m, v, 1)
    assert np.allclose(w, w0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    w1 = w.copy()
    orc.opt_step(1, lr, 0.9, 0.999, eps, w, g, m, v, 2)
    assert np.allclose(w, w1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    # and it matches torch.optim.Adam
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([wt], lr=lr, betas=(0.9, 0.999), eps=eps)
    w2, m2, v2 = w0.copy(), np.zeros(50), np.zeros(50)
    for tau in range(1, 6):
        gg = rng.normal(size=50)
        wt.grad = torch.tensor(gg)
        opt.step()
        orc.opt_step(1, lr, 0.9, 0.999, eps, w2, gg, m2, v2, tau)
    assert np.allclose(w2, wt.detach().numpy(), rtol=0, atol=1e-14)
