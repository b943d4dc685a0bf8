"""Pins for the oracle's Transformer dynamic model (Sec. 4.2.4).

The model, as read: x_p = Emb[c_p] + Pos[p]; [q|k|v]_p = x_p Wqkv + bqkv;
per head, the last position's query attends over all t positions with
scale 1/sqrt(dh); o = concat of the heads; z = o Wo + bo;
u = ReLU(z W1 + b1); g = u W2 + b2; logits = g Wh + bh.

  * forward and gradient against torch FP64 autograd on the same graph,
    the attention taken by torch's own scaled_dot_product_attention (a
    library routine independent of the oracle's loops), for several head
    counts, context lengths and widths, at 1e-12;
  * central finite differences on sampled coordinates of every tensor;
  * closed forms: with t = 1 the attention returns v_0 exactly; with zero
    key weights and biases it averages v over the positions;
  * the learning loop replayed from the definitions (SGD and Adam) equals
    trace_block's probabilities and final parameters;
  * round trips of the container, its header fields, and error paths.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import synth
from synth.workloads import model_small


def _cfg(t=5, E=6, A=8, F=12, heads=2, k=2, bs=4, **kw):
    c = model_small(s=k, k=k, t=t, E=E, hidden=[A, F], bs=bs, arch="transformer", heads=heads)
    c.update(kw)
    return c


def _tf(flat, ctx, cfg):
    """Logits [rows, V] of the model for integer contexts [rows, t]."""
    V, E, t, (A, F), H = 4 ** cfg["k"], cfg["E"], cfg["t"], cfg["hidden"], cfg["heads"]
    dh = A // H
    off = [0]

    def take(*shape):
        n = int(np.prod(shape))
        x = flat[off[0]:off[0] + n].view(*shape)
        off[0] += n
        return x
    emb, pos = take(V, E), take(t, E)
    Wqkv, bqkv = take(E, 3 * A), take(3 * A)
    Wo, bo = take(A, A), take(A)
    W1, b1 = take(A, F), take(F)
    W2, b2 = take(F, A), take(A)
    Wh, bh = take(A, V), take(V)
    assert off[0] == flat.numel()
    rows = ctx.shape[0]
    x = Fn.embedding(torch.as_tensor(ctx, dtype=torch.long), emb) + pos          # [rows, t, E]
    qkv = x @ Wqkv + bqkv
    q, k, v = qkv[..., :A], qkv[..., A:2 * A], qkv[..., 2 * A:]
    heads = lambda y: y.reshape(rows, y.shape[1], H, dh).transpose(1, 2)        # [rows, H, len, dh]
    o = Fn.scaled_dot_product_attention(heads(q[:, -1:, :]), heads(k), heads(v))  # [rows, H, 1, dh]
    o = o.transpose(1, 2).reshape(rows, A)
    z = o @ Wo + bo
    u = torch.relu(z @ W1 + b1)
    g = u @ W2 + b2
    return g @ Wh + bh


def _random_case(orc, cfg, seed):
    rng = np.random.default_rng(seed)
    V, bs, t = 4 ** cfg["k"], cfg["bs"], cfg["t"]
    w = orc.init_params(cfg) + rng.normal(0, 0.05, orc.param_count(cfg))
    ctx = rng.integers(0, V, size=(bs, t), dtype=np.uint8)
    tgt = rng.integers(0, V, size=bs, dtype=np.uint8)
    return w, ctx, tgt


SHAPES = [dict(), dict(heads=1), dict(heads=4, A=8), dict(t=1), dict(t=9, E=3, A=6, F=5, heads=3),
          dict(k=3, t=4, E=4, A=16, F=32, heads=4, bs=6)]


@pytest.mark.parametrize("kw", SHAPES)
def test_step_matches_torch_autograd(orc, kw):
    cfg = _cfg(**kw)
    w, ctx, tgt = _random_case(orc, cfg, 1)
    P, g, _, loss = orc.step(cfg, w, ctx, tgt)
    wt = torch.tensor(w, requires_grad=True)
    logits = _tf(wt, ctx, cfg)
    lt = Fn.cross_entropy(logits, torch.as_tensor(tgt, dtype=torch.long))
    lt.backward()
    np.testing.assert_allclose(P, torch.softmax(logits, 1).detach().numpy(), rtol=0, atol=1e-12)
    assert abs(loss - lt.item()) <= 1e-12
    gt = wt.grad.numpy()
    np.testing.assert_allclose(g, gt, rtol=0, atol=1e-12 * max(1.0, np.abs(gt).max()))
    for name, (off, shp) in orc.param_slices(cfg).items():
        # every tensor receives gradient
        assert np.abs(g[off:off + int(np.prod(shp))]).max() > 0, name


def test_gradient_against_finite_differences(orc):
    cfg = _cfg(t=4, E=5, A=6, F=7, heads=3, bs=3)
    w, ctx, tgt = _random_case(orc, cfg, 2)
    _, g, _, _ = orc.step(cfg, w, ctx, tgt)
    rng = np.random.default_rng(0)
    h = 1e-6
    for name, (off, shp) in orc.param_slices(cfg).items():
        n = int(np.prod(shp))
        cand = np.flatnonzero(np.abs(g[off:off + n]) > 1e-6) + off
        for i in rng.choice(cand, size=min(5, len(cand)), replace=False):
            wp, wm = w.copy(), w.copy()
            wp[i] += h
            wm[i] -= h
            fd = (orc.step(cfg, wp, ctx, tgt, grad=False)[3] - orc.step(cfg, wm, ctx, tgt, grad=False)[3]) / (2 * h)
            assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd)), (name, i, g[i], fd)


def test_single_position_attends_to_itself(orc):
    """t = 1: softmax over one score is 1, so o = v_0 exactly."""
    cfg = _cfg(t=1, E=4, A=6, F=5, heads=2, bs=5)
    w, ctx, tgt = _random_case(orc, cfg, 3)
    P, _, _, _ = orc.step(cfg, w, ctx, tgt, grad=False)
    S = orc.param_slices(cfg)
    get = lambda name: w[S[name][0]:S[name][0] + int(np.prod(S[name][1]))].reshape(S[name][1])
    A = 6
    x = get("emb")[ctx[:, 0]] + get("pos")[0]
    v = x @ get("Wqkv")[:, 2 * A:] + get("bqkv")[2 * A:]
    z = v @ get("Wo") + get("bo")
    u = np.maximum(z @ get("W1") + get("b1"), 0)
    logits = (u @ get("W2") + get("b2")) @ get("Wh") + get("bh")
    e = np.exp(logits - logits.max(1, keepdims=True))
    np.testing.assert_allclose(P, e / e.sum(1, keepdims=True), rtol=0, atol=1e-13)


def test_zero_keys_average_the_values(orc):
    """Zero key weights and biases: every score is 0, the attention is
    uniform and o is the mean of v over the t positions."""
    cfg = _cfg(t=6, E=4, A=8, F=5, heads=4, bs=4)
    w, ctx, tgt = _random_case(orc, cfg, 4)
    S = orc.param_slices(cfg)
    A = 8
    o_w, _ = S["Wqkv"]
    Wqkv = w[o_w:o_w + 4 * 3 * A].reshape(4, 3 * A)
    Wqkv[:, A:2 * A] = 0.0
    o_b, _ = S["bqkv"]
    w[o_b + A:o_b + 2 * A] = 0.0
    P, _, _, _ = orc.step(cfg, w, ctx, tgt, grad=False)
    get = lambda name: w[S[name][0]:S[name][0] + int(np.prod(S[name][1]))].reshape(S[name][1])
    x = get("emb")[ctx] + get("pos")                                   # [rows, t, E]
    v = x @ get("Wqkv")[:, 2 * A:] + get("bqkv")[2 * A:]
    o = v.mean(axis=1)
    z = o @ get("Wo") + get("bo")
    u = np.maximum(z @ get("W1") + get("b1"), 0)
    logits = (u @ get("W2") + get("b2")) @ get("Wh") + get("bh")
    e = np.exp(logits - logits.max(1, keepdims=True))
    np.testing.assert_allclose(P, e / e.sum(1, keepdims=True), rtol=0, atol=1e-12)


def _replay(cfg, tok, init, stop, probe_steps):
    V, t, bs = 4 ** cfg["k"], cfg["t"], cfg["bs"]
    L = len(tok) // bs
    n = len(init) - 1
    w = torch.tensor(init[:n], dtype=torch.float64, requires_grad=True)
    lr = float(np.float32(cfg["lr"]))
    if cfg["optimizer"] == "adam":
        opt = torch.optim.Adam([w], lr=lr, betas=(float(np.float32(cfg["beta1"])), float(np.float32(cfg["beta2"]))),
                               eps=float(np.float32(cfg["eps"])))
    else:
        opt = torch.optim.SGD([w], lr=lr)
    probes = {}
    for i in range(stop):
        if i < t:
            if i in probe_steps:
                probes[i] = np.full((bs, V), 1.0 / V)
            continue
        ctx = np.array([[tok[j * L + i - t + p] for p in range(t)] for j in range(bs)], dtype=np.int64)
        tgt = np.array([tok[j * L + i] for j in range(bs)], dtype=np.int64)
        opt.zero_grad()
        z = _tf(w, ctx, cfg)
        if i in probe_steps:
            probes[i] = torch.softmax(z, dim=1).detach().numpy()
        Fn.cross_entropy(z, torch.as_tensor(tgt)).backward()
        opt.step()
    return np.stack([probes[s] for s in sorted(probe_steps)]), w.detach().numpy()


@pytest.mark.parametrize("optimizer,lr", [("sgd", 0.05), ("adam", 0.01)])
def test_learning_loop_matches_definition_replay(orc, optimizer, lr):
    cfg = _cfg(t=3, E=4, A=6, F=5, heads=2, bs=3, optimizer=optimizer, lr=lr)
    rng = np.random.default_rng(13)
    V, bs, t = 16, 3, 3
    L = t + 6
    tok = rng.integers(0, V, size=bs * L + 1, dtype=np.uint8)
    n = orc.param_count(cfg)
    init = np.concatenate([orc.init_params(cfg), [0.0]])
    stop = t + 4
    steps = [t - 1, t, t + 2, t + 3]
    P_or, _, w_or = orc.trace_block(cfg, tok, steps=steps, init=init, stop=stop)
    P_ref, w_ref = _replay(cfg, tok, init, stop, set(steps))
    np.testing.assert_allclose(P_or, P_ref, rtol=0, atol=1e-12)
    # Adam divides by sqrt(v): coordinates whose gradient is near zero carry
    # the summation-order difference (~1e-16 relative, torch's batched
    # products against per-row sums) into the update magnified
    np.testing.assert_allclose(w_or[:n], w_ref, rtol=0, atol=1e-12 if optimizer == "sgd" else 1e-10)
    assert np.abs(w_or[:n] - init[:n]).max() > 1e-3


def test_container_round_trip_and_header(orc):
    a = synth.generate(synth.Recipe(n=5000, order=2, seed=80, n_rate=0.002, n_max=20))
    cfg = _cfg(t=4, E=4, A=8, F=16, heads=2, k=3, bs=8, n_blocks=2, lr=0.01)
    blob = orc.compress(cfg, a)
    h = blob[40:44]
    assert h[0] == 4 and h[1] == 1 and h[2] == 2 and h[3] == 0     # selector DM, arch 1, 2 heads
    assert np.array_equal(orc.decompress(blob), a)
    mlp = orc.compress(model_small(s=3, k=3, t=4, E=4, hidden=[8], bs=8, n_blocks=2), a)
    assert mlp[41:44] == b"\0\0\0"
    for kw in [dict(optimizer="adam"), dict(n_blocks=3, smp_ppm=50000), dict(selector="uniform")]:
        c = dict(cfg, **kw)
        assert np.array_equal(orc.decompress(orc.compress(c, a)), a), kw


def test_errors(orc):
    a = synth.generate(synth.Recipe(n=2000, order=2, seed=81))
    for bad in [dict(selector="spum_dm"), dict(selector="sprm_dm"), dict(heads=3), dict(hidden=[8])]:
        with pytest.raises(orc.OracleError) as e:
            orc.compress(_cfg(k=3, **bad), a, static=np.zeros(10, np.float32))
        assert e.value.code == -1, bad
