"""Pins for the oracle's one-layer BiGRU static private model (Sec. 4.2.2
shape, Sec. 4.2.3 training on the input).

  * the gradient of one learning step (mean cross-entropy of the rows'
    targets) against torch autograd through torch.nn.GRU (bidirectional,
    one layer, FP64) and the two dense layers, at 1e-12 per coordinate:
    torch's back-propagation through time is independent of the oracle's;
  * central finite differences of the loss on sampled coordinates of every
    tensor (1e-7 relative);
  * the private model stored in the container equals a torch FP64 replay of
    its training from the definitions (segment j of the training block from
    token floor(j l / bs) of the input's tokens, Lp = min(floor(l / bs),
    8192) steps, the first t uniform, one update per step from the mean loss
    of the bs rows, seed ^ 0x5350524D), SGD and Adam, rounded to FP32;
  * containers: round trip, the BiGRU shape in the header, the private
    model's CRC checked on decode; two layers refused for the private model.
"""
import numpy as np
import pytest
import torch

import synth
from synth.workloads import model_small
from tests import cbf


def _cfg(**kw):
    c = model_small(t=6, E=4, hidden=[8], bs=4, selector="sprm_dm", static_arch="bigru", static_E=5, gru_h=7,
                    gru_layers=1, dense=9)
    c.update(kw)
    return c


def _torch_model(cfg, ws):
    """(parameters as leaf tensors in the oracle's flat order, forward fn)."""
    V, E, h, D, t = 4 ** cfg["k"], cfg["static_E"], cfg["gru_h"], cfg["dense"], cfg["t"]
    w = torch.tensor(ws, dtype=torch.float64)
    off = [0]
    leaves = []

    def take(*shape):
        n = int(np.prod(shape))
        x = w[off[0]:off[0] + n].view(*shape).clone().requires_grad_(True)
        off[0] += n
        leaves.append(x)
        return x
    emb = take(V, E)
    gru = torch.nn.GRU(E, h, num_layers=1, bidirectional=True, batch_first=True, dtype=torch.float64)
    names = []
    for sfx in ["", "_reverse"]:
        for nm, shp in [("weight_ih_l0", (3 * h, E)), ("weight_hh_l0", (3 * h, h)), ("bias_ih_l0", (3 * h,)),
                        ("bias_hh_l0", (3 * h,))]:
            names.append((nm + sfx, take(*shp)))
    Wd, bd = take(2 * h, D), take(D)
    Wl, bl = take(D, V), take(V)
    assert off[0] == w.numel()

    def fwd(ctx):
        params = {n: p for n, p in names}
        x = emb[torch.as_tensor(ctx, dtype=torch.long)]
        _, hn = torch.func.functional_call(gru, params, (x,))
        feat = torch.cat([hn[0], hn[1]], dim=1)        # forward after t-1, backward after 0
        return torch.relu(feat @ Wd + bd) @ Wl + bl
    return leaves, fwd


def _loss(fwd, ctx, tgt):
    return torch.nn.functional.cross_entropy(fwd(ctx), torch.as_tensor(tgt, dtype=torch.long))


@pytest.mark.parametrize("kw", [dict(), dict(t=1, gru_h=3), dict(k=3, t=9, static_E=16, gru_h=12, dense=20),
                                dict(k=2, t=4, static_E=3, gru_h=2, dense=1)])
def test_gradient_matches_torch_autograd(orc, kw):
    cfg = _cfg(**kw)
    rng = np.random.default_rng(1)
    n = orc.static_param_count(cfg)
    ws = orc.static_init(cfg, 11) + rng.normal(0, 0.1, n)
    V = 4 ** cfg["k"]
    ctx = rng.integers(0, V, size=(13, cfg["t"]), dtype=np.uint8)
    tgt = rng.integers(0, V, size=13, dtype=np.uint8)
    P, g, loss = orc.static_step(cfg, ws, ctx, tgt)
    leaves, fwd = _torch_model(cfg, ws)
    L = _loss(fwd, ctx, tgt)
    L.backward()
    gt = torch.cat([x.grad.reshape(-1) for x in leaves]).numpy()
    assert abs(L.item() - loss) <= 1e-12
    np.testing.assert_allclose(P, torch.softmax(fwd(ctx), 1).detach().numpy(), rtol=0, atol=1e-13)
    np.testing.assert_allclose(g, gt, rtol=0, atol=1e-12)


def test_gradient_finite_differences(orc):
    cfg = _cfg()
    rng = np.random.default_rng(2)
    n = orc.static_param_count(cfg)
    ws = orc.static_init(cfg, 12) + rng.normal(0, 0.1, n)
    ctx = rng.integers(0, 64, size=(5, cfg["t"]), dtype=np.uint8)
    tgt = rng.integers(0, 64, size=5, dtype=np.uint8)
    _, g, _ = orc.static_step(cfg, ws, ctx, tgt)
    # every tensor of the layout gets sampled coordinates (embedding rows of
    # the context tokens, both directions' gate weights and biases, Dense, head)
    V, E, h, D = 64, 5, 7, 9
    sizes = [V * E] + [3 * h * E, 3 * h * h, 3 * h, 3 * h] * 2 + [2 * h * D, D, D * V, V]
    starts = np.cumsum([0] + sizes)
    idx = []
    for a, b in zip(starts[:-1], starts[1:]):
        idx += list(rng.choice(np.arange(a, b), size=min(4, b - a), replace=False))
    idx += [int(ctx[0, 0]) * E + e for e in range(E)]
    for i in idx:
        e = 1e-6
        wp, wm = ws.copy(), ws.copy()
        wp[i] += e
        wm[i] -= e
        fd = (orc.static_step(cfg, wp, ctx, tgt)[2] - orc.static_step(cfg, wm, ctx, tgt)[2]) / (2 * e)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def _replay(orc, cfg, tokens):
    """The private model's training from the definitions, torch FP64."""
    bs, t = cfg["bs"], cfg["t"]
    l = len(tokens)
    Lp = min(l // bs, 8192)
    blk = np.stack([tokens[(j * l) // bs:(j * l) // bs + Lp] for j in range(bs)])
    ws0 = orc.static_init(cfg, cfg["seed"] ^ 0x5350524D)
    leaves, fwd = _torch_model(cfg, ws0)
    if cfg["optimizer"] == "adam":
        opt = torch.optim.Adam(leaves, lr=np.float32(cfg["lr"]).item(), betas=(np.float32(cfg["beta1"]).item(),
                               np.float32(cfg["beta2"]).item()), eps=np.float32(cfg["eps"]).item())
    else:
        opt = torch.optim.SGD(leaves, lr=np.float32(cfg["lr"]).item())
    for i in range(t, Lp):
        opt.zero_grad()
        _loss(fwd, blk[:, i - t:i], blk[:, i]).backward()
        opt.step()
    return torch.cat([x.detach().reshape(-1) for x in leaves]).numpy()


@pytest.mark.parametrize("opt", [dict(optimizer="sgd", lr=0.05), dict(optimizer="adam", lr=0.01)])
def test_training_matches_torch_replay(orc, opt):
    bl = [700, 747]
    cfg = _cfg(k=3, s=3, t=5, bs=6, block_len=bl, **opt)
    a = synth.generate(synth.Recipe(n=sum(bl), order=2, seed=91, rho=0.05))
    blob = orc.compress(cfg, a)
    stored = np.frombuffer(cbf.parse(blob)["private"], dtype=np.float32)
    tok = np.concatenate([orc.encode_skmer(a[:bl[0]], 3, 3), orc.encode_skmer(a[bl[0]:], 3, 3)])
    want = _replay(orc, cfg, tok)
    assert stored.size == want.size == orc.static_param_count(cfg)
    np.testing.assert_allclose(stored, want.astype(np.float32), rtol=2e-7, atol=1e-9)
    assert not np.allclose(stored, orc.static_init(cfg, cfg["seed"] ^ 0x5350524D).astype(np.float32))


def test_container(orc):
    a = synth.generate(synth.Recipe(n=9000, order=2, seed=92, n_rate=0.002, n_max=20))
    cfg = _cfg(k=3, s=3, t=5, bs=8, n_blocks=2, lr=0.01)
    blob = orc.compress(cfg, a)
    assert blob[40] == 6 and blob[43] == 1 | (1 << 4)
    assert blob[60] == 5 and blob[61] == 7 and blob[62] | (blob[63] << 8) == 9
    assert np.array_equal(orc.decompress(blob), a)
    # the stored model is covered by the header's CRC
    bad = bytearray(blob)
    bad[cbf.parse(blob)["header"]["meta_start"] - 5] ^= 1
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(bytes(bad))
    assert e.value.code == -4
    # the Model Selector picks it above its size bound
    auto = orc.compress(dict(cfg, selector="auto", ms_threshold=1000), a)
    assert auto[40] == 6 and auto == blob
    with pytest.raises(orc.OracleError) as e:
        orc.compress(dict(cfg, gru_layers=2), a)
    assert e.value.code == -1


@pytest.mark.parametrize("n", [20, 3 * 8 * 5 + 2])
def test_short_inputs_store_the_initialisation(orc, n):
    """Fewer tokens than bs (no training block) or fewer steps than t (no
    learned step): the stored model is the seeded initialisation."""
    cfg = _cfg(k=3, s=3, t=5, bs=8, n_blocks=1)
    a = synth.generate(synth.Recipe(n=n, order=2, seed=93))
    blob = orc.compress(cfg, a)
    stored = np.frombuffer(cbf.parse(blob)["private"], dtype=np.float32)
    init = orc.static_init(cfg, cfg["seed"] ^ 0x5350524D).astype(np.float32)
    assert np.array_equal(stored, init)
    assert np.array_equal(orc.decompress(blob), a)

