"""Pins for the oracle's BiGRU static public model (Sec. 4.2.2).

The model, as read: a 16-d embedding, gl bidirectional GRU layers (gates
r, z, n; n = tanh(W_in x + b_in + r (W_hn h + b_hn)); h' = (1 - z) n + z h),
the last layer's final states of both directions concatenated, a Dense layer
(width 128 by default) with ReLU, a linear head to V.

  * logits against torch.nn.GRU (bidirectional, 1 and 2 layers, FP64, the
    oracle's weights loaded into it) followed by the two dense layers, at
    1e-12: torch's recurrence is independent of the oracle's loops;
  * a closed form: with all GRU weights and biases zero every state stays
    0, so the logits are Wl ReLU(bd) + bl for every context;
  * Eq. (1) with this model: the first learned step's probabilities equal
    softmax(alpha L^u + (1 - alpha) log P^m) at alpha = 1/2, L^u from the
    static forward and P^m from the dynamic model alone (the per-row
    constant of log P^m cancels in the softmax);
  * containers: round trips, header fields, the static model's size and
    CRC checked on decode; error paths.
"""
import numpy as np
import pytest
import torch

import synth
from synth.workloads import model_small


def _cfg(**kw):
    c = model_small(t=6, E=4, hidden=[8], bs=4, selector="spum_dm", static_arch="bigru", static_E=5, gru_h=7,
                    gru_layers=2, dense=9)
    c.update(kw)
    return c


def _torch_logits(cfg, ws, ctx):
    V, E, h, L, D, t = 4 ** cfg["k"], cfg["static_E"], cfg["gru_h"], cfg["gru_layers"], cfg["dense"], cfg["t"]
    w = torch.tensor(ws, dtype=torch.float64)
    off = [0]

    def take(*shape):
        n = int(np.prod(shape))
        x = w[off[0]:off[0] + n].view(*shape)
        off[0] += n
        return x
    emb = take(V, E)
    gru = torch.nn.GRU(E, h, num_layers=L, bidirectional=True, batch_first=True, dtype=torch.float64)
    with torch.no_grad():
        for l in range(L):
            inp = E if l == 0 else 2 * h
            for d, sfx in enumerate(["", "_reverse"]):
                getattr(gru, f"weight_ih_l{l}{sfx}").copy_(take(3 * h, inp))
                getattr(gru, f"weight_hh_l{l}{sfx}").copy_(take(3 * h, h))
                getattr(gru, f"bias_ih_l{l}{sfx}").copy_(take(3 * h))
                getattr(gru, f"bias_hh_l{l}{sfx}").copy_(take(3 * h))
    Wd, bd = take(2 * h, D), take(D)
    Wl, bl = take(D, V), take(V)
    assert off[0] == w.numel()
    x = emb[torch.as_tensor(ctx, dtype=torch.long)]
    _, hn = gru(x)                                     # [L * 2, rows, h]
    feat = torch.cat([hn[-2], hn[-1]], dim=1)          # last layer: forward after t-1, backward after 0
    return (torch.relu(feat @ Wd + bd) @ Wl + bl).detach().numpy()


@pytest.mark.parametrize("kw", [dict(), dict(gru_layers=1), dict(t=1, gru_h=3), dict(k=3, t=9, static_E=16,
                                                                                       gru_h=12, dense=20)])
def test_forward_matches_torch_gru(orc, kw):
    cfg = _cfg(**kw)
    rng = np.random.default_rng(1)
    n = orc.static_param_count(cfg)
    ws = orc.static_init(cfg, 11) + rng.normal(0, 0.05, n)
    ctx = rng.integers(0, 4 ** cfg["k"], size=(13, cfg["t"]), dtype=np.uint8)
    got = orc.static_forward(cfg, ws, ctx)
    want = _torch_logits(cfg, ws, ctx)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # the parameter count is torch's own
    V, E, h, L, D = 4 ** cfg["k"], cfg["static_E"], cfg["gru_h"], cfg["gru_layers"], cfg["dense"]
    gru = torch.nn.GRU(E, h, num_layers=L, bidirectional=True)
    assert n == V * E + sum(p.numel() for p in gru.parameters()) + 2 * h * D + D + D * V + V


def test_zero_recurrence_closed_form(orc):
    cfg = _cfg()
    n = orc.static_param_count(cfg)
    ws = orc.static_init(cfg, 12)
    V, E, h, D = 64, 5, 7, 9
    head = V * E
    tail = n - (2 * h * D + D + D * V + V)
    ws[head:tail] = 0.0                              # every GRU weight and bias
    ctx = np.random.default_rng(2).integers(0, V, size=(6, cfg["t"]), dtype=np.uint8)
    got = orc.static_forward(cfg, ws, ctx)
    bd = ws[tail + 2 * h * D:tail + 2 * h * D + D]
    Wl = ws[tail + 2 * h * D + D:tail + 2 * h * D + D + D * V].reshape(D, V)
    bl = ws[n - V:]
    want = np.maximum(bd, 0) @ Wl + bl
    np.testing.assert_allclose(got, np.tile(want, (6, 1)), rtol=0, atol=1e-13)


def test_mixing_with_the_bigru_model(orc):
    """First learned step (alpha = 1/2, seeded DM weights) of a block coded
    with the BiGRU static model."""
    cfg = _cfg(bs=3)
    rng = np.random.default_rng(3)
    V, t, bs = 64, cfg["t"], 3
    L = t + 5
    tok = rng.integers(0, V, size=bs * L, dtype=np.uint8)
    ws = orc.static_init(cfg, 13).astype(np.float32)
    P, _, _ = orc.trace_block(cfg, tok, steps=[t], static=ws, stop=t + 1)
    ctx = np.array([[tok[j * L + p] for p in range(t)] for j in range(bs)], dtype=np.uint8)
    tgt = np.array([tok[j * L + t] for j in range(bs)], dtype=np.uint8)
    Lu = orc.static_forward(cfg, ws.astype(np.float64), ctx)
    dm = dict(cfg, selector="dm", static_arch="mlp")
    Pm, _, _, _ = orc.step(dm, orc.init_params(dm), ctx, tgt, grad=False)
    z = 0.5 * Lu + 0.5 * np.log(Pm)
    e = np.exp(z - z.max(1, keepdims=True))
    np.testing.assert_allclose(P[0], e / e.sum(1, keepdims=True), rtol=0, atol=1e-12)


def test_container(orc):
    a = synth.generate(synth.Recipe(n=6000, order=2, seed=90, n_rate=0.002, n_max=20))
    cfg = _cfg(k=3, s=3, t=5, bs=8, n_blocks=2, lr=0.01)
    ws = orc.static_init(cfg, 14).astype(np.float32)
    blob = orc.compress(cfg, a, static=ws)
    assert blob[40] == 5 and blob[43] == 1 | (2 << 4)
    assert blob[60] == 5 and blob[61] == 7 and blob[62] | (blob[63] << 8) == 9
    assert np.array_equal(orc.decompress(blob, static=ws), a)
    assert blob != orc.compress(dict(cfg, static_arch="mlp"), a,
                                static=orc.init_params(dict(cfg, static_arch="mlp"), seed=14).astype(np.float32))
    for bad in [ws[:-1], ws + 1e-3]:
        with pytest.raises(orc.OracleError) as e:
            orc.decompress(blob, static=bad)
        assert e.value.code == -5
    with pytest.raises(orc.OracleError) as e:
        orc.compress(dict(cfg, selector="sprm_dm"), a)       # a BiGRU private model has one layer
    assert e.value.code == -1
