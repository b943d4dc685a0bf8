"""Pin of the oracle's learning loop: segments, context windows, targets and
the order of forward, coding and update (Sec. 2 steps (2)-(4)).

The reference here is a replay written from the definitions alone, in
torch FP64 on the CPU: a block's first bs*L tokens form bs contiguous
segments of L tokens; at step i, row j predicts token j*L + i from the t
tokens before it, {x_(jL+i-t), ..., x_(jL+i-1)} oldest first; the first t
steps of every segment are coded uniformly and do not train; every later
step makes one update from the mean cross-entropy of its bs rows (SGD, or
torch.optim.Adam for the Adam form), the mixing weight included when a
static model is mixed in (Eq. 1). The replay's probabilities at sampled
steps and its parameters after the last step must equal the oracle's
trace_block. A context window moved by one token, a segment stride off by
one, a wrong target or an update taken before the coding step all fail it.
"""
import numpy as np
import pytest
import torch

from synth.workloads import model_small

CASES = [
    dict(name="sgd_dm", optimizer="sgd", lr=0.05, selector="dm"),
    dict(name="adam_dm", optimizer="adam", lr=0.01, selector="dm"),
    dict(name="sgd_static", optimizer="sgd", lr=0.05, selector="spum_dm"),
]


def _mlp(flat, ctx, V, E, dims):
    off = 0
    emb = flat[off:off + V * E].view(V, E)
    off += V * E
    h = torch.nn.functional.embedding(torch.as_tensor(ctx, dtype=torch.long), emb).reshape(len(ctx), -1)
    for l in range(len(dims) - 1):
        W = flat[off:off + dims[l] * dims[l + 1]].view(dims[l], dims[l + 1])
        off += dims[l] * dims[l + 1]
        b = flat[off:off + dims[l + 1]]
        off += dims[l + 1]
        h = h @ W + b
        if l < len(dims) - 2:
            h = torch.relu(h)
    return h


def _replay(cfg, tok, init, static, stop, probe_steps):
    """The learning loop from the definitions; returns (P at probe steps, params after `stop` steps)."""
    V, E, t, bs = 4 ** cfg["k"], cfg["E"], cfg["t"], cfg["bs"]
    dims = [t * E] + list(cfg["hidden"]) + [V]
    L = len(tok) // bs
    n = len(init) - 1
    mixed = static is not None
    w = torch.tensor(init[:n], dtype=torch.float64, requires_grad=True)
    a = torch.tensor(init[n], dtype=torch.float64, requires_grad=True)
    params = [w, a] if mixed else [w]
    lr = float(np.float32(cfg["lr"]))
    if cfg["optimizer"] == "adam":
        opt = torch.optim.Adam(params, lr=lr, betas=(float(np.float32(cfg["beta1"])), float(np.float32(cfg["beta2"]))),
                               eps=float(np.float32(cfg["eps"])))
    else:
        opt = torch.optim.SGD(params, lr=lr)
    ws = None if static is None else torch.tensor(static.astype(np.float64))
    probes = {}
    for i in range(stop):
        if i < t:
            if i in probe_steps:
                probes[i] = np.full((bs, V), 1.0 / V)
            continue
        ctx = np.array([[tok[j * L + i - t + p] for p in range(t)] for j in range(bs)], dtype=np.int64)
        tgt = np.array([tok[j * L + i] for j in range(bs)], dtype=np.int64)
        opt.zero_grad()
        z = _mlp(w, ctx, V, E, dims)
        if mixed:
            al = torch.sigmoid(a)
            z = al * _mlp(ws, ctx, V, E, dims) + (1 - al) * z
        if i in probe_steps:
            probes[i] = torch.softmax(z, dim=1).detach().numpy()
        loss = torch.nn.functional.cross_entropy(z, torch.as_tensor(tgt))
        loss.backward()
        opt.step()
    out = np.concatenate([w.detach().numpy(), [a.item()]])
    return np.stack([probes[s] for s in sorted(probe_steps)]), out


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_learning_loop_matches_definition_replay(orc, case):
    cfg = model_small(s=2, k=2, t=4, E=3, hidden=[5], bs=3, optimizer=case["optimizer"], lr=case["lr"],
                      selector=case["selector"])
    rng = np.random.default_rng(11)
    V, bs, t = 4 ** cfg["k"], cfg["bs"], cfg["t"]
    L = t + 6
    tok = rng.integers(0, V, size=bs * L + 2, dtype=np.uint8)   # two remainder tokens stay out of the loop
    n = orc.param_count(cfg)
    init = np.concatenate([rng.uniform(-0.8, 0.8, size=n), [0.3]])
    static = rng.uniform(-0.8, 0.8, size=n).astype(np.float32) if case["selector"] == "spum_dm" else None
    stop = t + 4                                                # four learning steps
    steps = [t - 1, t, t + 1, t + 3]
    P_or, _, w_or = orc.trace_block(cfg, tok, steps=steps, static=static, init=init, stop=stop)
    P_ref, w_ref = _replay(cfg, tok, init, static, stop, set(steps))
    np.testing.assert_allclose(P_or, P_ref, rtol=0, atol=1e-12)
    if static is None:
        np.testing.assert_allclose(w_or[:n], w_ref[:n], rtol=0, atol=1e-12)
        assert w_or[n] == init[n]          # the mixing weight is untouched without a static model
    else:
        np.testing.assert_allclose(w_or, w_ref, rtol=0, atol=1e-12)
    # the updates moved the parameters (the comparison is not vacuous)
    assert np.abs(w_or[:n] - init[:n]).max() > 1e-3


def test_replay_detects_a_shifted_window(orc):
    """The pin's own sensitivity: the same replay with the window moved one
    token later (so it contains the target) disagrees with the oracle."""
    cfg = model_small(s=2, k=2, t=4, E=3, hidden=[5], bs=3, lr=0.05)
    rng = np.random.default_rng(12)
    V, bs, t = 16, 3, 4
    L = t + 6
    tok = rng.integers(0, V, size=bs * L, dtype=np.uint8)
    n = orc.param_count(cfg)
    init = np.concatenate([rng.uniform(-0.8, 0.8, size=n), [0.0]])
    P_or, _, _ = orc.trace_block(cfg, tok, steps=[t + 2], init=init, stop=t + 3)
    shifted = np.concatenate([tok[1:], tok[:1]])   # x_(i-t+1) .. x_i: the target inside the window
    # replay on the shifted copy reads tokens one later for every position of segment j
    P_sh, _ = _replay(cfg, shifted, init, None, t + 3, {t + 2})
    assert np.abs(P_or - P_sh).max() > 1e-3
