"""Host-side logic of bench.py (no GPU): the one-GPU guard, the
algorithmic FLOP model behind the roofline, and the rule that a stored
HBM-traffic measurement is reported only for the sources it was taken on.

The FLOP model is pinned against torch's own operation counter
(torch.utils.flop_counter) run on torch graphs of the same shapes, forward
and backward, with every operand that the online update differentiates
requiring a gradient: an independent count, not the formula retyped.
"""
import importlib.util
import os
import subprocess
import sys

import pytest
import torch
from torch.utils.flop_counter import FlopCounterMode

from synth.workloads import cfg1, cfg2, cfg4, tf_paper

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _count(fn) -> int:
    with FlopCounterMode(display=False) as fc:
        fn()
    return fc.get_total_flops()


def _mlp_row_flops(dims) -> int:
    """One row through Linear layers (ReLU between), forward and backward,
    the input (the context embeddings) differentiated for the embedding
    update."""
    torch.manual_seed(0)
    x = torch.randn(1, dims[0], dtype=torch.float64, requires_grad=True)
    layers = [torch.nn.Linear(dims[i], dims[i + 1], dtype=torch.float64) for i in range(len(dims) - 1)]

    def run():
        h = x
        for i, lay in enumerate(layers):
            h = lay(h)
            if i + 1 < len(layers):
                h = torch.relu(h)
        torch.log_softmax(h, dim=-1)[0, 0].neg().backward()
    return _count(run)


@pytest.mark.parametrize("make", [cfg1, cfg4], ids=["cfg1", "cfg4"])
def test_mlp_flops_per_row_matches_torch_count(bench, make):
    _, cfg = make() if make is cfg1 else make(n=1 << 20, n_blocks=1)
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [4 ** cfg["k"]]
    assert bench.flops_per_row(cfg) == _mlp_row_flops(dims)


def test_static_public_mlp_adds_one_forward(bench):
    """The frozen static model of the same shape adds its forward only."""
    _, cfg = cfg2(n=1 << 20, n_blocks=1)
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [4 ** cfg["k"]]
    torch.manual_seed(0)
    x = torch.randn(1, dims[0], dtype=torch.float64)
    layers = [torch.nn.Linear(dims[i], dims[i + 1], dtype=torch.float64) for i in range(len(dims) - 1)]

    def fwd():
        with torch.no_grad():
            h = x
            for lay in layers:
                h = lay(h)
    assert bench.flops_per_row(cfg) == _mlp_row_flops(dims) + _count(fwd)


def test_transformer_flops_per_row_matches_torch_count(bench):
    """Sec. 4.2.4's model at the last position: K and V for the t context
    positions, q for the last, per-head scores and weighted sum, the output
    projection, the FFN and the head; backward through all of it."""
    _, cfg = tf_paper(n=1 << 20, n_blocks=1)
    t, E, (A, F), H = cfg["t"], cfg["E"], cfg["hidden"], cfg["heads"]
    V, dh = 4 ** cfg["k"], A // H
    torch.manual_seed(0)
    f64 = dict(dtype=torch.float64)
    X = torch.randn(t, E, **f64, requires_grad=True)
    Wkv = torch.randn(E, 2 * A, **f64, requires_grad=True)
    Wq = torch.randn(E, A, **f64, requires_grad=True)
    Wo = torch.randn(A, A, **f64, requires_grad=True)
    W1 = torch.randn(A, F, **f64, requires_grad=True)
    W2 = torch.randn(F, A, **f64, requires_grad=True)
    Wh = torch.randn(A, V, **f64, requires_grad=True)

    def run():
        kv = X @ Wkv                                         # t x 2A
        k = kv[:, :A].reshape(t, H, dh).transpose(0, 1)      # H x t x dh
        v = kv[:, A:].reshape(t, H, dh).transpose(0, 1)
        q = (X[t - 1:] @ Wq).reshape(H, 1, dh)               # last position only
        p = torch.softmax(torch.bmm(q, k.transpose(1, 2)) / dh ** 0.5, dim=-1)
        z = torch.bmm(p, v).reshape(1, A) @ Wo
        u = torch.relu(z @ W1) @ W2
        torch.log_softmax(u @ Wh, dim=-1)[0, 0].neg().backward()
    assert bench.flops_per_row(cfg) == _count(run)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_stored_traffic_only_for_matching_sources(bench, monkeypatch, tmp_path):
    import json
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic_x.json").write_text(json.dumps({"kernel_source_sha256": bench.kernel_source_hash(),
                                                     "hbm_bytes_per_launch": 1234}))
    (prof / "traffic_y.json").write_text(json.dumps({"kernel_source_sha256": "0" * 64, "hbm_bytes_per_launch": 99}))
    real_hash = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: real_hash)
    assert bench.stored_traffic("traffic_x") == 1234
    assert bench.stored_traffic("traffic_y") is None          # taken on other sources
    assert bench.stored_traffic("traffic_z") is None          # never measured


@pytest.mark.parametrize("layers", [1, 2])
def test_bigru_static_flops_match_torch_count(bench, layers):
    """The BiGRU static model (Sec. 4.2.2) adds its forward: per layer and
    direction, the input and recurrent gate products at every context
    position, then the Dense layer on both directions' final states and the
    head. The GRU cell is written out as products so the counter sees each."""
    from synth.workloads import bigru_private
    _, cfg = bigru_private(n=1 << 20, n_blocks=1)
    cfg = dict(cfg, gru_layers=layers)
    dims = [cfg["t"] * cfg["E"]] + list(cfg["hidden"]) + [4 ** cfg["k"]]
    t, E, h, gd, V = cfg["t"], cfg["static_E"], cfg["gru_h"], cfg["dense"], 4 ** cfg["k"]
    torch.manual_seed(0)
    f64 = dict(dtype=torch.float64)

    def gru_dir(xs, Wih, Whh, reverse):
        hs, hcur = [None] * len(xs), torch.zeros(1, h, **f64)
        for j in (range(len(xs) - 1, -1, -1) if reverse else range(len(xs))):
            gi, gh = xs[j] @ Wih, hcur @ Whh
            r = torch.sigmoid(gi[:, :h] + gh[:, :h])
            z = torch.sigmoid(gi[:, h:2 * h] + gh[:, h:2 * h])
            n = torch.tanh(gi[:, 2 * h:] + r * gh[:, 2 * h:])
            hcur = (1 - z) * n + z * hcur
            hs[j] = hcur
        return hs

    def fwd():
        with torch.no_grad():
            xs = [torch.randn(1, E, **f64) for _ in range(t)]
            for l in range(layers):
                n_in = E if l == 0 else 2 * h
                fw = gru_dir(xs, torch.randn(n_in, 3 * h, **f64), torch.randn(h, 3 * h, **f64), False)
                bw = gru_dir(xs, torch.randn(n_in, 3 * h, **f64), torch.randn(h, 3 * h, **f64), True)
                xs = [torch.cat([fw[j], bw[j]], dim=1) for j in range(t)]
            last = torch.cat([fw[t - 1], bw[0]], dim=1)
            torch.relu(last @ torch.randn(2 * h, gd, **f64)) @ torch.randn(gd, V, **f64)
    assert bench.flops_per_row(cfg) == _mlp_row_flops(dims) + _count(fwd)
