"""The dynamic model as a differentiable op (hand-written HIP backward with
recomputed activations, behind torch.autograd.Function), on a 4 KB slice of
the fourth workload's source with its model (t 64, E 64, hidden [256, 256],
128 rows): gradient against the FP64 oracle's hand-written backward and
against FP64 central finite differences of the oracle's loss, 1e-3 relative
tolerance."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12805_amd as P
    P.load()
    return P


def _slice_case(orc, n=4096, rows=128, seed=4):
    from synth.workloads import cfg4
    rec, cfg = cfg4(n=n, n_blocks=1)
    rec.seed = seed
    a = synth.generate(rec)
    tok = orc.encode_skmer(a, cfg["s"], cfg["k"])
    t = cfg["t"]
    ctx = np.stack([tok[j:j + t] for j in range(rows)]).astype(np.uint8)
    tgt = tok[t:t + rows].astype(np.uint8)
    w = orc.init_params(cfg)
    return cfg, ctx, tgt, w


def test_autograd_function_matches_oracle_gradient(gpu, orc):
    import torch
    from paper_2507_12805_amd.autograd import DynamicModel
    cfg, ctx, tgt, w = _slice_case(orc)
    params = torch.tensor(w, dtype=torch.float32, device="cuda", requires_grad=True)
    tokens = torch.from_numpy(ctx).cuda()
    logits = DynamicModel.apply(params, tokens, cfg)
    loss = torch.nn.functional.cross_entropy(logits, torch.from_numpy(tgt.astype(np.int64)).cuda())
    loss.backward()
    g = params.grad.detach().cpu().numpy().astype(np.float64)
    Po, go, _, loss_o = orc.step(cfg, w, ctx, tgt)
    P = torch.softmax(logits.detach().double(), dim=1).cpu().numpy()
    assert np.abs(P - Po).max() <= 1e-4
    assert abs(loss.item() - loss_o) <= 1e-4
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    assert rel <= 1e-3, rel
    # every coordinate: 1e-3 relative, with an absolute floor of 1e-5 of the
    # tensor's largest gradient for coordinates that cancel to near zero
    # (FP32 sums of up to 4096 terms)
    for name, (off, shp) in orc.param_slices(cfg).items():
        n = int(np.prod(shp))
        gs, gos = g[off:off + n], go[off:off + n]
        err = np.abs(gs - gos)
        bound = 1e-3 * np.abs(gos) + 1e-5 * np.abs(gos).max()
        print(f"{name}: max err {err.max():.3g}, max |g| {np.abs(gos).max():.3g}")
        assert np.all(err <= bound), (name, int(np.argmax(err - bound)), float((err - bound).max()))


def test_gradient_against_finite_differences(gpu, orc):
    """FP64 central differences of the oracle's mean cross-entropy on sampled
    coordinates of every tensor (4 KB slice), against the HIP backward.
    A central difference is invalid where the step crosses a ReLU kink; such
    coordinates show up as FD disagreeing with the oracle's own analytic
    gradient and are counted, not compared (at most a few may occur)."""
    import torch
    from paper_2507_12805_amd.autograd import DynamicModel
    cfg, ctx, tgt, w = _slice_case(orc, rows=32)
    params = torch.tensor(w, dtype=torch.float32, device="cuda", requires_grad=True)
    logits = DynamicModel.apply(params, torch.from_numpy(ctx).cuda(), cfg)
    torch.nn.functional.cross_entropy(logits, torch.from_numpy(tgt.astype(np.int64)).cuda()).backward()
    g = params.grad.cpu().numpy().astype(np.float64)
    _, go, _, _ = orc.step(cfg, w, ctx, tgt)
    rng = np.random.default_rng(0)
    h = 1e-6
    checked = kinks = 0
    for name, (off, shp) in orc.param_slices(cfg).items():
        n = int(np.prod(shp))
        seg = g[off:off + n]
        # coordinates carrying gradient (embedding rows of unused tokens are exactly zero)
        cand = np.flatnonzero(np.abs(seg) > 1e-3 * np.abs(seg).max())
        for i in rng.choice(cand, size=min(6, len(cand)), replace=False) + off:
            wp, wm = w.copy(), w.copy()
            wp[i] += h
            wm[i] -= h
            fd = (orc.step(cfg, wp, ctx, tgt, grad=False)[3] - orc.step(cfg, wm, ctx, tgt, grad=False)[3]) / (2 * h)
            if abs(go[i] - fd) > 1e-3 * abs(fd) + 1e-8:
                kinks += 1
                continue
            assert abs(g[i] - fd) <= 1e-3 * abs(fd) + 1e-7, (name, i, g[i], fd)
            checked += 1
    assert checked >= 30 and kinks <= 2, (checked, kinks)


def test_backward_is_deterministic_and_matches_small_shapes(gpu, orc):
    from synth.workloads import model_small
    rng = np.random.default_rng(3)
    for kw in [dict(k=3, t=32, E=16, hidden=[32]), dict(k=2, t=5, E=3, hidden=[7]), dict(k=1, t=3, E=2, hidden=[])]:
        cfg = model_small(s=1, **kw)
        V = 4 ** cfg["k"]
        rows = 50
        ctx = rng.integers(0, V, size=(rows, cfg["t"]), dtype=np.uint8)
        tgt = rng.integers(0, V, size=rows, dtype=np.uint8)
        w = orc.init_params(cfg) + rng.normal(0, 0.05, orc.param_count(cfg))
        w = w.astype(np.float32).astype(np.float64)
        Po, go, _, _ = orc.step(cfg, w, ctx, tgt)
        dl = (Po - np.eye(V)[tgt]) / rows            # d(mean CE)/dlogits
        g1 = gpu.dm_backward(cfg, w, ctx, dl).cpu().numpy()
        g2 = gpu.dm_backward(cfg, w, ctx, dl).cpu().numpy()
        assert np.array_equal(g1, g2)
        assert np.linalg.norm(g1 - go) <= 1e-4 * max(np.linalg.norm(go), 1e-12)
    import torch
    with pytest.raises(gpu.PmklcError):
        bad = np.full((2, 3), 200, dtype=np.uint8)
        gpu.dm_forward(model_small(s=1, k=1, t=3, E=2, hidden=[]), np.zeros(gpu.param_count(
            model_small(s=1, k=1, t=3, E=2, hidden=[])), np.float32), bad)
    assert torch.cuda.is_available()
