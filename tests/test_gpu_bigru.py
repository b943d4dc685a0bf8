"""GPU parity of the BiGRU static public model (Sec. 4.2.2) mixed with the
MLP dynamic model by Eq. (1) on the launch-sequence loop.

  * FP32: probabilities along a block's trajectory within 1e-4 of the FP64
    oracle (static logits from the fused BiGRU kernel, the learned mixing
    weight's own updates included);
  * FP32 and BF16: lossless round trips, containers within 0.5% of the
    oracle's, the static model's shape in the header, decoding refused with
    another static model;
  * the paper's widths (16-d embedding, two layers, Dense 128) with the
    64 MiB workload's dynamic model, on a short input;
  * error paths.
"""
import numpy as np
import pytest

import synth
from synth.workloads import model_small

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12805_amd as P
    P.load()
    return P


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _cfg(**kw):
    c = model_small(t=8, E=8, hidden=[16], bs=16, selector="spum_dm", static_arch="bigru", static_E=6, gru_h=8,
                    gru_layers=2, dense=12, lr=0.01)
    c.update(kw)
    return c


def _dna(n, seed, n_rate=0.0):
    return synth.generate(synth.Recipe(n=n, order=3, seed=seed, n_rate=n_rate, n_max=30, rho=0.05))


def _static(orc, cfg, seed=21):
    rng = np.random.default_rng(seed)
    ws = orc.static_init(cfg, seed) + rng.normal(0, 0.05, orc.static_param_count(cfg))
    return ws.astype(np.float32)


@pytest.mark.parametrize("layers", [1, 2])
def test_trajectory_fp32(gpu, orc, layers):
    cfg = _cfg(precision="fp32", gru_layers=layers)
    ws = _static(orc, cfg)
    a = _dna(3 * 16 * 70 + 2, 30)
    tok = orc.encode_skmer(a, 3, 3)
    t = cfg["t"]
    steps = [t - 1, t, t + 1, t + 10, 69]
    Pg, wg = gpu.model_trace(cfg, tok, steps=steps, static=ws)
    Po, _, wo = orc.trace_block(cfg, tok, steps=steps, static=ws)
    d = np.abs(Pg.cpu().numpy() - Po).max()
    print(f"bigru {layers} layer(s): trajectory |dP| max {d:.3g}, mixing weight {wg[-1].item():.6f} vs {wo[-1]:.6f}")
    assert d <= 1e-4
    assert abs(wg[-1].item() - wo[-1]) <= 1e-4          # the learned mixing weight


@pytest.mark.parametrize("precision,path", [("fp32", 8), ("bf16", 7)])
def test_roundtrip_and_ratio(gpu, orc, precision, path):
    cfg = _cfg(precision=precision, block_len=[9000, 14001, 6000])
    ws = _static(orc, cfg, 22)
    a = _dna(29001, 31, n_rate=0.002)
    blob = gpu.compress(cfg, _cuda(a), static=ws)
    assert blob[5] == path and blob[40] == 5 and blob[43] == 1 | (2 << 4)
    assert blob[60] == 6 and blob[61] == 8 and blob[62] == 12
    assert np.array_equal(gpu.decompress(blob, static=ws).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a, static=ws)
    rel = len(blob) / len(blob_o) - 1
    print(f"{precision}: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005
    assert blob[56:64] == blob_o[56:64]                  # static CRC and widths as the oracle writes them
    with pytest.raises(gpu.PmklcError) as e:
        gpu.decompress(blob, static=_static(orc, cfg, 23))
    assert e.value.code == -5


def test_paper_widths(gpu, orc):
    """16-d embedding, two BiGRU layers of 32 units, Dense 128, with the
    64 MiB workload's dynamic model ((1,3)-mers, hidden 128), BF16."""
    cfg = model_small(s=1, k=3, hidden=[128], selector="spum_dm", static_arch="bigru", static_E=16, gru_h=32,
                      gru_layers=2, dense=128, lr=0.1, precision="bf16", n_blocks=2)
    ws = _static(orc, cfg, 24)
    a = _dna(2 * (64 * 60 + 2), 32)
    blob = gpu.compress(cfg, _cuda(a), static=ws)
    assert np.array_equal(gpu.decompress(blob, static=ws).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a, static=ws)
    rel = len(blob) / len(blob_o) - 1
    print(f"paper widths: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005


def test_errors(gpu, orc):
    cfg = _cfg()
    ws = _static(orc, cfg)
    a = _dna(5000, 33)
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress(cfg, _cuda(a), static=ws[:-1])
    assert e.value.code == -5
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress(dict(cfg, selector="sprm_dm"), _cuda(a))
    assert e.value.code == -1
    with pytest.raises(gpu.PmklcError) as e:
        gpu.compress(dict(cfg, gru_layers=3), _cuda(a), static=ws)
    assert e.value.code == -1
