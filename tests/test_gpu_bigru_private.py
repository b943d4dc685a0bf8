"""GPU parity of the one-layer BiGRU static private model (Sec. 4.2.2 shape,
trained on the input as in Sec. 4.2.3) mixed with the MLP dynamic model by
Eq. (1) on the launch-sequence loop.

  * the private model the GPU trains (FP32 training kernels: forward with
    kept states, dense backward, back-propagation through time, partial
    gradients summed in workgroup order, SGD / Adam) against the FP64
    oracle's, both as stored in the container: within 2e-5 per weight after
    about a hundred steps (FP32 sums of tens of products per step, the
    rounding differences carried through the updates; measured 4.8e-7 with
    SGD, 9.1e-7 with Adam);
  * FP32 and BF16: lossless round trips, containers within 0.5% of the
    oracle's, the BiGRU shape in the header, decoding with the stored model
    only (no static weights from the caller);
  * the Model Selector picks it above its size bound; the paper's widths
    (16-d embedding, 32 units, Dense 128) on a short input; error paths.
"""
import numpy as np
import pytest

import synth
from synth.workloads import model_small
from tests import cbf

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
    c = model_small(t=8, E=8, hidden=[16], bs=16, selector="sprm_dm", static_arch="bigru", static_E=6, gru_h=8,
                    gru_layers=1, dense=12, lr=0.01, block_len=[3000, 3000])
    c.update(kw)
    return c


def _dna(n, seed, n_rate=0.0):
    return synth.generate(synth.Recipe(n=n, order=3, seed=seed, n_rate=n_rate, n_max=30, rho=0.05))


@pytest.mark.parametrize("opt", [dict(optimizer="sgd", lr=0.05), dict(optimizer="adam", lr=0.01)])
def test_trained_private_model_matches_oracle(gpu, orc, opt):
    cfg = _cfg(precision="fp32", **opt)
    a = _dna(6000, 40)
    blob = gpu.compress(cfg, _cuda(a))
    blob_o = orc.compress(cfg, a)
    pg = np.frombuffer(cbf.parse(blob)["private"], dtype=np.float32)
    po = np.frombuffer(cbf.parse(blob_o)["private"], dtype=np.float32)
    init = orc.static_init(cfg, cfg["seed"] ^ 0x5350524D).astype(np.float32)
    d = np.abs(pg.astype(np.float64) - po).max()
    moved = np.abs(po.astype(np.float64) - init).max()
    print(f"{opt['optimizer']}: private model |GPU - oracle| max {d:.3g} (training moved weights by up to {moved:.3g})")
    assert pg.size == po.size == orc.static_param_count(cfg)
    assert moved > 1e-2 and d <= 2e-5
    assert blob[40] == 6 and blob[43] == 1 | (1 << 4) and blob[60:64] == blob_o[60:64]
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    rel = len(blob) / len(blob_o) - 1
    print(f"container {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005


@pytest.mark.parametrize("precision,path", [("fp32", 8), ("bf16", 7)])
def test_roundtrip_and_ratio(gpu, orc, precision, path):
    cfg = _cfg(precision=precision, block_len=[9000, 14001, 6000])
    a = _dna(29001, 41, n_rate=0.002)
    blob = gpu.compress(cfg, _cuda(a))
    assert blob[5] == path and blob[40] == 6
    assert blob[60] == 6 and blob[61] == 8 and blob[62] == 12
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    assert blob == gpu.compress(cfg, _cuda(a))          # training and coding are deterministic
    blob_o = orc.compress(cfg, a)
    rel = len(blob) / len(blob_o) - 1
    print(f"{precision}: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005
    # a corrupted stored model is refused
    bad = bytearray(blob)
    bad[cbf.parse(blob)["header"]["meta_start"] - 3] ^= 4
    with pytest.raises(gpu.PmklcError) as e:
        gpu.decompress(bytes(bad))
    assert e.value.code == -4


def test_model_selector_picks_it(gpu, orc):
    cfg = _cfg(selector="auto", ms_threshold=5000)
    a = _dna(6000, 42)
    blob = gpu.compress(cfg, _cuda(a))
    assert blob[40] == 6
    assert blob == gpu.compress(dict(cfg, selector="sprm_dm"), _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)


def test_paper_widths(gpu, orc):
    """16-d embedding, one BiGRU layer of 32 units, Dense 128, with the
    64 MiB workload's dynamic model ((1,3)-mers, hidden 128), BF16."""
    cfg = model_small(s=1, k=3, hidden=[128], selector="sprm_dm", static_arch="bigru", static_E=16, gru_h=32,
                      gru_layers=1, dense=128, lr=0.1, precision="bf16", n_blocks=2)
    a = _dna(2 * (64 * 60 + 2), 43)
    blob = gpu.compress(cfg, _cuda(a))
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)
    blob_o = orc.compress(cfg, a)
    rel = len(blob) / len(blob_o) - 1
    print(f"paper widths: {len(blob)} vs oracle {len(blob_o)} bytes, rel {rel:+.5f}")
    assert abs(rel) <= 0.005


@pytest.mark.parametrize("n", [20, 3 * 16 * 8 + 2])
def test_short_inputs_store_the_initialisation(gpu, orc, n):
    """Fewer tokens than bs, or fewer steps than t: the stored model is the
    seeded initialisation, bit for bit as the oracle stores it."""
    cfg = _cfg(n_blocks=1, block_len=None)
    a = _dna(n, 45)
    blob = gpu.compress(cfg, _cuda(a))
    assert cbf.parse(blob)["private"] == cbf.parse(orc.compress(cfg, a))["private"]
    assert np.array_equal(gpu.decompress(blob).cpu().numpy(), a)


def test_errors(gpu):
    a = _dna(5000, 44)
    for bad, code in [(dict(gru_layers=2), -1), (dict(static_E=40), -7), (dict(gru_h=70), -7),
                      (dict(selector="auto", ms_threshold=1000, gru_layers=2), -1)]:
        with pytest.raises(gpu.PmklcError) as e:
            gpu.compress(_cfg(**bad), _cuda(a))
        assert e.value.code == code, bad
