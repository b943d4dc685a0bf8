"""Pins for the oracle's static private model (Sec. 4.2.3, pipeline stage
(b) of Fig. 2) and its Model Selector (Sec. 4.2.1).

  * the stored model is what the dynamic model's own learning steps make
    of the seeded initialisation (seed ^ 0x5350524D) over bs segments spread
    evenly over the input's whole token sequence, each min(floor(l/bs), 8192)
    tokens long: checked against a training block gathered here from that
    definition (blocks split by hand, N runs removed, tokens from the
    worked-example-pinned encoder) and run through the pinned one-block
    trace, bit for bit;
  * the coding pass is Eq. (1) with S1 in place of S0: the container equals
    the public-model container made with the stored weights as the static
    model, apart from the selector byte and the inserted weights;
  * the selector's size rule: the private model strictly above the bound
    (500 * 10^6 bytes, or the bound given), otherwise the public model when
    one is supplied, else the dynamic model alone;
  * lossless round trips (blocks, N runs, model passing, files, Adam,
    inputs too short to train on), the container's size accounting, and
    the error paths (both static models at once, damaged stored weights).
"""
import numpy as np
import pytest

import synth
from tests import cbf
from synth.workloads import model_small

XOR = 0x5350524D
STEPS = 8192


def _dna(n, seed=0, order=2, n_rate=0.0):
    return synth.generate(synth.Recipe(n=n, order=order, seed=seed, n_rate=n_rate, n_max=20))


def _tiny(**kw):
    c = model_small(t=4, E=4, hidden=[8], bs=8, selector="sprm_dm")
    c.update(kw)
    return c


def _blocks(a, block_len):
    out, off = [], 0
    for ln in block_len:
        out.append(a[off:off + ln])
        off += ln
    assert off == len(a)
    return out


def _training_block(orc, cfg, a, block_len):
    """The definition, written out: all blocks' tokens in block order, then
    bs segments of Lp tokens starting at floor(j * l / bs)."""
    toks = []
    for blk in _blocks(a, block_len):
        stripped = blk[blk != ord("N")]
        toks.append(orc.encode_skmer(stripped, cfg["s"], cfg["k"]))
    T = np.concatenate(toks) if toks else np.zeros(0, np.uint8)
    l, bs = len(T), cfg["bs"]
    Lp = min(l // bs, STEPS)
    segs = [T[(j * l) // bs:(j * l) // bs + Lp] for j in range(bs)]
    return np.concatenate(segs).astype(np.uint8), Lp


def _stored(blob):
    return np.frombuffer(cbf.parse(blob)["private"], dtype="<f4")


@pytest.mark.parametrize("case", ["one_block", "blocks_with_n", "uneven_files"])
def test_stored_model_is_training_on_spread_segments(orc, case):
    if case == "one_block":
        a, bl = _dna(3000, seed=21), [3000]
    elif case == "blocks_with_n":
        a = _dna(7000, seed=22, n_rate=0.003)
        bl = [2000, 2500, 2500]
    else:
        a = _dna(9000, seed=23, n_rate=0.001)
        bl = [1000, 3000, 500, 4000, 500]
    cfg = _tiny(block_len=bl, file_blocks=[2, 3]) if case == "uneven_files" else _tiny(block_len=bl)
    blob = orc.compress(cfg, a)
    pre, Lp = _training_block(orc, cfg, a, bl)
    assert Lp > cfg["t"] + 10
    _, _, wf = orc.trace_block(dict(cfg, selector="dm", seed=cfg["seed"] ^ XOR, block_len=None,
                                    file_blocks=None, n_blocks=1), pre)
    P = orc.param_count(cfg)
    assert np.array_equal(_stored(blob), wf[:P].astype(np.float32))
    # the stored weights moved away from their initialisation
    assert not np.array_equal(_stored(blob), orc.init_params(cfg, seed=cfg["seed"] ^ XOR).astype(np.float32))
    assert np.array_equal(orc.decompress(blob), a)


def test_training_length_is_capped(orc):
    """floor(l / bs) above 8192: the segments are 8192 tokens, still spread
    over the whole input."""
    cfg = _tiny(s=1, k=1, t=3, E=4, hidden=[4], bs=4)
    a = _dna(4 * STEPS * 2 + 100, seed=24)
    bl = [len(a) // 2, len(a) - len(a) // 2]
    cfg["block_len"] = bl
    pre, Lp = _training_block(orc, cfg, a, bl)
    assert Lp == STEPS
    blob = orc.compress(cfg, a)
    _, _, wf = orc.trace_block(dict(cfg, selector="dm", seed=cfg["seed"] ^ XOR, block_len=None, n_blocks=1), pre)
    assert np.array_equal(_stored(blob), wf[:orc.param_count(cfg)].astype(np.float32))


@pytest.mark.parametrize("n", [0, 2, 30, 95])
def test_too_short_to_train_stores_the_initialisation(orc, n):
    """l < bs (no training step): the stored model is the seeded
    initialisation under the derived seed; the coding still round-trips."""
    cfg = _tiny(s=3, k=3)
    a = _dna(n, seed=n)
    blob = orc.compress(cfg, a)
    assert np.array_equal(_stored(blob), orc.init_params(cfg, seed=cfg["seed"] ^ XOR).astype(np.float32))
    assert np.array_equal(orc.decompress(blob), a)


@pytest.mark.parametrize("kw", [dict(), dict(optimizer="adam", hidden=[8, 6]), dict(s=1, k=2, hidden=[]),
                                dict(n_blocks=3, smp_ppm=50000)])
def test_coding_pass_is_eq1_with_the_stored_model(orc, kw):
    """Same bytes as the public-model container made with the stored model
    as static weights, but for the selector byte and the inserted model."""
    a = _dna(6000, seed=25, n_rate=0.002)
    cfg = _tiny(n_blocks=2)
    cfg.update(kw)
    blob = orc.compress(cfg, a)
    w = _stored(blob)
    pub = orc.compress(dict(cfg, selector="spum_dm"), a, static=w)
    hp, hs = cbf.parse(pub)["header"], cbf.parse(blob)["header"]
    assert hs["selector"] == 6 and hp["selector"] == 5
    assert hs["static_crc"] == hp["static_crc"] == orc.crc32(w.tobytes())
    cut = hp["meta_start"]
    expect = pub[:40] + bytes([6]) + pub[41:cut] + w.tobytes() + pub[cut:]
    assert blob == expect
    assert np.array_equal(orc.decompress(blob), a)
    assert np.array_equal(orc.decompress(pub, static=w), a)


def test_model_selector_size_rule(orc):
    """Sec. 4.2.1: the private model strictly above the size bound, else the
    public one when given, else the dynamic model alone."""
    cfg = _tiny(selector="auto")
    st = orc.init_params(cfg, seed=31).astype(np.float32)
    a = _dna(2000, seed=26)
    for bound, n, want in [(2000, 2000, "dm"), (1999, 2000, "sprm_dm"), (0, 2000, "dm")]:
        c = dict(cfg, ms_threshold=bound)
        got = orc.compress(c, a[:n])
        assert got == orc.compress(dict(cfg, selector=want), a[:n]), (bound, n)
        got_pub = orc.compress(c, a[:n], static=st)
        want_pub = "spum_dm" if want == "dm" else want
        assert got_pub == orc.compress(dict(cfg, selector=want_pub), a[:n],
                                       static=st if want_pub == "spum_dm" else None), (bound, n)
    # the recorded selector is the resolved one, which decodes as such
    blob = orc.compress(dict(cfg, ms_threshold=100), a)
    assert cbf.parse(blob)["header"]["selector"] == 6
    assert np.array_equal(orc.decompress(blob), a)


def test_private_model_round_trips(orc):
    for seed, kw in enumerate([dict(n_blocks=4, smp_ppm=50000), dict(block_len=[100, 3900, 2000]),
                               dict(s=2, k=3, n_blocks=2), dict(optimizer="adam")]):
        a = _dna(6000, seed=40 + seed, n_rate=0.002)
        blob = orc.compress(_tiny(**kw), a)
        assert np.array_equal(orc.decompress(blob), a), kw
        # size: the stored model adds exactly 4 P bytes to the metadata
        p = cbf.parse(blob)
        assert len(p["private"]) == 4 * orc.param_count(_tiny(**kw))


def test_private_model_errors(orc):
    a = _dna(3000, seed=50)
    with pytest.raises(orc.OracleError) as e:
        orc.compress(_tiny(selector="spum_sprm_dm"), a, static=orc.init_params(_tiny(), seed=1).astype(np.float32))
    assert e.value.code == -1
    blob = orc.compress(_tiny(), a)
    at = cbf.parse(blob)["header"]["meta_start"] - 7
    bad = bytearray(blob)
    bad[at] ^= 0x40                      # a bit of the stored weights
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(bytes(bad))
    assert e.value.code == -4
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(blob[:90])
    assert e.value.code == -4
    # the static weights argument plays no part for a private-model container
    assert np.array_equal(orc.decompress(blob, static=np.zeros(3, np.float32)), a)


def test_private_model_helps_many_short_blocks(orc):
    """Property the model is there for: when every block is too short for
    its own dynamic model to learn much, a model trained across the whole
    input codes them in fewer bytes, its own 4 P bytes included (order-3
    source, 100 blocks of 4000 bases, 166 steps each; measured 94,403 vs
    102,592 bytes)."""
    a = synth.generate(synth.Recipe(n=400000, order=3, seed=60))
    cfg = _tiny(n_blocks=100, lr=1e-2)
    dm = orc.compress(dict(cfg, selector="dm"), a)
    pr = orc.compress(cfg, a)
    assert len(pr) < 0.95 * len(dm), (len(pr), len(dm))
