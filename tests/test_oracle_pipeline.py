"""Pins for the oracle's whole compression pipeline.

  * closed form: under the uniform selector with s = k, every segment stream
    is exactly 2k*L + 2 bits (2 bits/base plus two flush bits), so the whole
    container size is known in advance;
  * lossless round trip of every mode: DM only, static + DM (Eq. 1), Adam,
    two hidden layers, N runs, step-wise model passing chains, uneven blocks;
  * edge cases: n = 0, n < k, all-N, a block with fewer tokens than bs, a
    block whose segments are not longer than t, s < k tails;
  * step-wise model passing (Sec. 4.3): block b+1 starts from block b's
    weights after ceil(5% of L_b) steps, checked against a container built
    with that initial state given explicitly;
  * error paths: invalid bytes, corrupt or truncated containers, wrong
    static weights.
"""
import math

import numpy as np
import pytest

import synth
from tests import cbf
from synth.workloads import model_small

T = 1 << 16


def _varint_len(v):
    n = 1
    while v >= 0x80:
        v >>= 7
        n += 1
    return n


def _dna(n, seed=0, order=2, n_rate=0.0):
    return synth.generate(synth.Recipe(n=n, order=order, seed=seed, n_rate=n_rate, n_max=20))


def _tiny(**kw):
    c = model_small(t=4, E=4, hidden=[8], bs=8)
    c.update(kw)
    return c


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_uniform_container_closed_form(orc, k):
    n = 5003
    a = _dna(n, seed=k)
    cfg = _tiny(s=k, k=k, selector="uniform", n_blocks=3)
    blob = orc.compress(cfg, a)
    nb = [n // 3, n // 3, n - 2 * (n // 3)]
    size = 80 + _varint_len(3)
    streams = 0
    for b in nb:
        l = (b - k) // k + 1
        L, rem = l // 8, l % 8
        tail = b - ((l - 1) * k + k)
        seg = (2 * k * L + 2 + 7) // 8
        size += _varint_len(b) + 1 + (2 * tail + 2 * k * rem + 7) // 8 + 8 * _varint_len(seg)
        streams += 8 * seg
    assert len(blob) == size + streams
    assert np.array_equal(orc.decompress(blob), a)
    # payload = 2 bits/base + 2 flush bits per segment stream
    L0 = ((nb[0] - k) // k + 1) // 8
    assert 8 * ((2 * k * L0 + 2 + 7) // 8) >= 2 * k * L0 + 2


ROUNDTRIP = {
    "dm": dict(),
    "dm_s1k3": dict(s=1, k=3),
    "dm_s2k3": dict(s=2, k=3),
    "spum_dm": dict(selector="spum_dm"),
    "adam_2layer": dict(optimizer="adam", hidden=[8, 6]),
    "no_hidden": dict(hidden=[]),
    "k4": dict(s=4, k=4, t=3, E=2, hidden=[4]),
}


@pytest.mark.parametrize("name", list(ROUNDTRIP))
def test_roundtrip_modes(orc, name):
    a = _dna(6000, seed=3, n_rate=0.002)
    cfg = _tiny(n_blocks=2, **ROUNDTRIP[name])
    static = orc.init_params(cfg, seed=77).astype(np.float32) if cfg["selector"] == "spum_dm" else None
    blob = orc.compress(cfg, a, static=static)
    assert np.array_equal(orc.decompress(blob, static=static), a)
    assert blob[5] == 0  # numeric path: FP64 oracle


def test_roundtrip_smp_chains_and_uneven_blocks(orc):
    a = _dna(9000, seed=4, n_rate=0.001)
    bl = [1000, 3000, 500, 4000, 500]
    cfg = _tiny(block_len=bl, file_blocks=[2, 3], smp_ppm=50000)
    blob = orc.compress(cfg, a)
    assert np.array_equal(orc.decompress(blob), a)
    blob2 = orc.compress(dict(cfg, smp_ppm=0), a)
    assert blob2 != blob


@pytest.mark.parametrize("n,raw", [
    (0, None), (2, None), (1, None), (40, "N" * 40), (37, None), (200, None), (7, "ANNNNNC"),
])
def test_edge_cases(orc, n, raw):
    a = np.frombuffer(raw.encode(), dtype=np.uint8).copy() if raw else _dna(n, seed=n)
    for nblk in [1, 3]:
        cfg = _tiny(n_blocks=nblk)
        blob = orc.compress(cfg, a)
        assert np.array_equal(orc.decompress(blob), a), (n, nblk)


def test_segments_not_longer_than_context_are_uniform(orc):
    # l = 8 * 4 tokens, L = 4 = t: every step is uniform, so the DM container
    # equals the uniform one apart from the selector byte
    a = _dna(96 + 2, seed=9)
    cfg = _tiny(s=3, k=3)
    b_dm = orc.compress(cfg, a)
    b_un = orc.compress(dict(cfg, selector="uniform"), a)
    assert len(b_dm) == len(b_un)
    assert b_dm[80:] == b_un[80:]


def test_smp_snapshot_is_predecessor_after_5_percent(orc):
    """Block 1's first weights are block 0's after ceil(0.05 * L_0) steps."""
    cfg = _tiny(t=3, bs=4)
    a = _dna(2 * 3 * 4 * 100, seed=12)  # two blocks, 100 steps each at (3,3)
    half = len(a) // 2
    cfg2 = dict(cfg, n_blocks=2, smp_ppm=50000)
    blob = orc.compress(cfg2, a)
    tok0 = orc.encode_skmer(a[:half], 3, 3)
    L0 = len(tok0) // 4
    S = math.ceil(0.05 * L0)
    assert S == 5
    _, _, w_snap = orc.trace_block(cfg, tok0, stop=S)
    # block 1 alone, starting from that snapshot, codes the same streams
    single = orc.compress(dict(cfg, n_blocks=1, init_override=w_snap), a[half:])
    assert np.array_equal(orc.decompress(blob), a)
    got = cbf.parse(blob)["blocks"][1]["streams"]
    assert got == cbf.parse(single)["blocks"][0]["streams"]
    # and without passing, block 1 starts from the seeded weights instead
    blob_nosmp = orc.compress(dict(cfg2, smp_ppm=0), a)
    assert cbf.parse(blob_nosmp)["blocks"][1]["streams"] != got


def test_errors(orc):
    cfg = _tiny()
    with pytest.raises(orc.OracleError) as e:
        orc.compress(cfg, np.frombuffer(b"ACGTX", dtype=np.uint8))
    assert e.value.code == -2
    a = _dna(3000, seed=1)
    blob = orc.compress(cfg, a)
    for bad in [blob[:40], blob[:-3], b"XXXX" + blob[4:]]:
        with pytest.raises(orc.OracleError) as e:
            orc.decompress(bad)
        assert e.value.code in (-4, -5)
    cs = dict(cfg, selector="spum_dm")
    st = orc.init_params(cs, seed=5).astype(np.float32)
    b2 = orc.compress(cs, a, static=st)
    wrong = st.copy()
    wrong[0] += 1
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(b2, static=wrong)
    assert e.value.code == -5
    with pytest.raises(orc.OracleError) as e:
        orc.decompress(b2, static=None)
    assert e.value.code == -5
