"""Pins for the oracle's quantiser and arithmetic coder.

Coder (Witten-Neal-Cleary 1987, 32-bit, total 2^16):
  * closed form: under a uniform distribution over V = 4^k symbols every
    interval is dyadic, so the stream is exactly the symbols' 2k-bit binary
    codes followed by the two flush bits "01" (2k*m + 2 bits);
  * information bounds: sum(-log2 f/T) <= bits <= that + 2 + m * 2^-13
    (truncation loses at most -log2(1 - 2^-14) bits per symbol);
  * round trip on random frequency tables.
Quantiser: total exactly 2^16, every f >= 1, order preserved apart from the
residual recipient, KL(p || f/T) below V/2^16 nats, and closed forms for a
uniform and a one-hot distribution.
"""
import math

import numpy as np
import pytest

T = 1 << 16


def _bits_of(data: bytes, nbits: int) -> str:
    return "".join(f"{b:08b}" for b in data)[:nbits]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_uniform_stream_closed_form(orc, k):
    V = 4 ** k
    rng = np.random.default_rng(k)
    for m in [0, 1, 2, 7, 333]:
        sym = rng.integers(0, V, size=m)
        f = T // V
        data, nbits = orc.wnc_encode(sym * f, (sym + 1) * f)
        assert nbits == 2 * k * m + 2
        expect = "".join(format(int(x), f"0{2 * k}b") for x in sym) + "01"
        assert _bits_of(data, nbits) == expect
        assert len(data) == (nbits + 7) // 8


def _random_cdfs(rng, m, V, skew):
    p = rng.dirichlet([skew] * V, size=m)
    return p


@pytest.mark.parametrize("V,skew", [(4, 0.3), (64, 0.1), (64, 1.0), (256, 0.05)])
def test_roundtrip_and_length_bounds(orc, V, skew):
    rng = np.random.default_rng(V)
    m = 3000
    P = _random_cdfs(rng, m, V, skew)
    cdf = orc.quantise(P)
    sym = np.array([rng.choice(V, p=P[i]) for i in range(m)])
    lo = cdf[np.arange(m), sym]
    hi = cdf[np.arange(m), sym + 1]
    data, nbits = orc.wnc_encode(lo, hi)
    info = float(np.sum(-np.log2((hi - lo) / T)))
    assert info - 1e-9 <= nbits <= info + 2 + m * 2.0 ** -13 + 1e-9
    dec = orc.wnc_decode(data, cdf)
    assert np.array_equal(dec, sym)


def test_extreme_frequencies_roundtrip(orc):
    # probability mass piled on one symbol, the coded ones having f = 1
    V = 64
    m = 500
    P = np.zeros((m, V))
    P[:, 5] = 1.0
    cdf = orc.quantise(P)
    assert np.all(np.diff(cdf, axis=1)[:, 5] == T - (V - 1))
    rng = np.random.default_rng(7)
    sym = rng.integers(0, V, size=m)
    lo, hi = cdf[np.arange(m), sym], cdf[np.arange(m), sym + 1]
    data, nbits = orc.wnc_encode(lo, hi)
    info = float(np.sum(-np.log2((hi - lo) / T)))
    assert info <= nbits <= info + 2 + m * 2.0 ** -13
    assert nbits <= 17 * m + 2
    assert np.array_equal(orc.wnc_decode(data, cdf), sym)


def test_coder_rejects_empty_interval(orc):
    with pytest.raises(orc.OracleError):
        orc.wnc_encode([5], [5])


@pytest.mark.parametrize("V", [4, 16, 64, 256])
def test_quantiser_invariants(orc, V):
    rng = np.random.default_rng(V + 1)
    P = rng.dirichlet([0.2] * V, size=400)
    cdf = orc.quantise(P)
    f = np.diff(cdf.astype(np.int64), axis=1)
    assert np.all(cdf[:, 0] == 0) and np.all(cdf[:, -1] == T)
    assert np.all(f >= 1)
    for r in range(len(P)):
        amax = int(np.argmax(P[r]))  # lowest index on ties
        base = 1 + np.floor(P[r] * (T - V)).astype(np.int64)
        fb = f[r].copy()
        assert fb[amax] >= base[amax]
        fb[amax] = base[amax]
        assert np.array_equal(fb, base)
        order = np.argsort(P[r], kind="stable")
        assert np.all(np.diff(base[order]) >= 0)
        q = f[r] / T
        kl = float(np.sum(np.where(P[r] > 0, P[r] * np.log(np.where(P[r] > 0, P[r], 1) / q), 0.0)))
        assert kl <= V / T + 1e-12


def test_quantiser_closed_forms(orc):
    for V in [4, 16, 64, 256]:
        cdf = orc.quantise(np.full((1, V), 1.0 / V))
        assert np.array_equal(np.diff(cdf[0]), np.full(V, T // V))
    onehot = np.zeros((1, 64))
    onehot[0, 63] = 1.0
    f = np.diff(orc.quantise(onehot)[0].astype(np.int64))
    assert f[63] == T - 63 and np.all(f[:63] == 1)
    tie = np.zeros((1, 64))
    tie[0, 3] = tie[0, 9] = 0.35
    tie[0, 20] = 0.3
    f = np.diff(orc.quantise(tie)[0].astype(np.int64))
    # floor(0.35 * 65472) = 22915 (twice), floor(0.3 * 65472) = 19641:
    # sum f = 64 + 65471, residual 1 goes to the lower of the tied indices
    assert f[3] == 1 + 22915 + 1 and f[9] == 1 + 22915 and f[20] == 1 + 19641


def test_quantiser_takes_fp32_exactly(orc):
    # an FP32 probability times 65472 is exact in FP64: the quantiser's
    # floor must see that exact product
    p = np.float32(0.3)
    P = np.full((1, 64), (1.0 - float(p)) / 63)
    P[0, 0] = float(p)
    f0 = np.diff(orc.quantise(P)[0].astype(np.int64))[0]
    assert f0 >= 1 + math.floor(float(p) * (T - 64))


def test_crc32_matches_zlib(orc):
    import zlib
    for data in [b"", b"a", b"123456789", bytes(range(256)) * 7]:
        assert orc.crc32(data) == zlib.crc32(data)
