"""The synthetic inputs against the recipe they are stated to follow (the
stand-ins for the paper's genomes): alphabet and determinism, the order-m
Markov rows (Dirichlet(0.5) draws from the recipe's seed, with and without
the GC tilt), the share of the sequence covered by planted repeats (forward and
reverse-complemented), the N-run
rate and lengths, the lognormal block lengths and the archive's ranges.
Every expected value comes from the recipe's definition, not from the
generator."""
import numpy as np
import pytest

import synth
from synth import Recipe, archive_files, lognormal_blocks

CODE = np.full(256, 255, dtype=np.uint8)
for i, ch in enumerate(b"ACGT"):
    CODE[ch] = i


def test_alphabet_length_and_determinism():
    r = Recipe(n=100_003, order=4, seed=7, rho=0.05, n_rate=1e-3)
    a, b = synth.generate(r), synth.generate(r)
    assert a.dtype == np.uint8 and len(a) == r.n
    assert set(np.unique(a).tolist()) <= set(b"ACGTN")
    assert np.array_equal(a, b)
    assert not np.array_equal(a, synth.generate(Recipe(n=100_003, order=4, seed=8, rho=0.05, n_rate=1e-3)))
    assert len(synth.generate(Recipe(n=0))) == 0


@pytest.mark.parametrize("gc", [None, 0.65])
def test_markov_rows_follow_the_seeded_dirichlet_draws(gc):
    """Empirical p(b | previous m bases) against the Dirichlet(0.5) rows the
    recipe draws from its seed (context = the m previous bases in base 4,
    oldest most significant), tilted by w_C = w_G = gc/0.5 and
    w_A = w_T = (1-gc)/0.5 when a GC target is set."""
    m, n, seed = 3, 1 << 22, 11
    r = Recipe(n=n, order=m, seed=seed, gc=None if gc is None else (gc, gc), gc_seg=n)
    rows = np.random.default_rng(seed).dirichlet([0.5] * 4, size=4 ** m)
    if gc is not None:
        rows = rows * np.array([1 - gc, gc, gc, 1 - gc]) / 0.5
        rows /= rows.sum(axis=1, keepdims=True)
    c = CODE[synth.generate(r)].astype(np.int64)
    ctx = sum(c[j:n - m + j] << (2 * (m - 1 - j)) for j in range(m))
    nxt = c[m:]
    counts = np.zeros((4 ** m, 4))
    np.add.at(counts, (ctx, nxt), 1)
    tot = counts.sum(axis=1)
    seen = tot >= 200
    assert seen.sum() >= 40
    emp = counts[seen] / tot[seen, None]
    p = rows[seen]
    sd = np.sqrt(p * (1 - p) / tot[seen, None])
    assert np.all(np.abs(emp - p) <= 6 * sd + 1e-12)


def _repeated_32mer_share(a):
    """Share of positions whose 32-mer (ACGT only) already occurred earlier."""
    c = CODE[a].astype(np.uint64)
    n = len(c) - 31
    key = np.zeros(n, dtype=np.uint64)
    for j in range(32):
        key = (key << np.uint64(2)) | c[j:j + n]
    return 1.0 - len(np.unique(key)) / n


def test_planted_repeats_cover_the_stated_share():
    """rho = 5% of forward copies of U{50..500} bases: a piece of length L
    repeats L - 31 of its 32-mers, so about 5% x E[L-31]/E[L] = 4.4% of the
    positions gain an earlier copy of their 32-mer."""
    base = dict(n=1 << 22, order=3, seed=12)
    extra = _repeated_32mer_share(synth.generate(Recipe(**base, rho=0.05))) - \
        _repeated_32mer_share(synth.generate(Recipe(**base)))
    expect = 0.05 * (275 - 31) / 275
    assert abs(extra - expect) <= 0.15 * expect, extra


def _revcomp_32mer_share(a):
    """Share of positions whose 32-mer's reverse complement occurred earlier."""
    c = CODE[a].astype(np.uint64)
    n = len(c) - 31
    fwd = np.zeros(n, dtype=np.uint64)
    rc = np.zeros(n, dtype=np.uint64)
    for j in range(32):
        fwd = (fwd << np.uint64(2)) | c[j:j + n]
        rc = (rc << np.uint64(2)) | (np.uint64(3) - c[31 - j:31 - j + n])
    uniq, first = np.unique(fwd, return_index=True)
    at = np.minimum(np.searchsorted(uniq, rc), len(uniq) - 1)
    return float(np.mean((uniq[at] == rc) & (first[at] < np.arange(n))))


def test_reverse_complement_repeats():
    """With p_rc = 1 every planted piece is the reverse complement of an
    earlier one: the same 4.4% of positions, found through the reverse
    complement and not as forward copies."""
    base = dict(n=1 << 22, order=3, seed=14)
    a0, a1 = synth.generate(Recipe(**base)), synth.generate(Recipe(**base, rho=0.05, p_revcomp=1.0))
    expect = 0.05 * (275 - 31) / 275
    assert abs(_revcomp_32mer_share(a1) - _revcomp_32mer_share(a0) - expect) <= 0.15 * expect
    assert abs(_repeated_32mer_share(a1) - _repeated_32mer_share(a0)) <= 0.25 * expect


def test_n_runs_rate_and_lengths():
    """N runs start at each position with probability rate / 50.5 and last
    U{1..100} bases: about rate of the bases are N, runs average 50.5."""
    n, rate = 1 << 25, 1e-4
    a = synth.generate(Recipe(n=n, order=2, seed=13, n_rate=rate, n_max=100))
    isn = a == ord("N")
    frac = isn.mean()
    assert 0.6 * rate <= frac <= 1.4 * rate, frac
    d = np.diff(np.concatenate([[0], isn.astype(np.int8), [0]]))
    lens = np.flatnonzero(d == -1) - np.flatnonzero(d == 1)
    assert lens.min() >= 1 and 30 <= lens.mean() <= 75
    assert np.mean(lens <= 100) >= 0.9                 # longer ones are two runs back to back


def test_lognormal_block_lengths():
    """256 lognormal(ln 2 MiB, 1) draws rescaled to 1 GiB: the lengths sum to
    the total exactly and keep the log-spread sigma = 1; a lognormal's median
    is exp(-sigma^2 / 2) = 0.61 of its mean."""
    total = 1 << 30
    bl = np.array(lognormal_blocks(total, 256, median=2 << 20, sigma=1.0, seed=3))
    assert len(bl) == 256 and bl.sum() == total and bl.min() >= 1
    assert 0.85 <= np.log(bl).std() <= 1.15
    assert 0.45 <= np.median(bl) / bl.mean() <= 0.8


def test_archive_ranges():
    files = archive_files()
    assert len(files) == 64
    sizes = np.array([f.n for f in files])
    assert sizes.min() >= 1 << 10 and sizes.max() <= 1 << 29
    # log-uniform over [2^10, 2^29]: the log2 sizes spread over most of the range
    assert np.log2(sizes).min() < 13 and np.log2(sizes).max() > 26
    for f in files:
        assert 2 <= f.order <= 8
        assert 0.3 <= f.gc[0] == f.gc[1] <= 0.7
        assert 0.0 <= f.rho <= 0.3 and f.p_revcomp == 0.5 and f.n_rate == 1e-4
    # scaling divides every size (floor(floor(x) / k) = floor(x / k)) and keeps the rest
    small = archive_files(scale=1 / 1024)
    assert [f.n for f in small] == [max(1, f.n // 1024) for f in files]
    assert [(f.order, f.gc, f.rho) for f in small] == [(f.order, f.gc, f.rho) for f in files]
