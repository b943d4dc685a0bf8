"""Pins for the oracle's (s,k)-mer encoder (Sec. 4.1, Fig. 3).

Independent references: the paper's printed worked example, and Python's
own base-4 integer parser (int(digits, 4)) applied to every window of every
ACGT string up to length 6, for all ten (s,k) pairs with 1 <= s <= k <= 4.
"""
import itertools
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden", "skmer_worked_example.txt")
PAIRS = [(s, k) for k in range(1, 5) for s in range(1, k + 1)]
DIGIT = str.maketrans("ACGT", "0123")


def _windows_by_int_parse(seq: str, s: int, k: int):
    out, j = [], 0
    while j * s + k <= len(seq):
        out.append(int(seq[j * s:j * s + k].translate(DIGIT), 4))
        j += 1
    return out


def test_paper_worked_example(orc):
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        bases, s, k, *tok = line.split()
        assert list(orc.encode_skmer(bases, int(s), int(k))) == [int(x) for x in tok]


@pytest.mark.parametrize("s,k", PAIRS)
def test_brute_force_all_short_strings(orc, s, k):
    for n in range(0, 7):
        for tup in itertools.product("ACGT", repeat=n):
            seq = "".join(tup)
            got = list(orc.encode_skmer(seq, s, k))
            assert got == _windows_by_int_parse(seq, s, k), (seq, s, k)


@pytest.mark.parametrize("s,k", PAIRS)
def test_random_long_input(orc, s, k):
    rng = np.random.default_rng(1000 * s + k)
    seq = "".join(rng.choice(list("ACGT"), size=20011))
    got = orc.encode_skmer(seq, s, k)
    assert got.tolist() == _windows_by_int_parse(seq, s, k)
    assert len(got) == orc.skmer_count(len(seq), s, k)


def test_rejects_bad_input(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.encode_skmer("ACGN", 1, 1)
    assert e.value.code == -2
    with pytest.raises(orc.OracleError):
        orc.encode_skmer("ACGa", 1, 1)
    for s, k in [(2, 1), (0, 3), (1, 5)]:
        with pytest.raises(orc.OracleError) as e:
            orc.encode_skmer("ACGT", s, k)
        assert e.value.code == -1
