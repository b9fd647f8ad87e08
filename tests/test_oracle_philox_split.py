"""Pins of the oracle's random splits: Philox and the (primary, secondary, i) selection.

Philox4x32-10 / 4x64-10 are the counter-based generators of Salmon et al.
(SC'11); the split of Z into groups of sizes (n, m) is the "randomly
partition Z" step of Algorithm 1.  Nothing here calls GPU code.
"""
from itertools import combinations
from math import comb
from pathlib import Path

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O

GOLDEN = Path(__file__).parent / "golden"


def _kat(name):
    rows = []
    for line in (GOLDEN / name).read_text().splitlines():
        if line.strip() and not line.startswith("#"):
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox4x32_known_answers():
    for row in _kat("philox4x32_10_kat.txt"):
        out = O.philox4x32(row[0:4], row[4:6])
        assert [int(x) for x in out] == row[6:10]


def test_philox4x64_known_answer():
    for row in _kat("philox4x64_10_kat.txt"):
        out = O.philox4x64(row[0:4], row[4:6])
        assert [int(x) for x in out] == row[6:10]


def test_philox4x64_matches_numpy_bitgenerator():
    # numpy.random.Philox is an independent Philox4x64-10; it increments the
    # 256-bit counter before producing a block.
    rng = np.random.default_rng(5)
    for _ in range(20):
        ctr = rng.integers(0, 2**64, 4, dtype=np.uint64)
        key = rng.integers(0, 2**64, 2, dtype=np.uint64)
        got = np.random.Philox(counter=ctr, key=key).random_raw(4)
        v = (sum(int(ctr[i]) << (64 * i) for i in range(4)) + 1) % (1 << 256)
        c1 = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
        assert np.array_equal(got, O.philox4x64(c1, key))


def test_philox_rounds_matter():
    a = O.philox4x32([1, 2, 3, 4], [5, 6], rounds=10)
    b = O.philox4x32([1, 2, 3, 4], [5, 6], rounds=7)
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("N", [1, 5, 16, 17, 63, 100])
def test_split_keys_layout(N):
    seed, pair, b = 0x1234_5678_9ABC_DEF0, 7, 42
    P, S = O.split_keys(seed, pair, b, N)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(N):
        w = O.philox4x32([i // 16, b, pair, 0], key)
        assert P[i] == (int(w[(i % 16) // 4]) >> (8 * (i % 4))) & 0xFF
        w = O.philox4x32([i // 4, b, pair, 1], key)
        assert S[i] == w[i % 4]


@pytest.mark.parametrize("N,n", [(8, 4), (40, 3), (100, 61), (257, 128), (1000, 999), (33, 1)])
def test_split_mask_is_first_n_in_key_order(N, n):
    for b in [0, 1, 99, 2**32 - 1]:
        P, S = O.split_keys(3, 1, b, N)
        order = sorted(range(N), key=lambda i: (int(P[i]), int(S[i]), i))
        want = np.zeros(N, bool)
        want[order[:n]] = True
        mk = O.split_mask(3, 1, b, N, n)
        assert np.array_equal(O.mask_to_bool(mk, N), want)
        assert sum(bin(int(x)).count("1") for x in mk) == n
        if N % 32:
            assert int(mk[-1]) >> (N % 32) == 0


def test_split_uniform_over_all_70_subsets():
    # N = 8, n = 4: every one of the C(8,4) = 70 subsets should be equally likely.
    N, n, R = 8, 4, 14000
    index = {c: k for k, c in enumerate(combinations(range(N), n))}
    counts = np.zeros(len(index))
    for b in range(R):
        sel = O.mask_to_bool(O.split_mask(11, 0, b, N, n), N)
        counts[index[tuple(np.flatnonzero(sel))]] += 1
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-3, chi2


def test_split_inclusion_frequency():
    N, n, R = 37, 11, 4000
    freq = np.zeros(N)
    for b in range(R):
        freq += O.mask_to_bool(O.split_mask(5, 2, b, N, n), N)
    expect = R * n / N
    sd = np.sqrt(R * (n / N) * (1 - n / N))
    assert np.all(np.abs(freq - expect) < 5 * sd)


def test_split_depends_on_seed_pair_and_b():
    base = O.split_mask(0, 0, 0, 300, 150)
    assert not np.array_equal(base, O.split_mask(1, 0, 0, 300, 150))
    assert not np.array_equal(base, O.split_mask(0, 1, 0, 300, 150))
    assert not np.array_equal(base, O.split_mask(0, 0, 1, 300, 150))
    assert comb(300, 150) > 0
