"""Pins of the oracle's lattice sampler (oracle/lattice_sample.py)."""
import math

import numpy as np
import pytest

from oracle import lattice_sample as ls

# Known-answer vectors of Philox4x32-10 as published with the generator's
# reference implementation (Salmon et al., SC'11): counter, key -> output.
KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    out = ls.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
    assert tuple(int(v[0]) for v in out) == want


def test_philox_vectorised_over_counters():
    # the array form agrees with element-by-element calls
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2**32, size=(4, 7), dtype=np.uint64)
    arr = ls.philox4x32_10(c[0], c[1], c[2], c[3], 123456789, 987654321)
    for k in range(7):
        one = ls.philox4x32_10(*[np.array([c[i, k]]) for i in range(4)], 123456789, 987654321)
        assert [int(v[0]) for v in one] == [int(v[k]) for v in arr]


@pytest.mark.parametrize("n,side", [(16, 4), (16, 6), (12, 3), (20, 8)])
def test_paint_against_brute_force(n, side):
    rng = np.random.default_rng(n * side)
    occ = rng.random((n, n)) < 0.05
    got = ls.paint(occ, side, 10.0, 1.0)
    want = np.ones((n, n))
    for i, j in zip(*np.nonzero(occ)):
        for u in range(side):
            for v in range(side):
                want[(i - side // 2 + u) % n, (j - side // 2 + v) % n] = 10.0
    assert np.array_equal(got, want)


def test_occupancy_and_coverage_frequencies():
    n, side = 256, 8
    mu = math.log(2.0) / side ** 2
    thr = int(round(2**32 * -math.expm1(-mu)))
    p = thr / 2**32
    occ_total, cov = 0, []
    R = 6
    for r in range(R):
        occ = ls.occupancy(n, 11, r, thr)
        occ_total += int(occ.sum())
        cov.append(float((ls.paint(occ, side, 2.0, 1.0) == 2.0).mean()))
    # occupancy: binomial(R n^2, p), within 5 standard deviations
    m, sd = R * n * n * p, math.sqrt(R * n * n * p * (1 - p))
    assert abs(occ_total - m) <= 5 * sd
    # coverage: 1 - (1 - p)^(side^2) = 1 - exp(-ln 2) = 1/2 in expectation
    assert abs(1 - (1 - p) ** (side * side) - 0.5) < 1e-6
    assert abs(np.mean(cov) - 0.5) < 0.03


def test_fields_depend_only_on_seed_and_index():
    thr = 2**28
    a = ls.field(64, 8, 5, 1000, thr, 10.0, 1.0)
    assert np.array_equal(a, ls.field(64, 8, 5, 1000, thr, 10.0, 1.0))
    assert not np.array_equal(a, ls.field(64, 8, 5, 1001, thr, 10.0, 1.0))
    assert not np.array_equal(a, ls.field(64, 8, 6, 1000, thr, 10.0, 1.0))
    # realization indices beyond 2^32 use the second counter word
    assert not np.array_equal(ls.field(64, 8, 5, 2**32 + 1000, thr, 10.0, 1.0), a)
    assert np.all(ls.field(64, 8, 5, 7, 0, 10.0, 1.0) == 1.0)


def test_fixed_count_centres_by_integer_arithmetic():
    # each centre from its own Philox call and an exact 64 x 64 -> 128-bit
    # product, in plain Python integers
    n, K, seed, r = 96, 50, (9 << 32) | 31337, (1 << 33) + 5
    got = ls.fixed_count_centres(n, K, seed, r)
    for k in range(K):
        w = ls.philox4x32_10([k], [r & 0xFFFFFFFF], [r >> 32], [ls.FIXED_TAG], seed & 0xFFFFFFFF, seed >> 32)
        v = int(w[0][0]) + (int(w[1][0]) << 32)
        assert got[k] == (v * n * n) // 2**64
    assert got.min() >= 0 and got.max() < n * n


def test_fixed_count_centres_uniform_and_coverage():
    # centres uniform over the nodes (chi-square over 16 row bands, and over
    # the residues mod 16 of the column); coverage of the painted field
    # against 1 - (1 - side^2 / n^2)^K, the covered fraction of K squares
    # with independent uniform centres
    n, side = 64, 2
    K = (n // 4) ** 2            # L^2 squares at m0 = 4
    c = np.concatenate([ls.fixed_count_centres(n, K, 3, r) for r in range(64)])
    for stat in ((c // n) // (n // 16), (c % n) % 16):
        counts = np.bincount(stat, minlength=16)
        e = c.size / 16
        chi2 = float(np.sum((counts - e) ** 2 / e))
        assert chi2 < 45.0          # 15 degrees of freedom: p < 1e-4
    cov = np.mean([(ls.fixed_count_field(n, side, K, 3, r, 1.0, 0.4) == 1.0).mean() for r in range(64)])
    want = 1.0 - (1.0 - side * side / (n * n)) ** K
    assert abs(cov - want) < 0.01
    f = ls.fixed_count_field(n, side, K, 3, 0, 1.0, 0.4)
    assert set(np.unique(f)) <= {0.4, 1.0}
    assert not np.array_equal(f, ls.fixed_count_field(n, side, K, 3, 1, 1.0, 0.4))
