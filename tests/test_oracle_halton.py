"""Pins of the oracle's Halton sampler (Sec. IV-A: the paper's experiments
draw configurations from multi-dimensional Halton sequences), independent of
the GPU: the radical inverse against its definition evaluated exactly in
rational arithmetic, closed-form points, the van der Corput stratification,
the point index, and the planner running on Halton samples."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W

PRIMES = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53]


def exact_radical_inverse(i, b):
    """sum_k d_k b^-(k+1) over the base-b digits of i (least significant
    first), as an exact fraction."""
    u, scale = Fraction(0), Fraction(1, b)
    while i:
        u += (i % b) * scale
        i //= b
        scale /= b
    return u


def test_radical_inverse_is_the_exact_value_rounded(orc):
    rng = np.random.default_rng(3)
    idx = list(range(0, 200)) + [int(x) for x in rng.integers(0, 2 ** 32, 300)] + [2 ** 32 - 1, 2 ** 31, 53 ** 5]
    for b in PRIMES:
        for i in idx:
            want = np.float32(float(exact_radical_inverse(i, b)))   # exact -> FP64 (correctly rounded) -> FP32
            assert orc.radical_inverse(i, b) == want, (i, b)


def test_radical_inverse_closed_forms(orc):
    assert [orc.radical_inverse(i, 2) for i in range(1, 8)] == [0.5, 0.25, 0.75, 0.125, 0.625, 0.375, 0.875]
    third = [1 / 3, 2 / 3, 1 / 9, 4 / 9, 7 / 9, 2 / 9, 5 / 9, 8 / 9]
    assert np.allclose([orc.radical_inverse(i, 3) for i in range(1, 9)], third, rtol=0, atol=1e-7)
    assert orc.radical_inverse(0, 5) == 0.0
    for b in PRIMES:
        for m in range(1, 5):
            assert orc.radical_inverse(b ** m, b) == np.float32(1.0 / b ** (m + 1))


@pytest.mark.parametrize("b", [2, 3, 7, 53])
def test_van_der_corput_stratification(orc, b):
    """The first b^m points of the base-b sequence are exactly the fractions
    k / b^m, each once."""
    m = {2: 10, 3: 6, 7: 3, 53: 2}[b]
    n = b ** m
    got = sorted(round(orc.radical_inverse(i, b) * n) for i in range(n))
    assert got == list(range(n))


def test_halton_config_index_and_mapping(orc, r7):
    lo, hi = r7["q_lo"], r7["q_hi"]
    seed, query, rnd, w, workers, tries, t = 0xABCDEF0012345678, 3, 17, 5, 64, 2, 1
    i = (0x12345678 + 65536 * query + (rnd * workers + w) * tries + t + 1) % 2 ** 32
    q = orc.halton_config(seed, query, rnd, w, workers, tries, t, lo, hi)
    for j in range(7):
        u = np.float32(orc.radical_inverse(i, PRIMES[j]))
        span = np.float32(hi[j]) - np.float32(lo[j])
        assert abs(float(q[j]) - (float(lo[j]) + float(u) * float(span))) <= 4e-7 * 2.8
        assert lo[j] <= q[j] <= hi[j]
    # consecutive workers take consecutive points; the index wraps modulo 2^32
    a = orc.halton_config(2 ** 32 - 2, 0, 0, 0, 1, 1, 0, lo, hi)
    b = orc.halton_config(0, 0, 0, 0, 1, 1, 0, lo, hi)
    np.testing.assert_array_equal(a, orc.halton_config(2 ** 32 - 3, 0, 0, 1, 1, 1, 0, lo, hi))
    assert not np.array_equal(a, b)


def test_halton_points_fill_the_box_evenly(orc):
    """Low discrepancy: the first 4096 2-D points (bases 2 and 3) put between
    28 and 36 points in every cell of an 8 x 16 grid (expected 32); uniform
    random points spread much wider."""
    n = 4096
    x = np.array([orc.radical_inverse(i, 2) for i in range(1, n + 1)])
    y = np.array([orc.radical_inverse(i, 3) for i in range(1, n + 1)])
    h, _, _ = np.histogram2d(x, y, bins=[8, 16], range=[[0, 1], [0, 1]])
    assert h.min() >= 28 and h.max() <= 36
    r = np.random.default_rng(0).random((n, 2))
    hr, _, _ = np.histogram2d(r[:, 0], r[:, 1], bins=[8, 16], range=[[0, 1], [0, 1]])
    assert hr.max() - hr.min() > h.max() - h.min()


def test_planner_on_halton_samples(orc, r7):
    """The planner with Halton samples finds valid paths, differs from the
    Philox planner, and is reproducible."""
    from conftest import free_query
    rob = orc.OracleRobot(r7)
    prims = W.scene_s12(r7, 2)
    s, g = free_query(orc, rob, prims, r7, W.SEED_QUERY + 2)
    st, path, stats = orc.plan(rob, prims, s, g, seed=5, workers=32, max_rounds=300, sampler=2)
    assert st == 0
    assert np.array_equal(path[0], s) and np.array_equal(path[-1], g)
    m, _ = orc.path_clearance(rob, prims, path, 4 * 32.0)
    assert m >= -orc.FLAG_BAND
    st2, path2, stats2 = orc.plan(rob, prims, s, g, seed=5, workers=32, max_rounds=300, sampler=2)
    assert st2 == st and np.array_equal(path2, path) and stats2 == stats
    st0, path0, stats0 = orc.plan(rob, prims, s, g, seed=5, workers=32, max_rounds=300)
    assert stats0 != stats or not np.array_equal(path0, path)
