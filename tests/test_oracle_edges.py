"""Pins of the oracle's edge checking (Alg. 2 / Sec. III-A), nearest neighbour
(Sec. III-B), steering and Philox sampling against brute force, closed forms
and published known-answer vectors."""
import os

import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- point count ---------------------------------------------------------------
def test_edge_count_exact_values(orc):
    z = np.zeros(7, np.float32)
    e = np.zeros(7, np.float32)
    assert orc.edge_count(z, z, 32.0) == 1                     # zero length -> one step
    e[0] = 1.0
    assert orc.edge_count(z, e, 32.0) == 32                    # exactly 32 * 1
    e[0] = 0.5
    assert orc.edge_count(z, e, 32.0) == 16
    e[0] = 1.0 + 2.0 ** -20                                    # just above 1 -> 33
    assert orc.edge_count(z, e, 32.0) == 33
    e[:] = 0
    e[0], e[1] = 0.375, 0.5                                    # 3-4-5 triangle: L = 0.625 exactly
    assert orc.edge_count(z, e, 32.0) == 20
    assert orc.edge_count(e, z, 32.0) == 20                    # direction does not matter
    e[:] = 0
    e[3] = 0.01
    assert orc.edge_count(z, e, 32.0) == 1                     # ceil(0.32) = 1


def test_edge_count_is_least_integer_covering(orc):
    """n is the smallest integer >= res * L (checked in FP64 away from rounding ties)."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        a = rng.uniform(-2.8, 2.8, 7).astype(np.float32)
        b = rng.uniform(-2.8, 2.8, 7).astype(np.float32)
        x = 32.0 * np.linalg.norm(b.astype(np.float64) - a.astype(np.float64))
        if abs(x - round(x)) < 1e-4:
            continue
        assert orc.edge_count(a, b, 32.0) == max(1, int(np.ceil(x)))


# ---- edge verdicts ----------------------------------------------------------------
def _tiny_scene(r7, seed=31):
    return W.random_scene(seed, r7, 2, 2, 1)


def test_edge_clearance_equals_explicit_point_loop(orc, r7):
    """The edge clearance is the min of the configuration clearance over the
    points i/n along the edge (points built here independently, in FP64)."""
    rob = orc.OracleRobot(r7)
    prims = _tiny_scene(r7)
    a, b = W.random_edges(r7, 20, seed=5)
    for k in range(20):
        n = orc.edge_count(a[k], b[k], 32.0)
        pts = [a[k].astype(np.float64) + (i / n) * (b[k].astype(np.float64) - a[k].astype(np.float64))
               for i in range(n + 1)]
        m = min(orc.config_clearance(rob, prims, p) for p in pts)
        assert orc.edge_clearance(rob, prims, a[k], b[k], 32.0, 0, False) == m
        m1 = min(orc.config_clearance(rob, prims, p) for p in pts[1:])
        assert orc.edge_clearance(rob, prims, a[k], b[k], 32.0, 1, False) == m1


def test_edge_verdict_catches_long_collisions_dense(orc, r7):
    """Against 2000-point dense sampling: if the edge collides over a t-interval
    longer than 1/n, some checked point lies inside it, so the edge is invalid;
    if dense sampling finds no collision at all, the edge is valid."""
    rob = orc.OracleRobot(r7)
    prims = _tiny_scene(r7, 77)
    a, b = W.random_edges(r7, 40, seed=6)
    ts = np.linspace(0.0, 1.0, 2001)
    for k in range(40):
        a64, b64 = a[k].astype(np.float64), b[k].astype(np.float64)
        hit = np.array([orc.config_clearance(rob, prims, a64 + t * (b64 - a64)) < 0 for t in ts])
        n = orc.edge_count(a[k], b[k], 32.0)
        valid, _, _ = orc.check_edges(rob, prims, a[k:k + 1], b[k:k + 1], 32.0, early_exit=False)
        # longest run of colliding dense samples, as a t-length
        run = best = 0
        for h in hit:
            run = run + 1 if h else 0
            best = max(best, run)
        if (best - 1) / 2000.0 > 1.0 / n:
            assert valid[0] == 0
        if not hit.any():
            assert valid[0] == 1


def test_edge_verdict_empty_and_enclosing(orc, r7):
    rob = orc.OracleRobot(r7)
    a, b = W.random_edges(r7, 200, seed=8)
    empty = np.zeros(0, W.PRIM_DTYPE)
    v, f, _ = orc.check_edges(rob, empty, a, b, 32.0)
    assert v.all() and not f.any()
    big = W.make_prims([(W.PRIM_SPHERE, (0, 0, 0.5), np.eye(3), (5.0, 0, 0))])
    v, _, _ = orc.check_edges(rob, big, a, b, 32.0)
    assert not v.any()


def test_edge_verdict_monotone_and_permutation_invariant(orc, r7):
    rob = orc.OracleRobot(r7)
    a, b = W.random_edges(r7, 300, seed=9)
    prims = W.scene_mixed(99, r7, 12)
    prev = np.ones(300, np.uint8)
    for k in range(1, 13):
        v, _, _ = orc.check_edges(rob, prims[:k], a, b, 32.0)
        assert np.all(v <= prev)      # an added obstacle never frees an edge
        prev = v
    perm = np.random.default_rng(0).permutation(12)
    v2, _, _ = orc.check_edges(rob, prims[perm], a, b, 32.0)
    assert np.array_equal(v2, prev)


def test_early_exit_mode_gives_identical_verdicts(orc, r7):
    rob = orc.OracleRobot(r7)
    prims = W.scene_s64(r7)
    a, b = W.random_edges(r7, 500, seed=10)
    v0, f0, _ = orc.check_edges(rob, prims, a, b, 32.0, early_exit=False)
    v1, f1, _ = orc.check_edges(rob, prims, a, b, 32.0, early_exit=True)
    assert np.array_equal(v0, v1) and np.array_equal(f0, f1)


# ---- nearest neighbour ------------------------------------------------------------
def test_nearest_matches_exhaustive_fp64(orc):
    rng = np.random.default_rng(3)
    dof, cap = 7, 700
    for size in (1, 2, 63, 64, 65, 500, 700):
        tree = rng.uniform(-2.8, 2.8, (dof, cap)).astype(np.float32)
        for _ in range(20):
            x = rng.uniform(-2.8, 2.8, dof).astype(np.float32)
            d = np.sum((tree[:, :size].astype(np.float64) - x[:, None]) ** 2, axis=0)
            order = np.argsort(d)
            if size > 1 and d[order[1]] - d[order[0]] < 1e-5 * d[order[0]]:
                continue  # FP32 may legitimately break a near-tie either way
            assert orc.nearest(tree, size, x) == order[0]


def test_nearest_ties_and_blocked(orc):
    tree = np.zeros((3, 10), np.float32)
    tree[0, :] = [5, 1, 1, 3, 1, 9, 9, 9, 9, 9]
    x = np.zeros(3, np.float32)
    assert orc.nearest(tree, 10, x) == 1              # nodes 1, 2, 4 tie -> lowest
    bl = np.zeros(10, np.uint8)
    bl[1] = 1
    assert orc.nearest(tree, 10, x, bl) == 2
    bl[[2, 4]] = 1
    assert orc.nearest(tree, 10, x, bl) == 3
    assert orc.nearest(tree, 4, x, np.ones(10, np.uint8)) == -1


# ---- steer -----------------------------------------------------------------------
def test_steer_short_and_long(orc):
    rng = np.random.default_rng(4)
    for _ in range(500):
        a = rng.uniform(-2.8, 2.8, 7).astype(np.float32)
        b = rng.uniform(-2.8, 2.8, 7).astype(np.float32)
        delta = float(rng.choice([0.1, 0.5, 1.0, 20.0]))
        out = orc.steer(a, b, delta)
        L = np.linalg.norm(b.astype(np.float64) - a.astype(np.float64))
        if L <= delta * (1 - 1e-6):
            assert np.array_equal(out, b)
        elif L > delta * (1 + 1e-6):
            d = out.astype(np.float64) - a
            assert np.linalg.norm(d) == pytest.approx(delta, rel=2e-6)
            u = (b.astype(np.float64) - a) / L
            assert np.linalg.norm(d - np.dot(d, u) * u) < 1e-5   # on the segment
            assert np.dot(d, u) > 0


# ---- Philox and RANDOM_CONFIG --------------------------------------------------------
def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) >= 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_sample_config_range_determinism_uniformity(orc, r7):
    lo, hi = r7["q_lo"], r7["q_hi"]
    s = np.array([orc.sample_config(0xABCDEF0123, 0, r, w, lo, hi) for r in range(20) for w in range(256)])
    assert np.all(s >= lo) and np.all(s < hi)
    s2 = np.array([orc.sample_config(0xABCDEF0123, 0, r, w, lo, hi) for r in range(20) for w in range(256)])
    assert np.array_equal(s, s2)
    assert not np.array_equal(s[0], orc.sample_config(0xABCDEF0123, 1, 0, 0, lo, hi))
    # chi-square on 16 bins per joint: 5120 samples, 15 dof -> 99.9% quantile 37.7
    u = (s.astype(np.float64) - lo) / (hi.astype(np.float64) - lo)
    for j in range(7):
        cnt = np.bincount(np.minimum((u[:, j] * 16).astype(int), 15), minlength=16)
        exp = len(u) / 16
        assert np.sum((cnt - exp) ** 2 / exp) < 37.7


def test_near_contact_construction(orc, wl, r7, r14):
    """The near-contact edge sets land where they are meant to: every built
    configuration's oracle clearance is within 1 um of its target (1e-6 ..
    1e-3 m either side of contact), a zero-length edge's clearance is that
    configuration's, and exactly the edges within 1e-5 m are flagged."""
    import near_contact as NC
    for name, robot, prims in NC.graze_scenes(wl, r7, r14):
        cf = NC.graze_configs(orc, robot, prims, 2, seed=11)
        assert len(cf) == 2 * len(NC.TARGETS), name
        for q, c, m, _, _ in cf:
            assert abs(m - c) <= 1e-6, (name, c, m)
        a, b = NC.graze_edges(cf)
        rob = orc.OracleRobot(robot)
        v, f, me = orc.check_edges(rob, prims, a, b, 32.0, early_exit=False, want_m=True)
        assert np.array_equal(me[0::2], [m for _, _, m, _, _ in cf]), name
        assert np.array_equal(f.astype(bool), np.abs(me) <= orc.FLAG_BAND), name
        assert np.array_equal(v.astype(bool), me >= 0), name
        # both sides of the band are populated
        assert np.sum((me > orc.FLAG_BAND) & (me < 1e-4)) >= 4 and np.sum((me < -orc.FLAG_BAND) & (me > -1e-4)) >= 4
