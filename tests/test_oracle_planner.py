"""Pins of the oracle's planner (Alg. 1 in deterministic rounds): properties
every returned path must have, closed-form special cases and failure codes."""
import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W

E_INVALID_ENDPOINT, E_NO_SOLUTION, E_ARG = -4, -5, -1


def _first_free_query(orc, rob, prims, robot, seed, n=50):
    for s, g in W.query_candidates(robot, seed, n):
        if (orc.config_clearance(rob, prims, s.astype(np.float64)) > 1e-4 and
                orc.config_clearance(rob, prims, g.astype(np.float64)) > 1e-4):
            return s, g
    raise RuntimeError("no free query")


def _check_path_properties(orc, rob, prims, path, s, g, delta, res):
    assert np.array_equal(path[0], s) and np.array_equal(path[-1], g)
    seg = np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1)
    assert np.all(seg <= delta * (1 + 1e-6))
    m, _ = orc.path_clearance(rob, prims, path, 4 * res)
    assert m >= -orc.FLAG_BAND


def test_empty_scene_connects_in_first_round(orc, r7):
    rob = orc.OracleRobot(r7)
    empty = np.zeros(0, W.PRIM_DTYPE)
    s, g = W.query_candidates(r7, 17, 1)[0]
    st, path, stats = orc.plan(rob, empty, s, g, seed=5, workers=16, max_rounds=5)
    assert st == 0 and stats["rounds"] == 1 and stats["connect_worker"] == 0
    _check_path_properties(orc, rob, empty, path, s, g, 0.5, 32.0)
    # with nothing in the way the path is start -> extension -> straight connect: its
    # arclength is at least |g - s| and at most |g - s| + 2 delta
    cost = np.sum(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1))
    direct = np.linalg.norm(g.astype(np.float64) - s)
    assert direct - 1e-6 <= cost <= direct + 2 * 0.5 + 1e-6


@pytest.mark.parametrize("instance", [0, 1])
def test_s12_paths_valid_and_deterministic(orc, r7, instance):
    rob = orc.OracleRobot(r7)
    prims = W.scene_s12(r7, instance)
    s, g = _first_free_query(orc, rob, prims, r7, W.SEED_QUERY + instance)
    st, path, stats = orc.plan(rob, prims, s, g, seed=11, workers=32, max_rounds=200)
    assert st == 0, stats
    _check_path_properties(orc, rob, prims, path, s, g, 0.5, 32.0)
    st2, path2, stats2 = orc.plan(rob, prims, s, g, seed=11, workers=32, max_rounds=200)
    assert st2 == 0 and np.array_equal(path, path2) and stats == stats2
    # a different seed explores differently but still gives a valid path
    st3, path3, _ = orc.plan(rob, prims, s, g, seed=12, workers=32, max_rounds=200)
    assert st3 == 0
    _check_path_properties(orc, rob, prims, path3, s, g, 0.5, 32.0)


def test_validation_failures_block_and_recover(orc, r7):
    """At a coarse resolution (2 points/rad) accepted edges can clip obstacles
    between their points; the 4x re-check must reject such paths (blocking the
    offending node) and the path finally returned is valid at 4x resolution.
    Instance 1 of the 12-obstacle scene with seed 3 hits this case twice."""
    rob = orc.OracleRobot(r7)
    prims = W.scene_s12(r7, 1)
    s, g = _first_free_query(orc, rob, prims, r7, W.SEED_QUERY + 1)
    st, path, stats = orc.plan(rob, prims, s, g, seed=3, workers=64, res=2.0, max_rounds=300)
    assert st == 0 and stats["validation_failures"] >= 1
    _check_path_properties(orc, rob, prims, path, s, g, 0.5, 2.0)
    # with the re-check off the first connection is accepted, earlier, and its
    # path is not valid at 4x the resolution
    st0, path0, stats0 = orc.plan(rob, prims, s, g, seed=3, workers=64, res=2.0, max_rounds=300,
                                  validate_factor=0)
    assert st0 == 0 and stats0["validation_failures"] == 0
    assert stats0["rounds"] < stats["rounds"]
    m0, _ = orc.path_clearance(rob, prims, path0, 8.0)
    assert m0 < 0


def test_failure_codes(orc, r7):
    rob = orc.OracleRobot(r7)
    prims = W.scene_s12(r7, 0)
    s, g = _first_free_query(orc, rob, prims, r7, W.SEED_QUERY)
    st, _, _ = orc.plan(rob, prims, s, g, max_rounds=0)
    assert st == E_NO_SOLUTION
    bad = s.copy()
    bad[0] = 3.0                                        # outside the +-2.8 limits
    assert orc.plan(rob, prims, bad, g)[0] == E_INVALID_ENDPOINT
    big = W.make_prims([(W.PRIM_SPHERE, (0, 0, 0.5), np.eye(3), (5.0, 0, 0))])
    assert orc.plan(rob, big, s, g)[0] == E_INVALID_ENDPOINT
    assert orc.plan(rob, big, s, g, max_rounds=0)[0] == E_INVALID_ENDPOINT   # checked before any round
    assert orc.plan(rob, prims, s, g, workers=0)[0] == E_ARG
    # a tree of capacity 2 fills after one node; the planner must stop cleanly
    st, _, stats = orc.plan(rob, prims, s, g, tree_capacity=2, workers=8, max_rounds=20)
    assert st in (0, E_NO_SOLUTION)
    assert stats["nodes_a"] <= 2 and stats["nodes_b"] <= 2


def test_dynamic_domain_off_is_plain_and_on_is_valid(orc, r7):
    """With the dynamic domain off, extra draws are never used, so any number
    of tries reproduces the plain planner exactly; with it on, paths stay
    valid."""
    rob = orc.OracleRobot(r7)
    prims = W.scene_s12(r7, 4)
    s, g = _first_free_query(orc, rob, prims, r7, W.SEED_QUERY + 4)
    base = orc.plan(rob, prims, s, g, seed=8, workers=32, max_rounds=300)
    same = orc.plan(rob, prims, s, g, seed=8, workers=32, max_rounds=300, dds_radius=0.0, dds_tries=5)
    assert base[0] == same[0] == 0 and np.array_equal(base[1], same[1]) and base[2] == same[2]
    st, path, stats = orc.plan(rob, prims, s, g, seed=8, workers=32, max_rounds=300, dds_radius=0.1,
                               dds_tries=4)
    assert st == 0
    _check_path_properties(orc, rob, prims, path, s, g, 0.5, 32.0)


def test_dynamic_domain_shrinks_extensions(orc, r7):
    """Once a node's radius is set, accepted samples lie within it, so after
    failures near an enclosed goal the extensions get shorter: with a tiny
    radius and one try per round, far fewer samples are accepted than drawn."""
    rob = orc.OracleRobot(r7)
    prims = W.scene_s64(r7)
    s, g = _first_free_query(orc, rob, prims, r7, 5)
    _, _, plain = orc.plan(rob, prims, s, g, seed=4, workers=32, max_rounds=20)
    _, _, dds = orc.plan(rob, prims, s, g, seed=4, workers=32, max_rounds=20, dds_radius=0.01, dds_tries=1)
    # rejected samples check no edge
    assert dds["edges_checked"] < plain["edges_checked"]
