"""GPU parity of prrtc_plan (Alg. 1 in deterministic rounds) against the
oracle's round replay, through the C ABI.

Several paths are correct for a planning query, so parity is: (i) every GPU
path is oracle-valid at 4x the planning resolution, starts and ends exactly
at the query and has segments no longer than delta; (ii) runs are
reproducible; (iii) when the oracle's replay meets no edge within the 1e-5 m
flag band, the GPU returns the identical path, round count, tree sizes and
edge count.
"""
import sys

import numpy as np
import pytest

from conftest import free_query, path_ok, replay_equal
from paper_2503_06757_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def params(P, **kw):
    p = P.prrtc_plan_params_default()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("instance", range(6))
def test_plan_r7_s12_replay(gpu, orc, r7, instance):
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, instance)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY + instance)
    say("plan R7 S12 instance", instance)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=11 + instance, max_rounds=300))
    assert st == 0, (st, stats)
    path_ok(orc, r7, prims, path, s, g)
    replay_equal(orc, r7, prims, s, g, st, path, stats, seed=11 + instance, max_rounds=300)


def test_plan_reproducible(gpu, orc, r7):
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, 4)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY + 4)
    say("reproducibility x8")
    ref = None
    for _ in range(8):
        st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=99))
        assert st == 0
        key = (path.tobytes(), stats["rounds"], stats["nodes_a"], stats["nodes_b"], stats["edges_checked"])
        ref = ref or key
        assert key == ref


@pytest.mark.parametrize("workers", [1, 7, 64, 300])
def test_plan_worker_counts(gpu, orc, r7, workers):
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, 2)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY + 2)
    say("workers", workers)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=5, workers=workers, max_rounds=400))
    assert st == 0
    path_ok(orc, r7, prims, path, s, g)
    replay_equal(orc, r7, prims, s, g, st, path, stats, seed=5, workers=workers, max_rounds=400)


def test_plan_validation_failures_replay(gpu, orc, r7):
    """Coarse resolution (2/rad): accepted paths clip obstacles; the 4x
    re-check blocks nodes and the rounds continue, as in the oracle."""
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, 1)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY + 1)
    say("validation failures replay")
    kw = dict(seed=3, workers=64, res=2.0, max_rounds=300)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
    assert st == 0 and stats["validation_failures"] >= 1
    path_ok(orc, r7, prims, path, s, g, res=2.0)
    replay_equal(orc, r7, prims, s, g, st, path, stats, **kw)
    st0, path0, stats0 = P.prrtc_plan(ctx, rid, sid, s, g, params(P, validate_factor=0, **kw))
    assert st0 == 0 and stats0["validation_failures"] == 0
    replay_equal(orc, r7, prims, s, g, st0, path0, stats0, validate_factor=0, **kw)


@pytest.mark.parametrize("k", range(4))
def test_plan_r14_replay(gpu, orc, r14, k):
    """Dual arm (inter-arm self pairs) among 12 random obstacles."""
    P, ctx, _ = gpu
    prims = W.scene_mixed(0x53140000 + k, r14, 12)
    rid, sid = P.prrtc_load_robot(ctx, r14), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r14), prims, r14, W.SEED_QUERY + 100 + k, n=3000)
    say("plan R14 mixed", k)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=7 + k, max_rounds=100))
    assert st == 0, (st, stats)
    path_ok(orc, r14, prims, path, s, g)
    replay_equal(orc, r14, prims, s, g, st, path, stats, seed=7 + k, max_rounds=100)


@pytest.mark.parametrize("instance,radius,tries", [(1, 0.1, 4), (4, 0.2, 2), (3, 0.05, 8)])
def test_plan_r7_dynamic_domain_replay(gpu, orc, r7, instance, radius, tries):
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, instance)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY + instance)
    say("dynamic domain", instance, radius, tries)
    kw = dict(seed=21 + instance, max_rounds=300, dds_radius=radius, dds_tries=tries)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
    assert st == 0, (st, stats)
    path_ok(orc, r7, prims, path, s, g)
    replay_equal(orc, r7, prims, s, g, st, path, stats, **kw)


def test_plan_r14_dynamic_domain_replay(gpu, orc, r14):
    P, ctx, _ = gpu
    prims = W.scene_mixed(0x53140000, r14, 12)
    rid, sid = P.prrtc_load_robot(ctx, r14), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r14), prims, r14, W.SEED_QUERY + 100, n=3000)
    say("dynamic domain R14")
    kw = dict(seed=7, max_rounds=60, dds_radius=0.15, dds_tries=4)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
    if st == 0:
        path_ok(orc, r14, prims, path, s, g)
    replay_equal(orc, r14, prims, s, g, st, path, stats, **kw)


def test_plan_status_codes(gpu, orc, r7):
    P, ctx, _ = gpu
    prims = W.scene_s12(r7, 0)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, W.SEED_QUERY)
    say("status codes")
    st, _, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, max_rounds=0))
    assert st == P.PRRTC_E_NO_SOLUTION and stats["rounds"] == 0
    bad = s.copy()
    bad[0] = 3.0
    assert P.prrtc_plan(ctx, rid, sid, bad, g, params(P))[0] == P.PRRTC_E_INVALID_ENDPOINT
    big = W.make_prims([(W.PRIM_SPHERE, (0, 0, 0.5), np.eye(3), (5.0, 0, 0))])
    sid_big = P.prrtc_load_scene(ctx, big)
    assert P.prrtc_plan(ctx, rid, sid_big, s, g, params(P))[0] == P.PRRTC_E_INVALID_ENDPOINT
    # the endpoints are checked even when no round may run (as the oracle does)
    assert P.prrtc_plan(ctx, rid, sid_big, s, g, params(P, max_rounds=0))[0] == P.PRRTC_E_INVALID_ENDPOINT
    # two-call pattern: too small a buffer reports the size needed
    st, _, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=1), path_cap=1)
    assert st == P.PRRTC_E_CAPACITY and stats["path_len"] > 1
    st2, path2, stats2 = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=1), path_cap=stats["path_len"])
    assert st2 == 0 and path2.shape[0] == stats["path_len"]
    # argument errors are raised by the binding
    for kw in (dict(workers=0), dict(delta=0.0), dict(res=-1.0), dict(tree_capacity=1),
               dict(max_rounds=-1), dict(dds_tries=0), dict(dds_radius=-1.0)):
        with pytest.raises(P.PrrtcError):
            P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
    # more workers than can be resident at once: refused before any launch
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, workers=4096, tile=64))
    assert st == P.PRRTC_E_CAPACITY and path is None and stats["path_len"] == 0
    assert "workers do not fit" in P.prrtc_last_error(ctx)
    # a tiny tree fills up; the planner stops cleanly
    st, _, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, tree_capacity=2, workers=8, max_rounds=20))
    assert st in (0, P.PRRTC_E_NO_SOLUTION) and stats["nodes_a"] <= 2 and stats["nodes_b"] <= 2


def test_plan_time_budget(gpu, orc, r7):
    """A query the planner does not solve quickly in the 64-obstacle scene
    stops on the 20 ms time budget long before its round budget."""
    P, ctx, _ = gpu
    prims = W.scene_s64(r7)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    s, g = free_query(orc, orc.OracleRobot(r7), prims, r7, 5)
    say("time budget")
    st, _, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, max_rounds=100000, time_budget_ms=20.0))
    assert st in (0, P.PRRTC_E_NO_SOLUTION)
    if st == P.PRRTC_E_NO_SOLUTION:
        assert stats["rounds"] < 100000 and stats["gpu_ms"] < 2000


@pytest.mark.parametrize("tile", [64, 16])
def test_plan_r14_shelf_queries(gpu, orc, r14, tile):
    """Stored dual-arm shelf queries under a short budget: every call ends in
    a solution or E_NO_SOLUTION (never a device abort, e.g. a group barrier
    that waited for a generation already released), and every solution is
    oracle-valid at 4x.  The four-wave workers (tile 64) meet at the same
    barriers as the one-wave workers (tile 16)."""
    import os
    P, ctx, _ = gpu
    say("R14 shelf queries, tile", tile)
    prims = W.scene_shelf(r14)
    rid, sid = P.prrtc_load_robot(ctx, r14), P.prrtc_load_scene(ctx, prims)
    Q = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "shelf_queries_r14.txt"), dtype=np.float32)
    solved = 0
    for k in range(20):
        s, g = Q[k, :14], Q[k, 14:]
        st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, seed=W.SEED_QUERY + k, max_rounds=4000,
                                                                   time_budget_ms=60.0, tile=tile))
        assert st in (0, P.PRRTC_E_NO_SOLUTION), (k, st)
        if st == 0:
            solved += 1
            path_ok(orc, r14, prims, path, s, g)
    say("  solved", solved, "of 20")


def test_plan_r14_shelf_replay(gpu, orc, r14):
    """Stored dual-arm shelf queries, bounded by 40 rounds (no time budget,
    so the run is a pure function of the seed): the GPU's status, rounds,
    trees, edge count and path equal the oracle's replay whenever the replay
    met no edge within the flag band."""
    import os
    P, ctx, _ = gpu
    say("R14 shelf replay")
    prims = W.scene_shelf(r14)
    rid, sid = P.prrtc_load_robot(ctx, r14), P.prrtc_load_scene(ctx, prims)
    Q = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "shelf_queries_r14.txt"), dtype=np.float32)
    replayed = solved = 0
    for k in range(8):
        s, g = Q[k, :14], Q[k, 14:]
        kw = dict(seed=W.SEED_QUERY + k, max_rounds=40)
        st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
        assert st in (0, P.PRRTC_E_NO_SOLUTION), (k, st)
        if st == 0:
            solved += 1
            path_ok(orc, r14, prims, path, s, g)
        replayed += replay_equal(orc, r14, prims, s, g, st, path, stats, **kw)
    say("  %d of 8 replayed, %d solved within 40 rounds" % (replayed, solved))
    assert replayed >= 4


@pytest.mark.parametrize("case", ["s12-0", "s12-3", "r14-1", "s64-0", "s64-3", "s64-dds"])
def test_plan_halton_replay(gpu, orc, r7, r14, case):
    """Halton samples (sampler 2): the GPU plan equals the oracle's replay,
    also over many rounds (64-obstacle scene, 40 rounds, solved or not) and
    with dynamic-domain redraws (several tries per worker and round)."""
    P, ctx, _ = gpu
    kind, k = case.split("-")
    robot = r14 if kind == "r14" else r7
    rob = orc.OracleRobot(robot)
    kw = dict(seed=0x1234, max_rounds=300, sampler=2, workers=128)
    if kind == "s12":
        prims = W.scene_s12(robot, int(k))
        s, g = free_query(orc, rob, prims, robot, W.SEED_QUERY + int(k))
    elif kind == "r14":
        prims = W.scene_mixed(0x53140000 + int(k), robot, 12)
        s, g = free_query(orc, rob, prims, robot, W.SEED_QUERY + 100 + int(k), n=3000)
    else:
        prims = W.scene_s64(robot)
        kk = 0 if k == "dds" else int(k)
        s, g = free_query(orc, rob, prims, robot, W.SEED_QUERY + 300 + kk, n=2000)
        kw = dict(seed=0x1234 + kk, max_rounds=40, sampler=2, workers=64, dds_tries=2)
        if k == "dds":
            kw.update(dds_radius=0.2, dds_tries=3)
    rid, sid = P.prrtc_load_robot(ctx, robot), P.prrtc_load_scene(ctx, prims)
    say("Halton plan", case)
    st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
    assert st in (0, P.PRRTC_E_NO_SOLUTION), (st, stats)
    if st == 0:
        path_ok(orc, robot, prims, path, s, g)
    assert replay_equal(orc, robot, prims, s, g, st, path, stats, **kw)


@pytest.mark.parametrize("instance", [0, 4])
def test_plan_esdf_replay(gpu, orc, r7, instance):
    """Planning against an ESDF grid (the oracle's grid of a 12-obstacle
    scene, no primitives): the GPU plan equals the oracle's replay."""
    P, ctx, _ = gpu
    o, h, n = (-1.3, -1.3, -1.3), 2.6 / 63, (64, 64, 64)
    prims = W.scene_s12(r7, instance)
    grid = orc.EsdfGrid(o, h, orc.esdf_of_scene(prims, o, h, n))
    empty = np.zeros(0, W.PRIM_DTYPE)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, empty)
    P.prrtc_scene_set_esdf(ctx, sid, o, h, grid.values)
    say("ESDF plan", instance)
    kw = dict(seed=31 + instance, max_rounds=300)
    with grid:
        s, g = free_query(orc, orc.OracleRobot(r7), empty, r7, W.SEED_QUERY + instance)
        st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, **kw))
        assert st == 0, (st, stats)
        path_ok(orc, r7, empty, path, s, g)
        assert replay_equal(orc, r7, empty, s, g, st, path, stats, **kw)


@pytest.mark.parametrize("case", ["r7-0", "r7-3", "r14-1"])
def test_plan_two_stage_replay(gpu, orc, r7, r14, case):
    """Plans of a robot with coarse spheres (two-stage checks in the planner's
    edge and connect checks) equal the oracle's replay of the fine robot."""
    P, ctx, _ = gpu
    name, k = case.split("-")
    robot = r7 if name == "r7" else r14
    if name == "r7":
        prims = W.scene_s12(robot, int(k))
        s, g = free_query(orc, orc.OracleRobot(robot), prims, robot, W.SEED_QUERY + int(k))
    else:
        prims = W.scene_mixed(0x53140000 + int(k), robot, 12)
        s, g = free_query(orc, orc.OracleRobot(robot), prims, robot, W.SEED_QUERY + 100 + int(k), n=3000)
    say("two-stage plan", case)
    for tile in (64, 16):
        rid = P.prrtc_load_robot(ctx, W.with_coarse_spheres(robot))
        sid = P.prrtc_load_scene(ctx, prims)
        kw = dict(seed=77 + int(k), max_rounds=300)
        st, path, stats = P.prrtc_plan(ctx, rid, sid, s, g, params(P, tile=tile, **kw))
        assert st == 0, (st, stats)
        path_ok(orc, robot, prims, path, s, g)
        assert replay_equal(orc, robot, prims, s, g, st, path, stats, **kw)
