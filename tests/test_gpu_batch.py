"""GPU tests of prrtc_plan_batch: many queries in one persistent launch,
one group of workers per query.  Every query must come out exactly as the
single-query planner returns it with the same parameters, seed and query
word (the oracle parity of that planner is covered by its own tests)."""
import sys

import numpy as np
import pytest

from conftest import free_query, path_ok, replay_equal
from paper_2503_06757_amd import proposal as PR
from paper_2503_06757_amd import workloads as W

pytestmark = pytest.mark.gpu

KEYS = ("rounds", "nodes_a", "nodes_b", "edges_checked", "validation_failures", "connect_worker",
        "learned_samples", "fallback")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def params(P, **kw):
    p = P.prrtc_plan_params_default()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# (robot id, scene id) of the module's queries -> (robot, primitives), for the oracle
SCENES = {}


def oracle_replay(orc, q, st, path, stats, **kw):
    """Query q's GPU result against the oracle's replay of the same query
    (seed, query word and parameters); every solution oracle-valid."""
    robot, prims = SCENES[(q[0], q[1])]
    rid, sid, s, g, seed, qw = q
    if st == 0:
        path_ok(orc, robot, prims, path, s, g, res=kw.get("res", 32.0))
    return replay_equal(orc, robot, prims, s, g, st, path, stats, seed=seed, query=qw, **kw)


@pytest.fixture(scope="module")
def mixed(gpu, orc, r7, r14):
    """12 R7 queries over 6 S12 scenes and 4 R14 queries on S12 scenes."""
    P, ctx, _ = gpu
    rid7, rid14 = P.prrtc_load_robot(ctx, r7), P.prrtc_load_robot(ctx, r14)
    qs = []
    for inst in range(6):
        prims = W.scene_s12(r7, inst)
        sid = P.prrtc_load_scene(ctx, prims)
        SCENES[(rid7, sid)] = (r7, prims)
        rob = orc.OracleRobot(r7)
        for j in range(2):
            s, g = free_query(orc, rob, prims, r7, W.SEED_QUERY + 100 * j + inst)
            qs.append((rid7, sid, s, g, 70 + 10 * inst + j, j))
    for inst in range(4):
        prims = W.scene_s12(r14, inst)
        sid = P.prrtc_load_scene(ctx, prims)
        SCENES[(rid14, sid)] = (r14, prims)
        s, g = free_query(orc, orc.OracleRobot(r14), prims, r14, W.SEED_QUERY + 500 + inst)
        qs.append((rid14, sid, s, g, 900 + inst, 3))
    return qs


def _single(P, ctx, q, prm):
    rid, sid, s, g, seed, qw = q[:6]
    prm.seed, prm.query = seed, qw
    if len(q) > 6 and q[6] >= 0:
        prm.model_id = q[6]          # the query's own proposal model
    return P.prrtc_plan(ctx, rid, sid, s, g, prm)


@pytest.mark.parametrize("groups,workers", [(4, 64), (16, 32), (0, 128)])
def test_batch_equals_single(gpu, orc, mixed, groups, workers):
    """Every query of a batch equals its single-query plan and the oracle's
    replay of it."""
    P, ctx, _ = gpu
    say("batch of %d queries, groups %d, workers %d" % (len(mixed), groups, workers))
    prm = params(P, workers=workers, max_rounds=500)
    used, out = P.prrtc_plan_batch(ctx, mixed, prm, groups=groups, path_cap=512)
    say("  groups used", used)
    # groups = 0: as many as are resident at once (LDS and registers decide), at most one per query
    assert used == groups if groups else 1 <= used <= len(mixed)
    for k, q in enumerate(mixed):
        st, path, stats = out[k]
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=workers, max_rounds=500))
        assert st == st1, (k, st, st1)
        for key in KEYS:
            assert stats[key] == stats1[key], (k, key, stats[key], stats1[key])
        if st == 0:
            assert np.array_equal(path, path1), k
    replayed = sum(oracle_replay(orc, q, *out[k], workers=workers, max_rounds=500) for k, q in enumerate(mixed))
    say("  %d of %d queries replayed by the oracle" % (replayed, len(mixed)))
    assert replayed >= len(mixed) - 2


def test_batch_rejections_and_budget(gpu, mixed, r7):
    P, ctx, _ = gpu
    say("batch rejections and memory budget")
    rid, sid = mixed[0][0], mixed[0][1]
    bad_limits = (rid, sid, np.full(7, 9.0, np.float32), mixed[0][3], 1, 0)
    bad_scene = (rid, 10_000, mixed[0][2], mixed[0][3], 1, 0)
    qs = [mixed[0], bad_limits, mixed[1], bad_scene, mixed[2]]
    prm = params(P, workers=32, max_rounds=500, tree_capacity=4096)
    used, out = P.prrtc_plan_batch(ctx, qs, prm, groups=0, path_cap=256)
    assert [o[0] for o in out][1] == P.PRRTC_E_INVALID_ENDPOINT
    assert [o[0] for o in out][3] == P.PRRTC_E_STATE
    for k in (0, 2, 4):
        st1, path1, _ = _single(P, ctx, qs[k], params(P, workers=32, max_rounds=500, tree_capacity=4096))
        assert out[k][0] == st1 and (st1 != 0 or np.array_equal(out[k][1], path1))
    # a budget for about one group: the launch runs everything on fewer groups
    used1, out1 = P.prrtc_plan_batch(ctx, [mixed[0], mixed[1], mixed[2]], prm, groups=0,
                                     memory_budget=1_000_000, path_cap=256)
    say("  groups under the budget:", used1)
    assert used1 >= 1 and used1 < 3
    for k in range(3):
        assert out1[k][0] == out[[0, 2, 4][k]][0]
    with pytest.raises(P.PrrtcError):
        P.prrtc_plan_batch(ctx, [mixed[0]], prm, memory_budget=1000, path_cap=256)
    # capacity: a path longer than path_cap is reported, not written
    used2, out2 = P.prrtc_plan_batch(ctx, [mixed[0]], params(P, workers=32, max_rounds=500), path_cap=1)
    if out[0][0] == 0:
        assert out2[0][0] == P.PRRTC_E_CAPACITY and out2[0][2]["path_len"] > 1


def _learned_models(P, ctx, seed):
    m7 = P.prrtc_load_proposal(ctx, PR.pack(PR.init_params(7, seed), 7))
    m14 = P.prrtc_load_proposal(ctx, PR.pack(PR.init_params(14, seed + 1), 14))
    return m7, m14


def _with_models(qs, m7, m14):
    """Each query with its own model: the 7-DoF model for the arm, the
    14-DoF one for the dual arm."""
    return [q[:6] + ((m7 if len(q[2]) == 7 else m14),) for q in qs]


def test_batch_learned_equals_single(gpu, mixed):
    """A learned batch of both robots (per-query models, more queries than a
    small batch): each worker group computes its query's mixture in the
    launch, and every query equals its single learned plan."""
    P, ctx, _ = gpu
    say("learned batch, mixed robots")
    m7, m14 = _learned_models(P, ctx, 77)
    qs = _with_models(mixed + [q[:4] + (q[4] + 1000, q[5]) for q in mixed[:8]], m7, m14)   # 24 queries
    prm = params(P, workers=64, max_rounds=500, sampler=1, model_id=m7, mix=0.7)
    used, out = P.prrtc_plan_batch(ctx, qs, prm, groups=3, path_cap=512)
    for k, q in enumerate(qs):
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=64, max_rounds=500, sampler=1, model_id=m7,
                                                       mix=0.7))
        st, path, stats = out[k]
        assert st == st1, (k, st, st1)
        for key in KEYS:
            assert stats[key] == stats1[key], (k, key)
        if st == 0:
            assert np.array_equal(path, path1)
    # the untrained 14-DoF mixture rarely lands inside all 14 limits; the 7-DoF one often does
    assert all(out[k][2]["learned_samples"] > 0 for k, q in enumerate(qs) if len(q[2]) == 7)
    # a query whose model does not match its robot is refused alone
    bad = [qs[0], qs[-1][:6] + (m7,) if len(qs[-1][2]) == 14 else qs[-1][:6] + (m14,), qs[1]]
    used, out2 = P.prrtc_plan_batch(ctx, bad, prm, groups=2, path_cap=512)
    assert out2[1][0] == P.PRRTC_E_ARG
    assert out2[0][0] == out[0][0] and out2[2][0] == out[1][0]


def test_serving_submit_poll(gpu, orc, mixed):
    """Queries submitted to the serving thread come out as single launches
    plan them; admission refuses submissions beyond max_pending until
    results are polled; other calls are refused while serving."""
    import time
    P, ctx, _ = gpu
    say("serving: submit / poll")
    prm = params(P, workers=64, max_rounds=500)
    P.prrtc_serve_start(ctx, prm, slots=6, max_pending=len(mixed), memory_budget=0, path_cap=512)
    try:
        with pytest.raises(P.PrrtcError):
            P.prrtc_plan(ctx, mixed[0][0], mixed[0][1], mixed[0][2], mixed[0][3], prm)
        tickets = [P.prrtc_submit(ctx, *q) for q in mixed]
        assert all(t is not None for t in tickets)
        assert P.prrtc_submit(ctx, *mixed[0]) is None          # admission: max_pending reached
        got = {}
        t0 = time.time()
        while len(got) < len(tickets) and time.time() - t0 < 60:
            for t, q in zip(tickets, mixed):
                if t not in got:
                    r = P.prrtc_poll(ctx, t, len(q[2]), 512)
                    if r is not None:
                        got[t] = r
            time.sleep(0.001)
        assert len(got) == len(tickets)
        with pytest.raises(P.PrrtcError):
            P.prrtc_poll(ctx, tickets[0], 7, 512)                # released
        assert P.prrtc_submit(ctx, *mixed[0]) is not None
    finally:
        launches = P.prrtc_serve_stop(ctx)
    say("  launches", launches)
    assert 1 <= launches <= len(mixed) + 1
    replayed = 0
    for t, q in zip(tickets, mixed):
        st, path, stats = got[t]
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=64, max_rounds=500))
        assert st == st1
        for key in KEYS:
            assert stats[key] == stats1[key], key
        if st == 0:
            assert np.array_equal(path, path1)
        replayed += oracle_replay(orc, q, st, path, stats, workers=64, max_rounds=500)
    say("  %d of %d served queries replayed by the oracle" % (replayed, len(mixed)))
    assert replayed >= len(mixed) - 2


def test_serving_ring_drains_and_relaunches(gpu, orc, mixed):
    """A uniform-sampling server plans in one persistent launch whose ring
    holds 64 x slots queries (at least 32); more submissions than that make
    the launch drain and a new one start on the reset ring.  Every result
    still equals the single-launch plan, whichever launch ran it."""
    import time
    P, ctx, _ = gpu
    say("serving: ring drain and relaunch")
    prm = params(P, workers=32, max_rounds=300)
    qs = [mixed[i % len(mixed)][:4] + (500 + i, i % 3) for i in range(3 * 64 + 7)]
    P.prrtc_serve_start(ctx, prm, slots=1, max_pending=len(qs), memory_budget=0, path_cap=512)
    try:
        tickets = [P.prrtc_submit(ctx, *q) for q in qs]
        assert all(t is not None for t in tickets)
        got = {}
        t0 = time.time()
        while len(got) < len(tickets) and time.time() - t0 < 120:
            for t, q in zip(tickets, qs):
                if t not in got:
                    r = P.prrtc_poll(ctx, t, len(q[2]), 512)
                    if r is not None:
                        got[t] = r
            time.sleep(0.001)
        assert len(got) == len(tickets)
    finally:
        launches = P.prrtc_serve_stop(ctx)
    say("  launches", launches)
    assert launches >= 4
    for t, q in list(zip(tickets, qs))[::5]:
        st, path, stats = got[t]
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=32, max_rounds=300))
        assert st == st1
        for key in KEYS:
            assert stats[key] == stats1[key], key
        if st == 0:
            assert np.array_equal(path, path1)
    for t, q in list(zip(tickets, qs))[::23]:
        oracle_replay(orc, q, *got[t], workers=32, max_rounds=300)


def test_serving_relaunch_after_idle(gpu, orc, mixed):
    """The persistent serving launch leaves after 50 ms without work; a later
    submission starts a new one and is answered like the first."""
    import time
    P, ctx, _ = gpu
    say("serving: idle exit and relaunch")
    prm = params(P, workers=32, max_rounds=300)

    def run(qs):
        tickets = [P.prrtc_submit(ctx, *q) for q in qs]
        got = {}
        t0 = time.time()
        while len(got) < len(tickets) and time.time() - t0 < 60:
            for t, q in zip(tickets, qs):
                if t not in got:
                    r = P.prrtc_poll(ctx, t, len(q[2]), 512)
                    if r is not None:
                        got[t] = r
            time.sleep(0.001)
        assert len(got) == len(tickets)
        return [got[t] for t in tickets]

    P.prrtc_serve_start(ctx, prm, slots=4, max_pending=16, memory_budget=0, path_cap=512)
    try:
        first = run(mixed[:3])
        time.sleep(0.3)                     # longer than the idle limit: the launch has left
        second = run(mixed[3:6])
    finally:
        launches = P.prrtc_serve_stop(ctx)
    say("  launches", launches)
    assert launches >= 2
    for (st, path, stats), q in zip(first + second, mixed[:6]):
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=32, max_rounds=300))
        assert st == st1
        for key in KEYS:
            assert stats[key] == stats1[key], key
        if st == 0:
            assert np.array_equal(path, path1)
        oracle_replay(orc, q, st, path, stats, workers=32, max_rounds=300)


def test_serving_learned_equals_single(gpu, mixed):
    """A learned-sampler server runs the persistent launch too: each group
    computes its query's mixture from the scene's grid embedding (made when
    serving starts).  Both robots, each with its own model; every result
    equals the single learned plan of the same query."""
    import time
    P, ctx, _ = gpu
    say("serving with the learned sampler, both robots")
    m7, m14 = _learned_models(P, ctx, 78)
    qs = _with_models(mixed, m7, m14)
    prm = params(P, workers=64, max_rounds=500, sampler=1, model_id=m7, mix=0.7)
    P.prrtc_serve_start(ctx, prm, slots=3, max_pending=len(qs) + 1, memory_budget=0, path_cap=512)
    try:
        tickets = [P.prrtc_submit(ctx, *q) for q in qs]
        # a query whose model does not fit its robot comes back refused
        wrong = qs[-1][:6] + (m7,) if len(qs[-1][2]) == 14 else qs[0][:6] + (m14,)
        t_wrong = P.prrtc_submit(ctx, *wrong)
        got = {}
        t0 = time.time()
        while len(got) < len(tickets) + 1 and time.time() - t0 < 60:
            for t, q in zip(tickets + [t_wrong], qs + [wrong]):
                if t not in got:
                    r = P.prrtc_poll(ctx, t, len(q[2]), 512)
                    if r is not None:
                        got[t] = r
            time.sleep(0.001)
        assert len(got) == len(tickets) + 1
    finally:
        launches = P.prrtc_serve_stop(ctx)
    say("  launches", launches)
    assert launches >= 1
    assert got[t_wrong][0] == P.PRRTC_E_ARG
    for t, q in zip(tickets, qs):
        st, path, stats = got[t]
        st1, path1, stats1 = _single(P, ctx, q, params(P, workers=64, max_rounds=500, sampler=1, model_id=m7,
                                                         mix=0.7))
        assert st == st1
        for key in KEYS:
            assert stats[key] == stats1[key], key
        if len(q[2]) == 7:
            assert stats["learned_samples"] > 0
        if st == 0:
            assert np.array_equal(path, path1)


def test_tune_launch_and_tiles(gpu, mixed):
    """The tuner returns the fastest (workers, tile) pair; the FK tile changes
    only speed: every query plans identically with tile 16 and tile 64."""
    P, ctx, _ = gpu
    say("launch-shape tuning")
    (bw, bt), rates = P.prrtc_tune_launch(ctx, mixed, params(P, max_rounds=300), workers=(16, 32, 64),
                                          tiles=(16, 64))
    say("  best", bw, bt, rates)
    assert (bw, bt) in rates and rates[(bw, bt)] == max(rates.values())
    assert all(r > 0 for r in rates.values())
    # a shape that cannot be resident at all rates 0 and is never chosen
    (bw2, _), rates2 = P.prrtc_tune_launch(ctx, mixed[:2], params(P, max_rounds=50, tree_capacity=4096),
                                           workers=(32, 4096), tiles=(16,), memory_budget=4 << 20)
    assert bw2 == 32 and rates2[(4096, 16)] == 0.0
    for q in mixed[:6] + mixed[-2:]:
        outs = [_single(P, ctx, q, params(P, workers=64, max_rounds=500, tile=t)) for t in (16, 64)]
        assert outs[0][0] == outs[1][0]
        for key in KEYS:
            assert outs[0][2][key] == outs[1][2][key], key
        if outs[0][0] == 0:
            assert np.array_equal(outs[0][1], outs[1][1])
    with pytest.raises(P.PrrtcError):
        _single(P, ctx, mixed[0], params(P, tile=32))


def test_tuning_records_persist(gpu, mixed, r7, tmp_path):
    """What a context timed (the check_edges schedule of a robot and scene
    shape, the best launch shape for a query mix) is saved to a file and
    taken up by a new context without timing again."""
    P, ctx, torch = gpu
    say("tuning records")
    prims = W.scene_s64(r7)
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, prims)
    P.prrtc_edge_schedule(ctx, rid, sid, -1)
    a, b = W.random_edges(r7, 16384, seed=31)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    tv = torch.zeros(16384, dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), 16384, 32.0, tv.data_ptr(), None)
    torch.cuda.synchronize()
    chosen = P.prrtc_edge_schedule(ctx, rid, sid)
    assert chosen in (0, 1)
    best, _ = P.prrtc_tune_launch(ctx, mixed[:4], params(P, max_rounds=100), workers=(16, 32), tiles=(16,))
    assert P.prrtc_tuned_launch(ctx, mixed[:4], workers=(16, 32), tiles=(16,)) == best
    assert P.prrtc_tuned_launch(ctx, mixed[:4], workers=(16, 64), tiles=(16,)) is None   # other candidates
    path = str(tmp_path / "tuning.txt")
    P.prrtc_tuning_save(ctx, path)
    ctx2 = P.prrtc_create(0)
    try:
        rid2 = P.prrtc_load_robot(ctx2, r7)
        sid2 = P.prrtc_load_scene(ctx2, W.scene_s64(r7, seed=W.SEED_S64 + 5))   # same shape, other scene
        assert P.prrtc_edge_schedule(ctx2, rid2, sid2) == -1
        P.prrtc_tuning_load(ctx2, path)
        assert P.prrtc_edge_schedule(ctx2, rid2, sid2) == chosen
        q2 = [(rid2, sid2) + q[2:] for q in mixed[:4] if len(q[2]) == 7]
        assert P.prrtc_tuned_launch(ctx2, q2, workers=(16, 32), tiles=(16,)) is None   # another query mix
        bad = tmp_path / "bad.txt"
        bad.write_text("no separator here\n")
        with pytest.raises(P.PrrtcError) as e:
            P.prrtc_tuning_load(ctx2, str(bad))
        assert e.value.status == P.PRRTC_E_ARG
    finally:
        P.prrtc_destroy(ctx2)
