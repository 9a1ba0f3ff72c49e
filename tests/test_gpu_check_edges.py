"""GPU parity of prrtc_fk_spheres and prrtc_check_edges against the oracle,
through the C ABI (Alg. 2 / Sec. III-A)."""
import sys

import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W

pytestmark = pytest.mark.gpu

FK_TOL = 1e-5      # metres: FP32 sphere centres vs the FP64 oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_check(gpu, rid, sid, a, b, res=32.0):
    P, ctx, torch = gpu
    n = a.shape[0]
    ta = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tb = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    tv = torch.full((max(n, 1),), 7, dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n, res, tv.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return tv[:n].cpu().numpy()


def assert_parity(orc, robot, prims, a, b, got, res=32.0, threads=0):
    rob = orc.OracleRobot(robot)
    v, f, _ = orc.check_edges(rob, prims, a, b, res, early_exit=True, n_threads=threads)
    assert set(np.unique(got)) <= {0, 1}
    mism = (got != v) & (f == 0)
    assert not mism.any(), f"{mism.sum()} unflagged mismatches, first at {np.nonzero(mism)[0][:10]}"
    return v, f


@pytest.mark.parametrize("robot_name", ["r7", "r14"])
def test_fk_spheres_parity(gpu, orc, robot_name, request):
    """Worst case over 10^6 random configurations (a little outside the
    joint limits too) of the FP32 sphere centres against the FP64 oracle."""
    P, ctx, torch = gpu
    robot = request.getfixturevalue(robot_name)
    say("fk parity", robot_name)
    rid = P.prrtc_load_robot(ctx, robot)
    rng = np.random.default_rng(1)
    dof = W.robot_dof(robot)
    ns = robot["sphere_xyzr"].shape[0]
    rob = orc.OracleRobot(robot)
    n_total, chunk = 1 << 20, 1 << 16
    out = torch.zeros((chunk, ns, 3), dtype=torch.float32, device="cuda")
    err = 0.0
    for c0 in range(0, n_total, chunk):
        q = rng.uniform(-3.2, 3.2, (chunk, dof)).astype(np.float32)
        tq = torch.from_numpy(q).cuda()
        P.prrtc_fk_spheres(ctx, rid, tq.data_ptr(), chunk, out.data_ptr(),
                           torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        err = max(err, float(np.max(np.abs(got - orc.fk_spheres_batch(rob, q)))))
    say("  max |fk err| over %d configurations = %.3g m" % (n_total, err))
    assert err <= FK_TOL


def test_check_edges_parity_s12_s64(gpu, orc, r7):
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    for name, prims in (("S12", W.scene_s12(r7, 0)), ("S64", W.scene_s64(r7))):
        sid = P.prrtc_load_scene(ctx, prims)
        a, b = W.random_edges(r7, 20011, seed=1234)     # ragged count
        say("check_edges parity", name, a.shape)
        got = gpu_check(gpu, rid, sid, a, b)
        v, f = assert_parity(orc, r7, prims, a, b, got)
        say("  valid frac %.4f flagged %d" % (v.mean(), f.sum()))


def test_check_edges_schedules_agree(gpu, orc, r7, r14):
    """Both check_edges schedules (items per lane, obstacle-type order) give
    the oracle's verdicts on the same batch; the timed choice on the first
    large batch picks one of them and changes no verdict."""
    P, ctx, _ = gpu
    for robot, prims, name in ((r7, W.scene_s64(r7), "R7 S64"), (r14, W.scene_shelf(r14), "R14 shelf")):
        rid, sid = P.prrtc_load_robot(ctx, robot), P.prrtc_load_scene(ctx, prims)
        a, b = W.random_edges(robot, 12011, seed=4321)
        say("check_edges schedules", name, a.shape)
        # a pair of the same shape timed by an earlier test left a record
        # that a new pair adopts; forget it so this pair is timed afresh
        P.prrtc_edge_schedule(ctx, rid, sid, -1)
        assert P.prrtc_edge_schedule(ctx, rid, sid) == -1          # nothing chosen yet
        outs = []
        for k in (0, 1):
            assert P.prrtc_edge_schedule(ctx, rid, sid, k) == k
            outs.append(gpu_check(gpu, rid, sid, a, b))
        assert np.array_equal(outs[0], outs[1])
        assert_parity(orc, robot, prims, a, b, outs[0])
        assert P.prrtc_edge_schedule(ctx, rid, sid, -1) == -1
        got = gpu_check(gpu, rid, sid, a, b)                      # >= 8192 edges: times both
        chosen = P.prrtc_edge_schedule(ctx, rid, sid)
        say("  timed choice", chosen)
        assert chosen in (0, 1)
        assert np.array_equal(got, outs[0])
        with pytest.raises(P.PrrtcError):
            P.prrtc_edge_schedule(ctx, rid, sid, 2)


def test_check_edges_parity_r14_shelf(gpu, orc, r14):
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r14)
    prims = W.scene_shelf(r14)
    sid = P.prrtc_load_scene(ctx, prims)
    a, b = W.random_edges(r14, 3001, seed=77)
    say("check_edges parity R14 shelf", a.shape)
    got = gpu_check(gpu, rid, sid, a, b)
    v, f = assert_parity(orc, r14, prims, a, b, got)
    say("  valid frac %.4f flagged %d" % (v.mean(), f.sum()))
    # an empty scene leaves only the self pairs between the arms
    sid0 = P.prrtc_load_scene(ctx, np.zeros(0, W.PRIM_DTYPE))
    got0 = gpu_check(gpu, rid, sid0, a, b)
    v0, f0 = assert_parity(orc, r14, np.zeros(0, W.PRIM_DTYPE), a, b, got0)
    say("  self-only valid frac %.4f" % v0.mean())
    assert 0.0 < v0.mean() < 1.0


def test_check_edges_near_contact(gpu, orc, r7, r14):
    """Edges built to end 1e-6 .. 1e-3 m from contact, on either side, against
    each primitive type, the shelf's thin boards and the inter-arm pairs.
    Unflagged edges (|clearance| > 1e-5 m) must match the oracle; flagged
    ones are counted, with how many still agree."""
    import near_contact as NC
    P, ctx, _ = gpu
    say("near-contact edges")
    for name, robot, prims in NC.graze_scenes(W, r7, r14):
        rid, sid = P.prrtc_load_robot(ctx, robot), P.prrtc_load_scene(ctx, prims)
        cf = NC.graze_configs(orc, robot, prims, 12, seed=0x4E43)
        a, b = NC.graze_edges(cf)
        got = gpu_check(gpu, rid, sid, a, b)
        rob = orc.OracleRobot(robot)
        v, f, m = orc.check_edges(rob, prims, a, b, 32.0, early_exit=False, want_m=True)
        mism = (got != v) & (f == 0)
        near = (f == 0) & (np.abs(m) < 1e-4)
        say("  %s: %d edges, %d within 1e-5..1e-4 m (unflagged, all equal: %s), %d flagged, %d of them agree"
            % (name, len(v), near.sum(), not mism.any(), f.sum(), np.sum((got == v) & (f == 1))))
        assert near.sum() >= 8 * 12 and f.sum() >= 4 * 12
        assert not mism.any(), (name, np.nonzero(mism)[0][:10], m[mism][:10])


def test_check_edges_edge_cases(gpu, orc, r7):
    P, ctx, torch = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    prims = W.scene_s12(r7, 2)
    sid = P.prrtc_load_scene(ctx, prims)
    rng = np.random.default_rng(5)
    say("edge cases")
    # n = 0 is a no-op
    P.prrtc_check_edges(ctx, rid, sid, 0, 0, 0, 32.0, 0, None)
    # zero-length edges, one edge, and long edges spanning many FK tiles
    a = rng.uniform(-2.8, 2.8, (300, 7)).astype(np.float32)
    b = a.copy()
    b[100:] = rng.uniform(-2.8, 2.8, (200, 7)).astype(np.float32)  # long: up to ~14 rad -> ~450 points
    got = gpu_check(gpu, rid, sid, a, b)
    assert_parity(orc, r7, prims, a, b, got)
    got1 = gpu_check(gpu, rid, sid, a[150:151], b[150:151])
    assert got1[0] == got[150]
    # coarse and fine resolutions
    for res in (0.5, 3.0, 200.0):
        got = gpu_check(gpu, rid, sid, a[100:160], b[100:160], res)
        assert_parity(orc, r7, prims, a[100:160], b[100:160], got, res)
    # empty scene: everything valid; enclosing sphere: nothing valid
    sid_e = P.prrtc_load_scene(ctx, np.zeros(0, W.PRIM_DTYPE))
    assert gpu_check(gpu, rid, sid_e, a, b).all()
    big = W.make_prims([(W.PRIM_SPHERE, (0, 0, 0.5), np.eye(3), (5.0, 0, 0))])
    assert not gpu_check(gpu, rid, P.prrtc_load_scene(ctx, big), a, b).any()
    # an obstacle touching only the fixed base spheres invalidates every edge
    base_hit = W.make_prims([(W.PRIM_CUBOID, (0.0, 0.0, 0.1), np.eye(3), (0.02, 0.02, 0.02))])
    got = gpu_check(gpu, rid, P.prrtc_load_scene(ctx, base_hit), a, b)
    assert_parity(orc, r7, base_hit, a, b, got)
    assert not got.any()


def test_check_edges_deterministic_and_stream_order(gpu, r7):
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    sid = P.prrtc_load_scene(ctx, W.scene_s64(r7))
    a, b = W.random_edges(r7, 50000, seed=99)
    say("determinism")
    g1 = gpu_check(gpu, rid, sid, a, b)
    g2 = gpu_check(gpu, rid, sid, a, b)
    assert np.array_equal(g1, g2)


def test_check_edges_argument_errors(gpu, r7):
    P, ctx, torch = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    sid = P.prrtc_load_scene(ctx, W.scene_s12(r7, 0))
    t = torch.zeros((4, 7), device="cuda")
    v = torch.zeros(4, dtype=torch.uint8, device="cuda")
    for args, code in (((rid + 100, sid, 32.0, 4), P.PRRTC_E_STATE),
                       ((rid, sid + 100, 32.0, 4), P.PRRTC_E_STATE),
                       ((rid, sid, 0.0, 4), P.PRRTC_E_ARG),
                       ((rid, sid, float("nan"), 4), P.PRRTC_E_ARG),
                       ((rid, sid, 32.0, -1), P.PRRTC_E_ARG)):
        r_, s_, res, n = args
        st = P.lib.prrtc_check_edges(ctx, r_, s_, t.data_ptr(), t.data_ptr(), n, res, v.data_ptr(), None)
        assert st == code
        assert P.prrtc_last_error(ctx)


def test_check_edges_full_size_configuration(gpu, orc, r7):
    """The benchmarked configuration: 64 obstacles, 2^20 edges, the same
    launch as the benchmark.  Every edge is compared with the oracle (OpenMP)."""
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    prims = W.scene_s64(r7)
    sid = P.prrtc_load_scene(ctx, prims)
    a, b = W.random_edges(r7, 1 << 20)
    say("full-size parity 2^20 edges")
    got = gpu_check(gpu, rid, sid, a, b)
    v, f = assert_parity(orc, r7, prims, a, b, got, threads=16)
    say("  valid frac %.4f flagged %d" % (v.mean(), f.sum()))


ESDF_O, ESDF_H, ESDF_N = (-1.3, -1.3, -1.3), 2.6 / 63, (64, 64, 64)


def test_esdf_builder_parity(gpu, orc, r7, r14):
    """The library's grid of a scene's primitives against the oracle's node
    values (FP32 against FP64 signed distances)."""
    P, ctx, torch = gpu
    for name, prims in (("S12", W.scene_s12(r7, 0)), ("S64", W.scene_s64(r7)), ("shelf", W.scene_shelf(r14))):
        sid = P.prrtc_load_scene(ctx, prims)
        out = torch.empty(ESDF_N[::-1], dtype=torch.float32, device="cuda")
        P.prrtc_esdf_from_scene(ctx, sid, ESDF_O, ESDF_H, ESDF_N, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        want = orc.esdf_of_scene(prims, ESDF_O, ESDF_H, ESDF_N)
        err = np.abs(out.cpu().numpy().astype(np.float64) - want)
        say("ESDF builder %s: max |err| %.3g m" % (name, err.max()))
        assert err.max() <= 2e-6


@pytest.mark.parametrize("with_prims", [False, True])
def test_check_edges_esdf_parity(gpu, orc, r7, with_prims):
    """Edges against an ESDF grid (the oracle's grid of the 64-obstacle scene,
    uploaded to the GPU): verdicts equal the oracle's trilinear clearances
    except within the flag band.  With the 12-obstacle scene's primitives
    in the same scene, both count."""
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    grid = orc.EsdfGrid(ESDF_O, ESDF_H, orc.esdf_of_scene(W.scene_s64(r7), ESDF_O, ESDF_H, ESDF_N))
    prims = W.scene_s12(r7, 2) if with_prims else np.zeros(0, W.PRIM_DTYPE)
    sid = P.prrtc_load_scene(ctx, prims)
    P.prrtc_scene_set_esdf(ctx, sid, ESDF_O, ESDF_H, grid.values)
    a, b = W.random_edges(r7, 20011, seed=99)
    got = gpu_check(gpu, rid, sid, a, b)
    with grid:
        v, f = assert_parity(orc, r7, prims, a, b, got)
    say("ESDF parity (prims %s): valid frac %.4f flagged %d" % (with_prims, v.mean(), f.sum()))
    assert 0.01 < v.mean() < 0.99
    # detached, only the primitives remain
    P.prrtc_scene_set_esdf(ctx, sid, None)
    got0 = gpu_check(gpu, rid, sid, a, b)
    assert_parity(orc, r7, prims, a, b, got0)


def test_check_edges_esdf_near_contact(gpu, orc, r7):
    """Edges ending 1e-6 .. 1e-3 m from the ESDF's zero level: unflagged
    verdicts match the oracle's."""
    import near_contact as NC
    P, ctx, _ = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    grid = orc.EsdfGrid(ESDF_O, ESDF_H, orc.esdf_of_scene(W.scene_s64(r7), ESDF_O, ESDF_H, ESDF_N))
    empty = np.zeros(0, W.PRIM_DTYPE)
    sid = P.prrtc_load_scene(ctx, empty)
    P.prrtc_scene_set_esdf(ctx, sid, ESDF_O, ESDF_H, grid.values)
    with grid:
        cf = NC.graze_configs(orc, r7, empty, 12, seed=0x4E44)
        a, b = NC.graze_edges(cf)
        got = gpu_check(gpu, rid, sid, a, b)
        v, f, m = orc.check_edges(orc.OracleRobot(r7), empty, a, b, 32.0, early_exit=False, want_m=True)
    mism = (got != v) & (f == 0)
    near = (f == 0) & (np.abs(m) < 1e-4)
    say("ESDF near contact: %d edges, %d within 1e-5..1e-4 m, %d flagged (%d agree)"
        % (len(v), near.sum(), f.sum(), np.sum((got == v) & (f == 1))))
    assert near.sum() >= 8 * 12 and not mism.any()


def test_esdf_argument_errors(gpu, r7):
    P, ctx, _ = gpu
    sid = P.prrtc_load_scene(ctx, np.zeros(0, W.PRIM_DTYPE))
    for origin, voxel, vals in (((0, 0, 0), 0.0, np.zeros((2, 2, 2))), ((0, 0, 0), 0.1, np.zeros((1, 2, 2))),
                                ((0, 0, float("nan")), 0.1, np.zeros((2, 2, 2))),
                                ((0, 0, 0), 0.1, np.full((2, 2, 2), np.nan))):
        with pytest.raises(P.PrrtcError) as e:
            P.prrtc_scene_set_esdf(ctx, sid, origin, voxel, vals)
        assert e.value.status == P.PRRTC_E_ARG
    with pytest.raises(P.PrrtcError) as e:
        P.prrtc_scene_set_esdf(ctx, 10_000, (0, 0, 0), 0.1, np.zeros((2, 2, 2)))
    assert e.value.status == P.PRRTC_E_STATE


@pytest.mark.parametrize("case", ["r7-s64", "r7-s12", "r14-shelf", "r14-esdf"])
def test_check_edges_two_stage(gpu, orc, r7, r14, case):
    """A robot with coarse spheres (two-stage checks) gives the one-stage
    robot's verdicts on every edge, flagged ones included (the coarse gate
    only skips fine tests that cannot hit), and so the oracle's."""
    P, ctx, _ = gpu
    name, scene = case.split("-")
    robot = r7 if name == "r7" else r14
    two = W.with_coarse_spheres(robot)
    prims = {"s64": lambda: W.scene_s64(robot), "s12": lambda: W.scene_s12(robot, 3),
             "shelf": lambda: W.scene_shelf(robot), "esdf": lambda: np.zeros(0, W.PRIM_DTYPE)}[scene]()
    rid1, rid2 = P.prrtc_load_robot(ctx, robot), P.prrtc_load_robot(ctx, two)
    sid = P.prrtc_load_scene(ctx, prims)
    grid = None
    if scene == "esdf":
        grid = orc.EsdfGrid(ESDF_O, ESDF_H, orc.esdf_of_scene(W.scene_shelf(robot), ESDF_O, ESDF_H, ESDF_N))
        P.prrtc_scene_set_esdf(ctx, sid, ESDF_O, ESDF_H, grid.values)
    a, b = W.random_edges(robot, 1 << 16 if scene == "s64" else 12011, seed=2024)
    for sched in (0, 1):
        P.prrtc_edge_schedule(ctx, rid1, sid, sched)
        P.prrtc_edge_schedule(ctx, rid2, sid, sched + 2)   # the same layout with the two-stage pass
        one = gpu_check(gpu, rid1, sid, a, b)
        got = gpu_check(gpu, rid2, sid, a, b)
        assert np.array_equal(got, one), (sched, np.nonzero(got != one)[0][:10])
    # the coarse robot's one-stage schedules ignore its coarse spheres
    P.prrtc_edge_schedule(ctx, rid2, sid, 1)
    assert np.array_equal(gpu_check(gpu, rid2, sid, a, b), one)
    # timing on a large batch picks among all four schedules
    if len(a) >= 8192:
        P.prrtc_edge_schedule(ctx, rid2, sid, -1)
        assert np.array_equal(gpu_check(gpu, rid2, sid, a, b), one)
        assert P.prrtc_edge_schedule(ctx, rid2, sid) in (0, 1, 2, 3)
    with pytest.raises(P.PrrtcError):
        P.prrtc_edge_schedule(ctx, rid2, sid, 4)
    if grid is not None:
        with grid:
            v, f = assert_parity(orc, robot, prims, a, b, got, threads=16)
    else:
        v, f = assert_parity(orc, robot, prims, a, b, got, threads=16)
    say("two-stage %s: %d edges, valid frac %.4f, flagged %d" % (case, len(a), v.mean(), f.sum()))


def test_two_stage_descriptor_checked(gpu, r7):
    """Coarse spheres that do not enclose their fine spheres are refused."""
    P, ctx, _ = gpu
    bad = W.with_coarse_spheres(r7)
    bad["coarse_xyzr"] = bad["coarse_xyzr"].copy()
    bad["coarse_xyzr"][2, 3] *= 0.5
    with pytest.raises(P.PrrtcError) as e:
        P.prrtc_load_robot(ctx, bad)
    assert e.value.status == P.PRRTC_E_ARG


def test_check_edges_in_hip_graph(gpu, orc, r7):
    """check_edges launches captured in a HIP graph (after the schedule is
    chosen, so the call does not synchronise): every replay gives the eager
    verdicts, with eager work and synchronisation between the replays."""
    P, ctx, torch = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    prims = W.scene_s64(r7)
    sid = P.prrtc_load_scene(ctx, prims)
    P.prrtc_edge_schedule(ctx, rid, sid, 1)
    batches = [W.random_edges(r7, n, seed=600 + k) for k, n in enumerate((4096, 777, 20011))]
    dev = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), torch.zeros(a.shape[0], dtype=torch.uint8,
                                                                             device="cuda")) for a, b in batches]
    eager = [gpu_check(gpu, rid, sid, a, b) for a, b in batches]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for ta, tb, tv in dev:
            tv.zero_()
            P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), ta.shape[0], 32.0, tv.data_ptr(),
                                s.cuda_stream)
    for rep in range(4):
        for _, _, tv in dev:
            tv.fill_(7)                                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, tv), want in zip(dev, eager):
            assert np.array_equal(tv.cpu().numpy(), want), rep
    say("graph replays equal the eager verdicts")


def test_check_edges_stream_order(gpu, r7):
    """Stream arguments: torch's default stream (handle 0, passed on as
    hipStreamLegacy) orders the call with torch's own work on that stream, so
    a copy issued after it sees the verdicts and events recorded around it
    bracket the kernel; NULL (None) runs on the context's stream, which a
    device synchronisation waits for.  Both give the same verdicts."""
    P, ctx, torch = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    sid = P.prrtc_load_scene(ctx, W.scene_s64(r7))
    P.prrtc_edge_schedule(ctx, rid, sid, 1)
    n = 1 << 18
    a, b = W.random_edges(r7, n, seed=611)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    want = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n, 32.0, want.data_ptr(), None)
    torch.cuda.synchronize()
    want = want.cpu().numpy()
    assert set(np.unique(want)) <= {0, 1}
    cur = torch.cuda.current_stream()
    assert cur.cuda_stream == 0
    for rep in range(3):
        tv = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n, 32.0, tv.data_ptr(), cur.cuda_stream)
        e1.record(cur)
        got = tv.cpu().numpy()                 # a copy on the same stream, no synchronisation first
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        say("  default-stream launch %d: %.3f ms" % (rep, ms))
        assert np.array_equal(got, want), rep
        assert ms > 0.02                       # the kernel ran between the events


@pytest.mark.gpu
def test_check_edges_static_and_dynamic_handout_agree(gpu, orc, r7):
    """A batch of up to 48 edges per resident wave is interleaved statically
    over the waves, a larger one handed out in chunks from per-XCD counters.
    The same 2^19 edges as one batch (dynamic on a 256-CU device) and as
    eight batches of 2^16 (static) give the same verdicts, and a sample of
    them equals the oracle's."""
    P, ctx, torch = gpu
    rid = P.prrtc_load_robot(ctx, r7)
    prims = W.scene_s64(r7)
    sid = P.prrtc_load_scene(ctx, prims)
    P.prrtc_edge_schedule(ctx, rid, sid, 1)
    n, part = 1 << 19, 1 << 16
    a, b = W.random_edges(r7, n, seed=733)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    whole = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n, 32.0, whole.data_ptr(), None)
    parts = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    for k in range(0, n, part):
        P.prrtc_check_edges(ctx, rid, sid, ta[k:].data_ptr(), tb[k:].data_ptr(), part, 32.0,
                            parts[k:].data_ptr(), None)
    torch.cuda.synchronize()
    whole, parts = whole.cpu().numpy(), parts.cpu().numpy()
    say("  static vs dynamic hand-out: %d valid of %d" % (int(whole.sum()), n))
    assert set(np.unique(whole)) <= {0, 1}
    assert np.array_equal(whole, parts)
    idx = np.random.default_rng(9).choice(n, 3000, replace=False)
    want, flag, _ = orc.check_edges(orc.OracleRobot(r7), prims, a[idx], b[idx], 32.0, early_exit=True)
    ok = flag == 0
    assert np.array_equal(whole[idx][ok], want[ok].astype(np.uint8))
