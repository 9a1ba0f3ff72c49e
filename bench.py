#!/usr/bin/env python3
"""Benchmark of the pRRTC hot path on one MI355X.

Timed step: one prrtc_check_edges launch over the 2^20-edge batch of the
7-DoF arm among 64 obstacles (inputs resident in HBM), the workload the
edge-checks/s figure is quoted on.  Also reported, each timed on its own:
  - roofline of the collision kernel (HIP events around every timed launch),
  - ms-to-solution of prrtc_plan on the 7-DoF / 12-obstacle queries,
  - the serial oracle on the host (cpu_baseline).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2503_06757_amd import workloads as W  # noqa: E402

METRIC = "p50 ms-to-solution + edge checks/s (7/14-DoF), learned vs plain sampler"
N_EDGES = 1 << 20
RES = 32.0
SEED_VARIANT_EDGES = 0x45000001   # edges of the collision-model variants
PEAK_FP32_TFLOPS = 157.3          # MI355X published FP32 vector peak

# Algorithmic FP32 work per checked configuration, the dense per-point model
# (FMA = 2, add/sub/mul = 1, compare/min/max = 0): every robot sphere against
# every obstacle (sphere 10, cuboid 28, cylinder 27) and every self pair (10),
# plus FK: 67 per joint frame composition, 18 per sphere transform, 2 per
# joint of interpolation (sin/cos not counted).  7-DoF arm (60 spheres) among
# 32 spheres, 21 cuboids and 11 cylinders: 73,863 FLOP per configuration.
MODEL_SPHERE, MODEL_CUBOID, MODEL_CYLINDER, MODEL_PAIR = 10, 28, 27, 10
MODEL_JOINT, MODEL_SPHERE_XFORM, MODEL_INTERP = 67, 18, 2


def point_flops_model(robot, prims):
    t = np.bincount(prims["type"], minlength=3)
    n_sph = robot["sphere_xyzr"].shape[0]
    dof = sum(robot["chain_dof"])
    per_sphere = MODEL_SPHERE * t[0] + MODEL_CUBOID * t[1] + MODEL_CYLINDER * t[2]
    return int(n_sph * per_sphere + MODEL_PAIR * len(robot["self_pairs"]) +
               dof * (MODEL_JOINT + MODEL_INTERP) + n_sph * MODEL_SPHERE_XFORM)


# A reduced count of the same work, as this kernel organises it: base-frame
# spheres never move, so they are tested once per launch, not per
# configuration; cuboid 27 and cylinder 26 (box-frame coordinates from three
# FMAs each), frame update 48.
FLOP_SPHERE, FLOP_CUBOID, FLOP_CYLINDER = 10, 27, 26
FLOP_JOINT = 48
FLOP_SPHERE_XFORM = 18
FLOP_INTERP = 2


def point_flops(robot, prims):
    """Reduced count per configuration: FK of the moving spheres and every
    moving-sphere x obstacle test."""
    bases = set()
    f = 0
    for d in robot["chain_dof"]:
        bases.add(f)
        f += d + 1
    moving = int(np.sum([fr not in bases for fr in robot["sphere_frame"]]))
    t = np.bincount(prims["type"], minlength=3)
    per_sphere = FLOP_SPHERE * t[0] + FLOP_CUBOID * t[1] + FLOP_CYLINDER * t[2]
    dof = sum(robot["chain_dof"])
    return dof * (FLOP_JOINT + FLOP_INTERP) + moving * (FLOP_SPHERE_XFORM + per_sphere)


def kernel_source_hash():
    """Hash of the source text that decides what k_check_edges executes: the
    shared device header, the device part of prrtc.hip, the robot and scene
    table layouts and the launch configuration (planner, proposal and other
    host code are excluded)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2503_06757_amd", "csrc")
    with open(os.path.join(csrc, "prrtc_device.h"), "rb") as fh:
        h.update(fh.read())
    with open(os.path.join(csrc, "prrtc.hip")) as fh:
        text = fh.read()
    h.update(text[:text.index("// Host side")].encode())
    a = text.index("prrtc_status prrtc_load_robot(")
    h.update(text[a:text.index("prrtc_status prrtc_fk_spheres(", a)].encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


EDGE_SCHEDULES = {0: "k_check_edges<16, 3, false, false>: 3 items per lane, spheres swept first",
                  1: "k_check_edges<16, 2, true, false>: 2 items per lane, cuboids swept first"}


def edge_counts(a, b, res):
    """Points per edge for the FLOP model (FP32, as the kernel decides it)."""
    d = (b - a).astype(np.float32)
    s = np.zeros(a.shape[0], np.float32)
    for j in range(a.shape[1]):
        s = s + d[:, j] * d[:, j]
    n = np.ceil(np.float32(res) * np.sqrt(s)).astype(np.int64)
    return np.maximum(n, 1)


def bench_check_edges(P, ctx, torch, steps, warmup, schedule_pin=-1):
    robot = W.robot_r7()
    prims = W.scene_s64(robot)
    rid = P.prrtc_load_robot(ctx, robot)
    sid = P.prrtc_load_scene(ctx, prims)
    if schedule_pin >= 0:
        P.prrtc_edge_schedule(ctx, rid, sid, schedule_pin)   # a profiler run times every launch the same way
    a, b = W.random_edges(robot, N_EDGES)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    tv = torch.empty(N_EDGES, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), N_EDGES, RES, tv.data_ptr(),
                            stream.cuda_stream)

    for _ in range(warmup):
        step()          # the first call also times the two kernel schedules on this pair
    torch.cuda.synchronize()
    schedule = P.prrtc_edge_schedule(ctx, rid, sid)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs]))
    valid = tv.cpu().numpy().astype(bool)
    n_pts = edge_counts(a, b, RES) + 1
    fl_model = point_flops_model(robot, prims)
    fl_point = int(point_flops(robot, prims))
    # Lower bound of the work any correct checker must do: every configuration
    # of every collision-free edge in full; colliding edges counted as zero.
    free_points = float(np.sum(n_pts[valid]))
    # The collision-free edges alone as their own launch (inputs resident):
    # every configuration of every edge must be checked, so early exit cannot help.
    fa, fb = ta[torch.from_numpy(valid).cuda()].contiguous(), tb[torch.from_numpy(valid).cuda()].contiguous()
    nf = int(fa.shape[0])
    tvf = torch.empty(max(nf, 1), dtype=torch.uint8, device="cuda")

    def step_free():
        P.prrtc_check_edges(ctx, rid, sid, fa.data_ptr(), fb.data_ptr(), nf, RES, tvf.data_ptr(), stream.cuda_stream)

    for _ in range(warmup):
        step_free()
    evf = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in evf:
        e0.record(stream)
        step_free()
        e1.record(stream)
    torch.cuda.synchronize()
    free_ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evf]))
    free_ok = bool(tvf[:nf].all().item())
    return dict(robot=robot, prims=prims, a=a, b=b, wall_s=t1 - t0, kernel_ms=kernel_ms, schedule=schedule,
                valid=valid, valid_frac=float(valid.mean()), free_points=free_points,
                flop_per_point_model=fl_model, flop_per_point=fl_point, mean_points=float(n_pts.mean()),
                free_edges=nf, free_ms=free_ms, free_all_valid=free_ok)


def time_edges(P, ctx, torch, rid, sid, a, b, reps=10, warmup=2):
    """Mean kernel time (HIP events on the launch stream) of prrtc_check_edges
    over a resident batch, and its verdicts."""
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    n = a.shape[0]
    tv = torch.empty(n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n, RES, tv.data_ptr(), stream.cuda_stream)

    for _ in range(warmup):
        step()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs])), tv.cpu().numpy().astype(bool)


def bench_collision_variants(P, ctx, torch):
    """check_edges throughput of the other collision models on their own
    batches: two-stage checks (coarse spheres gating fine ones, Sec. III-A)
    against one stage on the 7-DoF arm among 64 and among 12 obstacles and
    the dual arm in the shelf (the two-stage pass pinned, and the schedule
    the library's timing picks among one- and two-stage for the coarse
    robot), and the 7-DoF arm against an ESDF grid of the 64 obstacles (64^3
    nodes over [-1.3, 1.3]^3, built by the library) instead of the
    primitives.  Verdicts of the two-stage robot must equal the one-stage
    robot's."""
    out = {}
    r7, r14 = W.robot_r7(), W.robot_r14()
    for name, robot, prims, n in (("r7_s64", r7, W.scene_s64(r7), N_EDGES),
                                  ("r7_s12", r7, W.scene_s12(r7, 3), N_EDGES),
                                  ("r14_shelf", r14, W.scene_shelf(r14), N_EDGES // 4)):
        sid = P.prrtc_load_scene(ctx, prims)
        a, b = W.random_edges(robot, n, seed=SEED_VARIANT_EDGES)
        rows = {}
        rid1 = P.prrtc_load_robot(ctx, robot)
        ms, v1 = time_edges(P, ctx, torch, rid1, sid, a, b)
        rows["one_stage"] = {"edges": n, "kernel_ms": ms, "edge_checks_per_s": n / (ms * 1e-3),
                             "schedule": P.prrtc_edge_schedule(ctx, rid1, sid), "valid_fraction": float(v1.mean())}
        rid2 = P.prrtc_load_robot(ctx, W.with_coarse_spheres(robot))
        best, equal = None, True
        for sched in (2, 3):                      # the two-stage pass, both item layouts
            P.prrtc_edge_schedule(ctx, rid2, sid, sched)
            ms, v2 = time_edges(P, ctx, torch, rid2, sid, a, b)
            equal &= bool(np.array_equal(v1, v2))
            if best is None or ms < best[0]:
                best = (ms, sched)
        rows["two_stage"] = {"edges": n, "kernel_ms": best[0], "edge_checks_per_s": n / (best[0] * 1e-3),
                             "schedule": best[1]}
        P.prrtc_edge_schedule(ctx, rid2, sid, -1)  # the timed choice among all four
        ms, v2 = time_edges(P, ctx, torch, rid2, sid, a, b)
        equal &= bool(np.array_equal(v1, v2))
        rows["coarse_robot_tuned"] = {"kernel_ms": ms, "schedule": P.prrtc_edge_schedule(ctx, rid2, sid)}
        rows["verdicts_equal"] = equal
        rows["speedup"] = rows["one_stage"]["kernel_ms"] / rows["two_stage"]["kernel_ms"]
        out[name] = rows
    o, h, dims = (-1.3, -1.3, -1.3), 2.6 / 63, (64, 64, 64)
    src = P.prrtc_load_scene(ctx, W.scene_s64(r7))
    grid = torch.empty((64, 64, 64), dtype=torch.float32, device="cuda")
    P.prrtc_esdf_from_scene(ctx, src, o, h, dims, grid.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    sid = P.prrtc_load_scene(ctx, np.zeros(0, W.PRIM_DTYPE))
    P.prrtc_scene_set_esdf(ctx, sid, o, h, grid.cpu().numpy())
    a, b = W.random_edges(r7, N_EDGES, seed=SEED_VARIANT_EDGES)
    rid = P.prrtc_load_robot(ctx, r7)
    ms, v = time_edges(P, ctx, torch, rid, sid, a, b)
    out["r7_esdf_s64"] = {"edges": N_EDGES, "kernel_ms": ms, "edge_checks_per_s": N_EDGES / (ms * 1e-3),
                          "valid_fraction": float(v.mean()), "grid": "64^3 nodes, voxel %.4f m" % h}
    return out


def bench_graph_launches(P, ctx, torch, n_edges=4096, launches=200):
    """Small check_edges batches back to back: launched one call at a time,
    and the same calls captured once in a HIP graph and replayed (what a
    caller gains from graphs where batches are small and launches dominate)."""
    r7 = W.robot_r7()
    rid, sid = P.prrtc_load_robot(ctx, r7), P.prrtc_load_scene(ctx, W.scene_s64(r7))
    P.prrtc_edge_schedule(ctx, rid, sid, 1)
    a, b = W.random_edges(r7, n_edges, seed=SEED_VARIANT_EDGES + 1)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    tv = torch.empty(n_edges, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()

    def calls():
        for _ in range(launches):
            P.prrtc_check_edges(ctx, rid, sid, ta.data_ptr(), tb.data_ptr(), n_edges, RES, tv.data_ptr(), s.cuda_stream)

    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        calls()
    torch.cuda.synchronize()
    eager = time.perf_counter() - t0
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        calls()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.replay()
    torch.cuda.synchronize()
    graph = time.perf_counter() - t0
    # what one planner launch costs beyond its work: a query whose start and
    # goal connect in the first round of an empty scene, as a single plan and
    # as a one-query batch (host calls, argument upload, the launch, result
    # copy); a batch of a thousand queries pays this once
    sid0 = P.prrtc_load_scene(ctx, np.zeros(0, W.PRIM_DTYPE))
    q0 = np.zeros(7, np.float32)
    q1 = np.full(7, 0.05, np.float32)
    prm = P.prrtc_plan_params_default()
    prm.workers = 64
    ts, tb_, ok = [], [], 0
    for rep in range(60):
        t0 = time.perf_counter()
        st, _, _ = P.prrtc_plan(ctx, rid, sid0, q0, q1, prm)
        ts.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        P.prrtc_plan_batch(ctx, [(rid, sid0, q0, q1, 1, 0)], prm)
        tb_.append(time.perf_counter() - t0)
        ok += st == P.PRRTC_OK
    return {"edges_per_launch": n_edges, "launches": launches, "eager_us_per_launch": eager / launches * 1e6,
            "graph_us_per_launch": graph / launches * 1e6,
            "trivial_plan_ms": float(np.median(ts[10:]) * 1e3), "trivial_plan_batch_ms": float(np.median(tb_[10:]) * 1e3),
            "trivial_plans_solved": int(ok)}


def bench_plan(P, ctx, n_instances=100, n_seeds=50):
    """ms-to-solution on the 7-DoF arm among 12 obstacles: one query per
    scene instance, plus scene 0 under n_seeds planner seeds."""
    robot = W.robot_r7()
    rid = P.prrtc_load_robot(ctx, robot)
    prm = P.prrtc_plan_params_default()
    prm.max_rounds, prm.time_budget_ms = 1 << 30, 1000.0
    times, rounds, costs, fails = [], [], [], 0
    jobs = [(k, k) for k in range(n_instances)] + [(0, 1000 + s) for s in range(n_seeds)]
    scene_ids, queries = {}, {}
    for inst, seed in jobs:
        if inst not in scene_ids:
            scene_ids[inst] = P.prrtc_load_scene(ctx, W.scene_s12(robot, inst))
        prm.seed = seed
        cands = queries.get(inst) or W.query_candidates(robot, W.SEED_QUERY + inst, 200)
        while True:
            s, g = cands[0]
            t0 = time.perf_counter()
            st, path, stats = P.prrtc_plan(ctx, rid, scene_ids[inst], s, g, prm)
            dt = (time.perf_counter() - t0) * 1e3
            if st == P.PRRTC_E_INVALID_ENDPOINT:
                cands = cands[1:]
                continue
            break
        queries[inst] = cands
        if st == P.PRRTC_OK:
            times.append(dt)
            rounds.append(stats["rounds"])
            costs.append(float(np.sum(np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1))))
        else:
            fails += 1
            times.append(float("inf"))
    t = np.array(times)

    def pct(q):
        # failures count as infinitely slow; a percentile they reach is reported as null
        with np.errstate(invalid="ignore"):   # interpolating between two failures
            v = float(np.percentile(t, q))
        return v if np.isfinite(v) else None

    ok = t[np.isfinite(t)]
    return {"workload": "plan_r7_s12", "queries": len(jobs), "success": float(np.mean(np.isfinite(t))),
            "p50_ms": pct(50), "p95_ms": pct(95), "p99_ms": pct(99),
            "max_solved_ms": float(ok.max()) if ok.size else None, "mean_rounds": float(np.mean(rounds)) if rounds else None,
            "mean_cost": float(np.mean(costs)) if costs else None, "workers": prm.workers,
            "time_budget_ms": prm.time_budget_ms}


def query_pool(P, ctx, torch, n_scenes=64, per_scene=4, seed=0x56000000, max_rounds=3000):
    """Served workload pool: scenes with U{8..128} obstacles (6:4:2 mix) for
    the 7-DoF arm and the dual arm alternately, up to `per_scene` free
    queries each (endpoints checked by prrtc_check_edges), kept when the
    uniform planner (256 workers, its seed) solves them within max_rounds
    rounds (many generated queries in dense scenes have no solution; serving
    them measures only the budget).  A round budget, not a time budget,
    keeps the pool the same for every build of the planner."""
    from paper_2503_06757_amd import proposal as PR
    robots = [W.robot_r7(), W.robot_r14()]
    rids = [P.prrtc_load_robot(ctx, r) for r in robots]
    prm = P.prrtc_plan_params_default()
    prm.max_rounds, prm.time_budget_ms = max_rounds, 0.0
    pool, tried = [], 0
    for i in range(n_scenes):
        kind = i % 2
        rng = np.random.default_rng(seed + i)
        prims = W.scene_mixed(seed + i, robots[kind], int(rng.integers(8, 129)))
        sid = P.prrtc_load_scene(ctx, prims)
        for j in range(per_scene):
            q = PR.free_query(P, ctx, torch, rids[kind], sid, robots[kind], seed + 1000 * j + i)
            if q is None:
                continue
            tried += 1
            prm.seed = seed + 1000 * j + i
            st, _, _ = P.prrtc_plan(ctx, rids[kind], sid, q[0], q[1], prm)
            if st == P.PRRTC_OK:
                pool.append((rids[kind], sid, q[0], q[1], kind))
    return pool, tried


SERVE_HEADROOM = 1.05  # tuned batch rate over the arrival rate a served launch shape must keep


def served_shape(rates, rate, fastest):
    """Launch shape for serving at `rate` queries/s from the tuner's
    {(workers, tile): queries/s}: a query's latency falls with its worker
    count as long as the launch keeps up with the arrivals, so the most
    workers per query whose rate has SERVE_HEADROOM over the arrival rate
    (the faster tile among those), else the fastest shape."""
    fits = [(w, v, t) for (w, t), v in rates.items() if v >= SERVE_HEADROOM * rate]
    if not fits:
        return fastest
    w, _, t = max(fits)
    return w, t


def bench_serve(P, ctx, torch, pool, n_queries=10000, rate=2000.0, workers=None, slots=256, max_pending=1024,
                budget=2 << 30, max_rounds=4000, budget_ms=100.0, seed=0x56000000, log=None, models=None, tile=16,
                arrivals=None):
    """The served workload through the library's serving thread: queries
    arrive as a Poisson stream (exponential gaps) and are submitted at their
    arrival time (refused submissions are retried: admission); the thread
    keeps one persistent launch that takes each query as it is published.
    models: None (uniform sampling) or (7-DoF model, 14-DoF model): learned
    sampling, each query with its robot's model (the group computes the
    mixture in the launch).  Latency = completion seen by polling - arrival,
    on the host clock."""
    pool, tried = pool
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_queries)
    if arrivals is None:
        arrivals = np.cumsum(gaps)
    n_queries = len(arrivals)
    picks = rng.integers(0, len(pool), n_queries)
    prm = P.prrtc_plan_params_default()
    prm.max_rounds, prm.time_budget_ms = max_rounds, budget_ms
    if models is not None:
        prm.sampler, prm.model_id, prm.mix = 1, models[0], 0.5
    tune = None
    if workers is not None:
        prm.tile = tile
    if workers is None:
        # launch shape from the autotuner on a sample of the pool
        sample = [(pool[k % len(pool)][0], pool[k % len(pool)][1], pool[k % len(pool)][2], pool[k % len(pool)][3],
                   seed + 777 + k, 0) for k in range(slots)]
        (best_w, best_t), rates = P.prrtc_tune_launch(ctx, sample, prm, memory_budget=budget)
        workers, tile = served_shape(rates, rate, (best_w, best_t))
        tune = {"workers": workers, "tile": tile, "fastest": {"workers": best_w, "tile": best_t},
                "headroom": SERVE_HEADROOM, "queries_per_s": {"%d/%d" % k: v for k, v in rates.items()}}
        if log:
            log("  launch shape: %d workers per query, tile %d (fastest batch shape %d/%d)" % (workers, tile, best_w,
                                                                                            best_t))
        prm.tile = tile
    prm.workers = workers
    done = np.full(n_queries, np.nan)
    status = np.zeros(n_queries, np.int32)
    refused = 0
    outstanding = {}
    nxt = 0
    P.prrtc_serve_start(ctx, prm, slots=slots, max_pending=max_pending, memory_budget=budget, path_cap=128)
    t0 = time.perf_counter()
    try:
        while nxt < n_queries or outstanding:
            now = time.perf_counter() - t0
            while nxt < n_queries and arrivals[nxt] <= now:
                rid, sid, s, g, kind = pool[picks[nxt]]
                t = P.prrtc_submit(ctx, rid, sid, s, g, seed + nxt, 0, -1 if models is None else models[kind])
                if t is None:
                    refused += 1
                    break
                outstanding[t] = (nxt, len(s))
                nxt += 1
            for t in list(outstanding):
                k, dof = outstanding[t]
                r = P.prrtc_poll(ctx, t, dof, 128)
                if r is not None:
                    done[k] = time.perf_counter() - t0
                    status[k] = r[0]
                    del outstanding[t]
    finally:
        launches = P.prrtc_serve_stop(ctx)
    lat = (done - arrivals) * 1e3
    ok = status == P.PRRTC_OK
    span = float(np.nanmax(done))
    return {"workload": "serve_mixed_r7_r14", "sampler": "uniform" if models is None else "learned",
            "queries": n_queries, "rate_per_s": rate, "workers": workers, "tile": int(prm.tile),
            "slots": slots, "max_pending": max_pending, "memory_budget_bytes": budget, "success": float(ok.mean()),
            "p50_latency_ms": float(np.percentile(lat, 50)), "p99_latency_ms": float(np.percentile(lat, 99)),
            "queries_per_s": n_queries / span, "launches": launches, "mean_batch": n_queries / max(launches, 1),
            "refused_submissions": refused, "pool": len(pool), "pool_tried": tried, "tuning": tune,
            "time_budget_ms": budget_ms, "_latency_ms": lat, "_ok": ok}


def bench_serve_burst(P, ctx, torch, pool, log=None):
    """A quiet stream then a burst through one server: 200 queries at 100/s
    (about 2 s; the mean gap of 10 ms is below the launch's 50 ms idle
    limit), a 0.2 s pause (the launch closes: no group has claimed a query
    for 50 ms), then 2000 queries submitted at once, which start a new launch
    with every group.  Reports each phase's latency, the burst's throughput
    and the number of launches."""
    rng = np.random.default_rng(0x56100000)
    quiet = np.cumsum(rng.exponential(1.0 / 100.0, 200))
    t_burst = float(quiet[-1]) + 0.2
    arrivals = np.concatenate([quiet, np.full(2000, t_burst)])
    r = bench_serve(P, ctx, torch, pool, workers=16, tile=16, arrivals=arrivals, log=log)
    lat, ok = r.pop("_latency_ms"), r.pop("_ok")
    q, b = slice(0, 200), slice(200, None)
    out = {"workload": "serve_mixed_r7_r14 quiet 100/s then a burst of 2000", "workers": 16, "tile": 16,
           "launches": r["launches"],
           "quiet": {"queries": 200, "success": float(ok[q].mean()), "p50_latency_ms": float(np.percentile(lat[q], 50)),
                     "p99_latency_ms": float(np.percentile(lat[q], 99))},
           "burst": {"queries": 2000, "success": float(ok[b].mean()), "p50_latency_ms": float(np.percentile(lat[b], 50)),
                     "p99_latency_ms": float(np.percentile(lat[b], 99)),
                     "queries_per_s": 2000.0 / (float(np.max(lat[b])) / 1e3)}}
    if log:
        log("  %s" % json.dumps(out))
    return out


def bench_throughput(P, ctx, torch, pool, n_queries=1024, workers=(16, 64, 256), max_rounds=4000,
                     budget_ms=100.0, log=None):
    """Queries/s of one prrtc_plan_batch launch over the served pool for each
    worker count (the planner's launch-shape tuning)."""
    pool, _ = pool
    rows = []
    for wk in workers:
        prm = P.prrtc_plan_params_default()
        prm.workers, prm.max_rounds, prm.time_budget_ms, prm.tile = wk, max_rounds, budget_ms, 16
        qs = [(pool[k % len(pool)][0], pool[k % len(pool)][1], pool[k % len(pool)][2], pool[k % len(pool)][3],
               7 + k, 0) for k in range(n_queries)]
        t0 = time.perf_counter()
        used, out = P.prrtc_plan_batch(ctx, qs, prm, groups=0, path_cap=128)
        dt = time.perf_counter() - t0
        ok = np.mean([o[0] == P.PRRTC_OK for o in out])
        rows.append({"workers": wk, "tile": 16, "groups": used, "queries_per_s": n_queries / dt,
                     "success": float(ok), "time_budget_ms": budget_ms})
        if log:
            log("  workers %d: %s" % (wk, rows[-1]))
    return rows


SHELF_QUERIES = os.path.join(ROOT, "tests", "golden", "shelf_queries_r14.txt")


SHELF_BUDGET_MS = 1000.0     # per query, fixed beforehand for both samplers
SHELF_MAX_ROUNDS = 1 << 30   # the time budget ends a query, not a round count


def pcts(t):
    """p50 / p90 / p99 of per-query times with failures as +inf (a percentile
    that a failure reaches is reported as null)."""
    out = {}
    for q in (50, 90, 99):
        with np.errstate(invalid="ignore"):   # interpolating between two failures
            v = float(np.percentile(t, q)) if len(t) else float("inf")
        out["p%d_ms" % q] = v if np.isfinite(v) else None
    return out


def bench_shelf(P, ctx, n_queries=500, max_rounds=SHELF_MAX_ROUNDS, budget_ms=SHELF_BUDGET_MS, workers=256):
    """ms-to-solution of the dual arm (14-DoF, 3600 inter-arm pairs) reaching
    into the 5x3 shelf with 24 random spheres: the stored generated queries
    (start in front of the shelf, each hand in a cell on its side)."""
    robot = W.robot_r14()
    rid = P.prrtc_load_robot(ctx, robot)
    sid = P.prrtc_load_scene(ctx, W.scene_shelf(robot))
    Q = np.loadtxt(SHELF_QUERIES, dtype=np.float32)[:n_queries]
    prm = P.prrtc_plan_params_default()
    prm.max_rounds, prm.time_budget_ms, prm.workers = max_rounds, budget_ms, workers
    rows = []
    for k, row in enumerate(Q):
        prm.seed = W.SEED_QUERY + k
        t0 = time.perf_counter()
        st, _, stats = P.prrtc_plan(ctx, rid, sid, row[:14], row[14:], prm)
        dt = (time.perf_counter() - t0) * 1e3
        rows.append((st == P.PRRTC_OK, dt, stats["rounds"], stats["edges_checked"], stats["gpu_ms"]))
    a = np.array(rows, np.float64)
    ok = a[:, 0] > 0
    t = np.where(ok, a[:, 1], np.inf)
    return {"workload": "plan_r14_shelf", "queries": len(a), "success": float(ok.mean()), **pcts(t),
            "mean_rounds": float(a[ok, 2].mean()) if ok.any() else None,
            "edge_checks_per_s": float(a[:, 3].sum() / (a[:, 4].sum() * 1e-3)),
            "max_rounds": max_rounds, "time_budget_ms": budget_ms, "workers": workers}


def bench_sampling(P, ctx, n_shelf=100, n_r7=100, budget_ms=SHELF_BUDGET_MS, dds=(1.0, 4)):
    """Sampling variants on the same queries, seeds and budgets: uniform
    Philox draws, dynamic-domain sampling (Sec. III: a node whose extension
    failed only accepts samples within dds_radius; redrawn up to dds_tries
    times) and Halton points (the sampler of the paper's experiments,
    Sec. IV-A), on the dual-arm shelf and the 7-DoF arm among 12 obstacles."""
    variants = {"uniform": dict(), "dynamic_domain": dict(dds_radius=dds[0], dds_tries=dds[1]),
                "halton": dict(sampler=2)}
    Q = np.loadtxt(SHELF_QUERIES, dtype=np.float32)[:n_shelf]
    r14, r7 = W.robot_r14(), W.robot_r7()
    rid14, rid7 = P.prrtc_load_robot(ctx, r14), P.prrtc_load_robot(ctx, r7)
    sid_shelf = P.prrtc_load_scene(ctx, W.scene_shelf(r14))
    r7_jobs = []
    for inst in range(n_r7):
        sid = P.prrtc_load_scene(ctx, W.scene_s12(r7, inst))
        for s, g in W.query_candidates(r7, W.SEED_QUERY + inst, 200):
            prm = P.prrtc_plan_params_default()
            prm.max_rounds = 0
            if P.prrtc_plan(ctx, rid7, sid, s, g, prm)[0] != P.PRRTC_E_INVALID_ENDPOINT:
                r7_jobs.append((sid, s, g, inst))
                break
    out = {"dds_radius": dds[0], "dds_tries": dds[1], "time_budget_ms": budget_ms}
    for name, kw in variants.items():
        legs = {}
        for leg, rid, jobs in (("r14_shelf", rid14, [(sid_shelf, row[:14], row[14:], k) for k, row in enumerate(Q)]),
                               ("r7_s12", rid7, r7_jobs)):
            rows = []
            for sid, s, g, k in jobs:
                prm = P.prrtc_plan_params_default()
                prm.seed, prm.max_rounds, prm.time_budget_ms = W.SEED_QUERY + k, SHELF_MAX_ROUNDS, budget_ms
                for key, v in kw.items():
                    setattr(prm, key, v)
                t0 = time.perf_counter()
                st, _, stats = P.prrtc_plan(ctx, rid, sid, s, g, prm)
                rows.append((st == P.PRRTC_OK, (time.perf_counter() - t0) * 1e3, stats["rounds"]))
            a = np.array(rows, np.float64)
            t = np.where(a[:, 0] > 0, a[:, 1], np.inf)
            legs[leg] = {"queries": len(a), "success": float(a[:, 0].mean()), **pcts(t),
                         "mean_rounds_solved": float(a[a[:, 0] > 0, 2].mean()) if a[:, 0].any() else None}
        out[name] = legs
    return out


def bench_learned(P, ctx, torch, n_train, n_eval, epochs, log):
    """The learned proposal end to end on the 7-DoF arm: data from the
    uniform planner on generated scenes, training (throughput against the
    BF16 matrix-core peak), held-out NLL, then uniform against learned
    sampling on held-out scenes (same seeds and budgets)."""
    from paper_2503_06757_amd import proposal as PR
    robot = W.robot_r7()
    rid = P.prrtc_load_robot(ctx, robot)
    t0 = time.perf_counter()
    ds = PR.generate(P, ctx, torch, rid, robot, n_train, log=log)
    gen_s = time.perf_counter() - t0
    ev = PR.generate(P, ctx, torch, rid, robot, n_eval, base=PR.SEED_EVAL)
    mid = P.prrtc_load_proposal(ctx, PR.pack(PR.init_params(7, 1), 7))
    nll0 = PR.mean_nll(P, ctx, torch, mid, rid, ev, robot["q_lo"], robot["q_hi"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = PR.train(P, ctx, torch, mid, rid, ds, epochs, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    n_samples = len(ds.scene_of)
    dof, hid, cw = 7, 256, 8 * 15
    fwd_sample = 2 * ((2 * dof + hid) * hid + 2 * hid * hid + hid * cw)
    fwd_scene = 2 * 4096 * hid
    flop = 3 * epochs * (n_samples * fwd_sample + ds.vox.shape[0] * fwd_scene)
    nll = PR.mean_nll(P, ctx, torch, mid, rid, ev, robot["q_lo"], robot["q_hi"])
    cmp = PR.compare(P, ctx, torch, mid, rid, robot, n_eval, log=log)
    return {"_model": mid, "workload": "learned_r7_mixed_scenes", "train_scenes": n_train,
            "solved_scenes": int(ds.vox.shape[0]),
            "samples": n_samples, "epochs": epochs, "datagen_s": gen_s, "train_s": train_s,
            "train_samples_per_s": epochs * n_samples / train_s,
            "train_tflops": flop / train_s / 1e12, "bf16_peak_tflops": 2500.0,
            "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1]),
            "heldout_nll_init": nll0, "heldout_nll": nll, "eval_scenes": n_eval,
            "free_queries": cmp["free_queries"], "solvable_queries": cmp["solvable_queries"],
            "time_budget_ms": cmp["time_budget_ms"], "screen_ms": cmp["screen_ms"],
            "plain": cmp["plain"], "learned": cmp["learned"]}


def bench_learned_shelf(P, ctx, torch, n_train, n_eval, epochs, log, budget_ms=SHELF_BUDGET_MS, tail=1.0):
    """The learned proposal on the dual arm: training queries made with the
    library's FK and checks, paths from the uniform planner (one batched
    launch), a 14-DoF model trained on them, then uniform against learned
    sampling on the stored shelf queries (same seeds, rounds and budget)."""
    from paper_2503_06757_amd import proposal as PR
    robot = W.robot_r14()
    rid = P.prrtc_load_robot(ctx, robot)
    sid = P.prrtc_load_scene(ctx, W.scene_shelf(robot))
    vox = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    P.prrtc_voxelize(ctx, sid, vox.data_ptr(), torch.cuda.current_stream().cuda_stream)
    vox_row = vox.cpu().numpy()
    t0 = time.perf_counter()
    starts, goals = PR.shelf_queries(P, ctx, torch, rid, sid, robot, n_train, seed=0x57000000, max_batches=4000,
                                     log=log)
    ds = PR.shelf_dataset(P, ctx, torch, rid, sid, starts, goals, vox_row, tail=tail)
    gen_s = time.perf_counter() - t0
    log("  shelf training data: %d of %d queries solved, %d samples, %.1f s" % (ds.vox.shape[0], n_train,
                                                                                 len(ds.scene_of), gen_s))
    mid = P.prrtc_load_proposal(ctx, PR.pack(PR.init_params(14, 2), 14))
    losses = PR.train(P, ctx, torch, mid, rid, ds, epochs, log=log)
    Q = np.loadtxt(SHELF_QUERIES, dtype=np.float32)[:n_eval]
    res, runs = {}, {}

    def plan_one(k, sampler, seed):
        row = Q[k]
        prm = P.prrtc_plan_params_default()
        prm.seed, prm.max_rounds, prm.time_budget_ms = seed, SHELF_MAX_ROUNDS, budget_ms
        prm.sampler, prm.model_id, prm.mix = sampler, mid, 0.5
        t1 = time.perf_counter()
        st, _, stats = P.prrtc_plan(ctx, rid, sid, row[:14], row[14:], prm)
        return st == P.PRRTC_OK, (time.perf_counter() - t1) * 1e3, stats["rounds"]

    for name, sampler in (("plain", 0), ("learned", 1)):
        a = np.array([plan_one(k, sampler, W.SEED_QUERY + k) for k in range(len(Q))], np.float64)
        runs[name] = a
        t = np.where(a[:, 0] > 0, a[:, 1], np.inf)
        res[name] = {"queries": len(a), "success": float(a[:, 0].mean()), **pcts(t),
                     "mean_rounds_solved": float(a[a[:, 0] > 0, 2].mean()) if a[:, 0].any() else None}
        log("  shelf %s: %s" % (name, res[name]))
    # where the two differ: the queries only one sampler failed, and whether
    # the failures repeat under four other seeds (a systematic miss) or not
    fails = {}
    for name, sampler in (("plain", 0), ("learned", 1)):
        other = "learned" if name == "plain" else "plain"
        idx = [k for k in range(len(Q)) if not runs[name][k, 0]]
        fails[name] = {"failed": idx,
                       "failed_only_here": [k for k in idx if runs[other][k, 0]],
                       "other_sampler_ms_on_those": [round(float(runs[other][k, 1]), 2) for k in idx if runs[other][k, 0]],
                       "solved_with_other_seeds": [int(sum(plan_one(k, sampler, W.SEED_QUERY + k + 7919 * r)[0]
                                                           for r in range(1, 5))) for k in idx]}
        log("  shelf %s failures: %s" % (name, fails[name]))
    res["failures"] = fails
    return {"_model": mid, "workload": "learned_r14_shelf", "train_queries": n_train,
            "solved_train_queries": int(ds.vox.shape[0]),
            "samples": int(len(ds.scene_of)), "epochs": epochs, "datagen_s": gen_s,
            "loss_first_epoch": float(losses[0]) if len(losses) else None,
            "loss_last_epoch": float(losses[-1]) if len(losses) else None,
            "time_budget_ms": budget_ms, "path_tail": tail, "plain": res["plain"], "learned": res["learned"],
            "failures": res["failures"]}


def host_cpu():
    """Model name and logical CPU counts of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(ce, max_threads=16):
    """The oracle (C, FP64, boolean mode: each edge stops at its first
    colliding point) on the host: OpenMP over the full 2^20-edge batch on the
    cores this process may use (at most 16), and one core on the first 65,536
    edges.  Also returns the oracle's verdicts of the full batch."""
    import oracle
    rob = oracle.OracleRobot(ce["robot"])
    model, nproc, avail = host_cpu()
    threads = max(1, min(max_threads, avail))
    t0 = time.perf_counter()
    v, f, _ = oracle.check_edges(rob, ce["prims"], ce["a"], ce["b"], RES, early_exit=True, n_threads=threads)
    t_all = time.perf_counter() - t0
    n1 = 65536
    t0 = time.perf_counter()
    oracle.check_edges(rob, ce["prims"], ce["a"][:n1], ce["b"][:n1], RES, early_exit=True, n_threads=1)
    t_one = time.perf_counter() - t0
    out = {"value": N_EDGES / t_all, "unit": "edge checks/s", "cores": threads, "kind": "oracle",
           "sample": f"the full 2^20-edge batch, early-exit boolean mode, OpenMP on {threads} threads, {t_all:.1f} s",
           "single_core": {"value": n1 / t_one, "unit": "edge checks/s", "cores": 1,
                           "sample": f"first {n1} edges of the batch, 1 thread, {t_one:.1f} s"},
           "cpu_model": model, "nproc": nproc, "cpus_available": avail}
    return out, v.astype(bool), f.astype(bool)


def finite_or_null(x):
    """Plain JSON: numpy scalars to Python numbers, non-finite floats to null."""
    if isinstance(x, dict):
        return {k: finite_or_null(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite_or_null(v) for v in x]
    if isinstance(x, (np.integer,)):
        return int(x)
    if isinstance(x, (float, np.floating)):
        return float(x) if np.isfinite(x) else None
    return x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the oracle CPU baseline")
    ap.add_argument("--skip-plan", action="store_true", help="omit the planner ms-to-solution run")
    ap.add_argument("--skip-learned", action="store_true", help="omit the learned-proposal leg")
    ap.add_argument("--skip-shelf", action="store_true", help="omit the 14-DoF shelf leg")
    ap.add_argument("--skip-learned-shelf", action="store_true", help="omit the 14-DoF learned-proposal leg")
    ap.add_argument("--learned-shelf-train", type=int, default=1500)
    ap.add_argument("--learned-shelf-eval", type=int, default=500)
    ap.add_argument("--learned-shelf-tail", type=float, default=1.0,
                    help="train the shelf proposal on the last fraction of each path only")
    ap.add_argument("--shelf-queries", type=int, default=500, help="stored shelf queries planned (500 in all)")
    ap.add_argument("--learned-scenes", type=int, default=10000, help="training scenes")
    ap.add_argument("--learned-eval", type=int, default=500, help="held-out scenes")
    ap.add_argument("--learned-epochs", type=int, default=16)
    ap.add_argument("--skip-serve", action="store_true", help="omit the batched / served planner legs")
    ap.add_argument("--skip-variants", action="store_true",
                    help="omit the two-stage and ESDF check_edges variants")
    ap.add_argument("--skip-sampling", action="store_true",
                    help="omit the sampling variants (uniform, dynamic domain, Halton)")
    ap.add_argument("--serve-queries", type=int, default=10000)
    ap.add_argument("--edge-schedule", type=int, default=-1,
                    help="pin the check_edges schedule of the headline leg (default: the timed choice)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(queries and edge batches shard across GPUs without exchange).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2503_06757_amd import prrtc as P
    ctx = P.prrtc_create(0)
    ce = bench_check_edges(P, ctx, torch, args.steps, args.warmup, args.edge_schedule)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    plan = None if args.skip_plan else bench_plan(P, ctx)
    variants = None if args.skip_variants else bench_collision_variants(P, ctx, torch)
    graphs = None if args.skip_variants else bench_graph_launches(P, ctx, torch)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    shelf = None
    if not args.skip_shelf:
        log("14-DoF shelf")
        shelf = bench_shelf(P, ctx, args.shelf_queries)
        log("  " + json.dumps(finite_or_null(shelf)))
    sampling = None
    if not args.skip_sampling:
        log("sampling variants")
        sampling = bench_sampling(P, ctx)
        log("  " + json.dumps(finite_or_null(sampling)))
    serve = batch = pool = burst = None
    if not args.skip_serve:
        log("batched planner: launch shapes")
        pool = query_pool(P, ctx, torch)
        log("  pool: %d solvable of %d free queries" % (len(pool[0]), pool[1]))
        batch = bench_throughput(P, ctx, torch, pool, log=log)
        log("served planner: Poisson arrivals")
        serve = bench_serve(P, ctx, torch, pool, n_queries=args.serve_queries, log=log)
        serve.pop("_latency_ms"), serve.pop("_ok")
        log("  " + json.dumps(finite_or_null(serve)))
        log("served planner: quiet stream, then a burst")
        burst = bench_serve_burst(P, ctx, torch, pool, log=log)
    learned = None
    if not args.skip_learned:
        log("learned proposal")
        learned = bench_learned(P, ctx, torch, args.learned_scenes, args.learned_eval, args.learned_epochs, log)
        log("  " + json.dumps(finite_or_null({k: v for k, v in learned.items() if k != "_model"})))
    learned_shelf = None
    if not args.skip_learned_shelf:
        log("learned proposal, dual-arm shelf")
        learned_shelf = bench_learned_shelf(P, ctx, torch, args.learned_shelf_train, args.learned_shelf_eval,
                                            args.learned_epochs, log, tail=args.learned_shelf_tail)
        log("  " + json.dumps(finite_or_null({k: v for k, v in learned_shelf.items() if k != "_model"})))
    served_learned = None
    if serve is not None and learned is not None and learned_shelf is not None:
        # the same pool, arrivals and launch shape with learned sampling: the
        # 7-DoF model of the generated scenes, the dual arm's shelf model
        log("served planner, learned sampling")
        served_learned = bench_serve(P, ctx, torch, pool, n_queries=args.serve_queries, log=log,
                                     models=(learned["_model"], learned_shelf["_model"]),
                                     workers=serve["workers"], tile=serve["tile"])
        served_learned.pop("_latency_ms"), served_learned.pop("_ok")
        log("  " + json.dumps(finite_or_null(served_learned)))
    for leg in (learned, learned_shelf):
        if leg is not None:
            leg.pop("_model", None)
    ms_per_step = ce["wall_s"] * 1e3 / args.steps
    value = N_EDGES / (ce["wall_s"] / args.steps)
    alg_flop = ce["free_points"] * ce["flop_per_point_model"]
    achieved = alg_flop / (ce["kernel_ms"] * 1e-3) / 1e12
    reduced = ce["free_points"] * ce["flop_per_point"] / (ce["kernel_ms"] * 1e-3) / 1e12
    free_tflops = ce["free_points"] * ce["flop_per_point_model"] / (ce["free_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "edge checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "check_edges_r7_s64_2p20", "robot": "7-DoF arm, 60 spheres",
                   "obstacles": "32 spheres, 21 cuboids, 11 cylinders", "edges": N_EDGES,
                   "res_per_rad": RES, "valid_fraction": ce["valid_frac"],
                   "mean_points_per_edge": ce["mean_points"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": load_traffic("k_check_edges", "r7_s64_2p20"),
                     "kernel": "k_check_edges", "kernel_ms": ce["kernel_ms"],
                     "schedule": EDGE_SCHEDULES.get(ce["schedule"], "none"),
                     "flop_per_launch": alg_flop, "flop_per_point": ce["flop_per_point_model"],
                     "points_counted": ce["free_points"],
                     "reduced_model": {"flop_per_point": ce["flop_per_point"], "achieved": reduced,
                                       "frac": reduced / PEAK_FP32_TFLOPS},
                     "collision_free_launch": {"edges": ce["free_edges"], "kernel_ms": ce["free_ms"],
                                               "achieved": free_tflops, "frac": free_tflops / PEAK_FP32_TFLOPS,
                                               "all_valid": ce["free_all_valid"]}},
        "collision_variants": variants,
        "graph_launches": graphs,
        "ms_to_solution": plan,
        "ms_to_solution_r14_shelf": shelf,
        "sampling_variants": sampling,
        "batched": batch,
        "served": serve,
        "served_burst": burst,
        "served_learned": served_learned,
        "learned": learned,
        "learned_r14_shelf": learned_shelf,
    }
    if not args.skip_cpu:
        cb, ov, of = cpu_baseline(ce)
        cb["gpu_verdicts_equal_unflagged"] = bool(np.array_equal(ov[~of], ce["valid"][~of]))
        cb["flagged"] = int(of.sum())
        out["cpu_baseline"] = cb
    P.prrtc_destroy(ctx)
    print(json.dumps(finite_or_null(out)), flush=True)


if __name__ == "__main__":
    main()
