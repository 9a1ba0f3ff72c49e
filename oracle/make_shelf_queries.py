"""Write the dual-arm shelf queries (start, goal) used by the tests and the
benchmark: ``python oracle/make_shelf_queries.py N OUT [JOBS]``.

Calls only the oracle (FK and clearances) and the seeded generators.  Query i
uses numpy seed SEED_QUERY + 1000 + i:
  * start: uniform 14-DoF configurations until one is collision-free with
    clearance > 1e-3 m and every sphere in front of the shelf (x < 0.4 m);
  * goal, per arm: uniform arm configurations whose hand-bar centre lies in a
    shelf cell on the arm's side (arm 0: y < 0, arm 1: y > 0), the eight with
    the largest clearance (arm alone) refined by a seeded random hill climb on
    that clearance until it exceeds GOAL_CLEARANCE, kept if a straight
    joint-space retreat of 0.5-2 rad leads, collision-free, to a configuration
    with the arm in front of the shelf; the two arms' goals together must be
    collision-free (including the inter-arm pairs) with clearance > 1e-3 m.
Rows are written as float32 with 9 significant digits (exact round trip).
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2503_06757_amd import workloads as W  # noqa: E402


GOAL_CLEARANCE = 0.02   # m: a grasp pose with room around the hand, not a jammed one
ESCAPE_TRIES = 256      # straight joint-space retreats tried per goal
ESCAPE_STEP = (0.5, 2.0)  # rad: length of a retreat


def _escapes(rng, rob_arm, prims, q):
    """Is there a straight joint-space segment of ESCAPE_STEP length from q to
    a configuration with every sphere in front of the shelf (x < 0.4 m) that
    is collision-free at 32 points per rad?  (A grasp pose the arm can back
    out of, as pick poses in a shelf are.)"""
    d = rng.standard_normal((ESCAPE_TRIES, 7))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    b = np.clip(q[None, :] + rng.uniform(*ESCAPE_STEP, (ESCAPE_TRIES, 1)) * d, -W.R7_LIMIT, W.R7_LIMIT)
    b = b.astype(np.float32)
    out = [k for k in range(ESCAPE_TRIES) if np.all(O.fk_spheres(rob_arm, b[k])[:, 0] < 0.4)]
    if not out:
        return False
    a = np.repeat(q[None, :], len(out), 0).astype(np.float32)
    valid = O.check_edges(rob_arm, prims, a, b[out], 32.0, early_exit=True, n_threads=1)[0]
    return bool(valid.any())


def _arm_goal(rng, rob_arm, prims, arm):
    def score(q):
        xyz = O.fk_spheres(rob_arm, q)
        c = W.hand_cell(xyz[W.HAND_SPHERES])
        if c < 0:
            return None
        lo, hi = W.shelf_cells()[c]
        if (arm == 0 and hi[1] > 1e-9) or (arm == 1 and lo[1] < -1e-9):
            return None
        return O.config_clearance(rob_arm, prims, q.astype(np.float64))
    cands = []
    while len(cands) < 8:
        for q in rng.uniform(-W.R7_LIMIT, W.R7_LIMIT, (4096, 7)).astype(np.float32):
            s = score(q)
            if s is not None:
                cands.append((s, q))
    cands.sort(key=lambda x: -x[0])
    for s, q in cands[:8]:
        step = 0.1
        for it in range(600):
            if s > GOAL_CLEARANCE:
                return q if _escapes(rng, rob_arm, prims, q) else None
            qn = np.clip(q + rng.normal(0.0, step, 7).astype(np.float32), -W.R7_LIMIT, W.R7_LIMIT)
            sn = score(qn)
            if sn is not None and sn > s:
                q, s = qn, sn
            if it % 150 == 149:
                step *= 0.6
    return None


def make_query(i, rob14, arms, prims):
    rng = np.random.default_rng(W.SEED_QUERY + 1000 + i)
    while True:
        start = None
        while start is None:
            for q in rng.uniform(-W.R7_LIMIT, W.R7_LIMIT, (512, 14)).astype(np.float32):
                xyz = O.fk_spheres(rob14, q)
                if np.all(xyz[:, 0] < 0.4) and O.config_clearance(rob14, prims, q.astype(np.float64)) > 1e-3:
                    start = q
                    break
        ga = _arm_goal(rng, arms[0], prims, 0)
        gb = _arm_goal(rng, arms[1], prims, 1)
        if ga is None or gb is None:
            continue
        goal = np.concatenate([ga, gb]).astype(np.float32)
        if O.config_clearance(rob14, prims, goal.astype(np.float64)) > 1e-3:
            return start, goal


_STATE = {}


def _one(i):
    if not _STATE:
        r14 = W.robot_r14()
        _STATE["rob14"] = O.OracleRobot(r14)
        _STATE["arms"] = [O.OracleRobot(W.robot_r14_arm(a)) for a in (0, 1)]
        _STATE["prims"] = W.scene_shelf(r14)
    s, g = make_query(i, _STATE["rob14"], _STATE["arms"], _STATE["prims"])
    return np.concatenate([s, g])


def main():
    import multiprocessing as mp
    n = int(sys.argv[1]) if len(sys.argv) > 1 else 500
    out = sys.argv[2] if len(sys.argv) > 2 else os.path.join(ROOT, "tests", "golden", "shelf_queries_r14.txt")
    jobs = int(sys.argv[3]) if len(sys.argv) > 3 else min(8, os.cpu_count() or 1)
    with mp.Pool(jobs) as pool:
        rows = []
        for i, r in enumerate(pool.imap(_one, range(n))):   # query i depends on i only
            rows.append(r)
            print(i, flush=True)
    with open(out, "w") as fh:
        fh.write("# Dual-arm shelf queries: 14 start joints then 14 goal joints (rad), float32.\n")
        fh.write("# Written by oracle/make_shelf_queries.py %d (oracle FK and clearances only).\n" % n)
        for r in rows:
            fh.write(" ".join("%.9g" % v for v in r) + "\n")


if __name__ == "__main__":
    main()
