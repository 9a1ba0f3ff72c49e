"""Seeded synthetic workloads: robots, scenes, edges and query candidates.

This module only *generates inputs*.  It holds none of the planner's or the
collision checker's arithmetic (no forward kinematics, no clearance test, no
sampling of the planner's random configurations): the HIP library and the
oracle both consume the exact float32 arrays built here, so that both sides
see identical bytes.

The paper evaluates on MotionBenchMaker scenes (Sec. IV-A), which are not
available here; these generators stand in for them with the shapes fixed by
the workload descriptions (a 7-DoF revolute arm with collision spheres along
its links, random scenes of spheres / oriented cuboids / cylinders, a 14-DoF
dual arm in front of a shelf).  Randomness comes from numpy's PCG64 streams
with named 64-bit seeds.
"""
from __future__ import annotations

import math

import numpy as np

PRIM_SPHERE, PRIM_CUBOID, PRIM_CYLINDER = 0, 1, 2

# One scene primitive, 64 bytes, little endian.  ``rot`` is a row-major 3x3
# whose columns are the primitive's axes (cylinder axis = column 2); ``dims``
# holds the radius (sphere), half-extents (cuboid) or (radius, half-height)
# (cylinder).
PRIM_DTYPE = np.dtype([("type", "<i4"), ("c", "<f4", (3,)), ("rot", "<f4", (9,)),
                       ("dims", "<f4", (3,))])
assert PRIM_DTYPE.itemsize == 64

# Named seeds of the synthetic workloads.
SEED_R7_SPHERES = 0x52370001
SEED_S12 = 0x53120000          # + instance index
SEED_S64 = 0x53640000
SEED_EDGES = 0x45000000
SEED_SHELF_SPHERES = 0x53480000
SEED_QUERY = 0x51000000        # + query index

# 7-DoF arm, modified (Craig) DH: joint j applies Rx(alpha_j) Tx(a_j) Rz(q_j) Tz(d_j).
R7_D = (0.333, 0.0, 0.316, 0.0, 0.384, 0.0, 0.107)
R7_A = (0.0, 0.0, 0.0, 0.0825, -0.0825, 0.0, 0.088)
R7_ALPHA = (0.0, -math.pi / 2, math.pi / 2, math.pi / 2, -math.pi / 2, math.pi / 2, math.pi / 2)
R7_LIMIT = 2.8
R7_LINK_SPHERES = 52
R7_HAND_SPHERES = 8
R7_RADIUS = (0.03, 0.08)
R7_HAND_HALF_WIDTH = 0.05      # the hand bar (with its spheres) fits a 0.28 m shelf cell

SCENE_HALF = 0.8            # scenes live in the cube [-0.8, 0.8]^3
BASE_BALL = 0.25            # keep-out ball around each chain base


def _segment_offsets(alpha, a, d):
    """Origin of frame j+1 expressed in frame j (it does not depend on q_j).

    With the per-joint product Rx(alpha) Tx(a) Rz(q) Tz(d), the point (0,0,d)
    is fixed by Rz(q), so the next origin sits at (a, -sin(alpha) d, cos(alpha) d).
    This places collision spheres; it is robot-model construction, not FK.
    """
    return [np.array([aj, -math.sin(al) * dj, math.cos(al) * dj]) for al, aj, dj in zip(alpha, a, d)]


def _r7_sphere_layout(radii):
    """52 spheres evenly by arc length along the link polyline + 8 on a hand bar
    (y in [-0.05, 0.05] m at z = 0.06 m in the flange frame).

    Returns (frame ids 0..7 within the chain, local xyz (60,3) float64).
    """
    segs = _segment_offsets(R7_ALPHA, R7_A, R7_D)
    lens = [float(np.linalg.norm(s)) for s in segs]
    total = sum(lens)
    frames, xyz = [], []
    for k in range(R7_LINK_SPHERES):
        s = (k + 0.5) * total / R7_LINK_SPHERES
        acc = 0.0
        for j, (v, ln) in enumerate(zip(segs, lens)):
            if ln > 0.0 and s <= acc + ln:
                frames.append(j)
                xyz.append((s - acc) / ln * v)
                break
            acc += ln
        else:  # numerical tail: last non-empty segment end
            frames.append(6)
            xyz.append(segs[6].copy())
    for k in range(R7_HAND_SPHERES):
        y = -R7_HAND_HALF_WIDTH + 2.0 * R7_HAND_HALF_WIDTH * k / (R7_HAND_SPHERES - 1)
        frames.append(7)
        xyz.append(np.array([0.0, y, 0.06]))
    return np.array(frames, np.int32), np.array(xyz)


def _pose(t):
    p = np.zeros(12, np.float32)
    p[0] = p[5] = p[10] = 1.0
    p[3], p[7], p[11] = t
    return p


def robot_r7(seed: int = SEED_R7_SPHERES) -> dict:
    """Synthetic 7-DoF revolute arm with 60 collision spheres (single chain),
    radii ~ U[0.03, 0.08]."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(*R7_RADIUS, R7_LINK_SPHERES + R7_HAND_SPHERES)
    frames, xyz = _r7_sphere_layout(radii)
    xyzr = np.concatenate([xyz, radii[:, None]], axis=1).astype(np.float32)
    dh = np.array([R7_ALPHA, R7_A, R7_D], np.float64).T.astype(np.float32)
    return dict(
        name="R7", n_chains=1, chain_dof=[7], base_pose=_pose((0.0, 0.0, 0.0))[None, :],
        dh=dh, q_lo=np.full(7, -R7_LIMIT, np.float32), q_hi=np.full(7, R7_LIMIT, np.float32),
        sphere_frame=frames.astype(np.int32), sphere_xyzr=xyzr,
        self_pairs=np.zeros((0, 2), np.int32),
    )


def robot_r14(seed: int = SEED_R7_SPHERES) -> dict:
    """Two copies of the 7-DoF chain with bases 0.6 m apart along y.

    Spheres 0..59 belong to chain A (global frames 0..7), 60..119 to chain B
    (global frames 8..15).  Self-collision pairs: every (A, B) sphere pair.
    """
    r7 = robot_r7(seed)
    n = r7["sphere_xyzr"].shape[0]
    frames = np.concatenate([r7["sphere_frame"], r7["sphere_frame"] + 8]).astype(np.int32)
    xyzr = np.concatenate([r7["sphere_xyzr"], r7["sphere_xyzr"]]).astype(np.float32)
    ia, ib = np.meshgrid(np.arange(n), np.arange(n, 2 * n), indexing="ij")
    pairs = np.stack([ia.ravel(), ib.ravel()], axis=1).astype(np.int32)
    return dict(
        name="R14", n_chains=2, chain_dof=[7, 7],
        base_pose=np.stack([_pose((0.0, -0.3, 0.0)), _pose((0.0, 0.3, 0.0))]),
        dh=np.concatenate([r7["dh"], r7["dh"]]).astype(np.float32),
        q_lo=np.full(14, -R7_LIMIT, np.float32), q_hi=np.full(14, R7_LIMIT, np.float32),
        sphere_frame=frames, sphere_xyzr=xyzr, self_pairs=pairs,
    )


def robot_r14_arm(arm: int, seed: int = SEED_R7_SPHERES) -> dict:
    """One arm of the dual-arm robot on its own (chain ``arm`` at its base), for
    per-arm goal sampling."""
    r7 = robot_r7(seed)
    r7["name"] = f"R14-arm{arm}"
    r7["base_pose"] = robot_r14(seed)["base_pose"][arm:arm + 1].copy()
    return r7


def with_coarse_spheres(robot: dict, group: int = 8) -> dict:
    """The robot with a second, coarse sphere set for two-stage collision
    checking (Sec. III-A checks low-resolution spheres first and re-checks
    only the links they flag with the fine ones; the paper gets both sets from
    `foam`, here they are synthetic): on each frame, runs of up to `group`
    consecutive fine spheres share one coarse sphere centred on the run's
    bounding box, its radius reaching the farthest fine sphere's far side.
    Adds coarse_xyzr (n_c, 4), coarse_frame (n_c,) and sphere_coarse (fine ->
    coarse index)."""
    frames = np.asarray(robot["sphere_frame"])
    xyzr = np.asarray(robot["sphere_xyzr"], np.float64)
    coarse, cframe = [], []
    owner = np.zeros(len(frames), np.int32)
    for f in np.unique(frames):
        idx = np.nonzero(frames == f)[0]
        for k0 in range(0, len(idx), group):
            run = idx[k0:k0 + group]
            c = 0.5 * (xyzr[run, :3].min(axis=0) + xyzr[run, :3].max(axis=0))
            r = np.max(np.linalg.norm(xyzr[run, :3] - c, axis=1) + xyzr[run, 3])
            owner[run] = len(coarse)
            coarse.append(np.concatenate([c, [r]]))
            cframe.append(int(f))
    out = dict(robot)
    out["coarse_xyzr"] = np.array(coarse, np.float32)
    # float32 centres: widen the radius so every fine sphere stays inside
    cx = out["coarse_xyzr"]
    for k in range(len(frames)):
        d = np.linalg.norm(xyzr[k, :3] - cx[owner[k], :3].astype(np.float64)) + xyzr[k, 3]
        if d > cx[owner[k], 3]:
            cx[owner[k], 3] = np.nextafter(np.float32(d), np.float32(np.inf))
    out["coarse_frame"] = np.array(cframe, np.int32)
    out["sphere_coarse"] = owner
    out["name"] = robot["name"] + "-2stage"
    return out


def robot_dof(robot: dict) -> int:
    return int(sum(robot["chain_dof"]))


def _fixed_sphere_world(robot: dict):
    """World positions/radii of spheres on chain base frames (they never move)."""
    out = []
    off = 0
    for c, dof in enumerate(robot["chain_dof"]):
        pose = robot["base_pose"][c].astype(np.float64).reshape(3, 4)
        for k in range(robot["sphere_frame"].shape[0]):
            if robot["sphere_frame"][k] == off:
                p = robot["sphere_xyzr"][k, :3].astype(np.float64)
                out.append((pose[:, :3] @ p + pose[:, 3], float(robot["sphere_xyzr"][k, 3])))
        off += dof + 1
    return out


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def make_prims(entries) -> np.ndarray:
    """entries: iterable of (type, centre(3), rot(3x3), dims(3)) -> PRIM_DTYPE array."""
    entries = list(entries)
    out = np.zeros(len(entries), PRIM_DTYPE)
    for i, (t, c, r, d) in enumerate(entries):
        out[i]["type"] = t
        out[i]["c"] = np.asarray(c, np.float64)
        out[i]["rot"] = np.asarray(r, np.float64).reshape(9)
        out[i]["dims"] = np.asarray(d, np.float64)
    return out


def random_scene(seed: int, robot: dict, n_sphere: int, n_cuboid: int, n_cylinder: int,
                 sphere_r=(0.05, 0.15), cuboid_h=(0.05, 0.3), cyl_r=(0.03, 0.1),
                 cyl_h=(0.2, 0.6)) -> np.ndarray:
    """Random primitives with centres uniform in the scene cube.

    Obstacles whose bounding sphere reaches a chain's 0.25 m base ball or one
    of the fixed base-frame spheres are redrawn (a conservative bounding-sphere
    rejection, so start configurations near the base stay feasible).
    Cylinder heights are full heights; the primitive stores half-heights.
    """
    rng = np.random.default_rng(seed)
    fixed = _fixed_sphere_world(robot)
    bases = [robot["base_pose"][c].astype(np.float64).reshape(3, 4)[:, 3]
             for c in range(robot["n_chains"])]
    entries = []
    for t, count in ((PRIM_SPHERE, n_sphere), (PRIM_CUBOID, n_cuboid), (PRIM_CYLINDER, n_cylinder)):
        for _ in range(count):
            while True:
                c = rng.uniform(-SCENE_HALF, SCENE_HALF, 3)
                rot = _random_rotation(rng)
                if t == PRIM_SPHERE:
                    dims = np.array([rng.uniform(*sphere_r), 0.0, 0.0])
                    bound = dims[0]
                    rot = np.eye(3)
                elif t == PRIM_CUBOID:
                    dims = rng.uniform(cuboid_h[0], cuboid_h[1], 3)
                    bound = float(np.linalg.norm(dims))
                else:
                    r = rng.uniform(*cyl_r)
                    h = rng.uniform(*cyl_h)
                    dims = np.array([r, 0.5 * h, 0.0])
                    bound = math.hypot(r, 0.5 * h)
                ok = all(np.linalg.norm(c - b) >= bound + BASE_BALL for b in bases)
                ok = ok and all(np.linalg.norm(c - p) >= bound + r_s for p, r_s in fixed)
                if ok:
                    break
            entries.append((t, c, rot, dims))
    return make_prims(entries)


def scene_s12(robot: dict, instance: int = 0) -> np.ndarray:
    """12 obstacles: 6 spheres, 4 oriented cuboids, 2 cylinders."""
    return random_scene(SEED_S12 + instance, robot, 6, 4, 2)


def scene_s64(robot: dict, seed: int = SEED_S64) -> np.ndarray:
    """64 obstacles with the 6:4:2 type mix: 32 spheres, 21 cuboids, 11 cylinders."""
    return random_scene(seed, robot, 32, 21, 11)


def scene_mixed(seed: int, robot: dict, n_obstacles: int) -> np.ndarray:
    """n obstacles split 6:4:2 across spheres, cuboids and cylinders."""
    n_s = int(round(n_obstacles * 6 / 12))
    n_b = int(round(n_obstacles * 4 / 12))
    n_c = n_obstacles - n_s - n_b
    return random_scene(seed, robot, n_s, n_b, n_c)


# ---- shelf scene (14-DoF workload) -------------------------------------------------
SHELF_FRONT_X = 0.45
SHELF_CELL = 0.3
SHELF_WALL = 0.02
SHELF_COLS, SHELF_ROWS = 5, 3
SHELF_Y0 = -0.75
SHELF_Z0 = 0.10


def shelf_cells():
    """Inner boxes (lo, hi) of the 5x3 shelf cells, in world coordinates."""
    cells = []
    for row in range(SHELF_ROWS):
        for col in range(SHELF_COLS):
            lo = np.array([SHELF_FRONT_X, SHELF_Y0 + col * SHELF_CELL, SHELF_Z0 + row * SHELF_CELL])
            hi = lo + SHELF_CELL
            cells.append((lo, hi))
    return cells


def scene_shelf(robot: dict, n_random_spheres: int = 24, seed: int = SEED_SHELF_SPHERES) -> np.ndarray:
    """5x3 shelf of 0.3 m cells built from 40 axis-aligned cuboids, plus random spheres.

    20 horizontal boards (4 levels x 5 columns), 18 vertical dividers
    (6 x 3 rows), one back panel and one pedestal.  The opening faces -x.
    The random spheres (r ~ U[0.05, 0.15]) lie in the upper half of the scene
    cube, clear of the shelf, of the arm bases and of the approach slab
    between the bases and the shelf front (0 <= x <= 0.45 m): clutter around
    and behind the robot, not a wall across every route into the cells.
    """
    ident = np.eye(3)
    t = SHELF_WALL / 2.0
    depth = SHELF_CELL
    xc = SHELF_FRONT_X + depth / 2.0
    entries = []
    for level in range(SHELF_ROWS + 1):
        z = SHELF_Z0 + level * SHELF_CELL
        for col in range(SHELF_COLS):
            y = SHELF_Y0 + (col + 0.5) * SHELF_CELL
            entries.append((PRIM_CUBOID, (xc, y, z), ident, (depth / 2, SHELF_CELL / 2, t)))
    for k in range(SHELF_COLS + 1):
        y = SHELF_Y0 + k * SHELF_CELL
        for row in range(SHELF_ROWS):
            z = SHELF_Z0 + (row + 0.5) * SHELF_CELL
            entries.append((PRIM_CUBOID, (xc, y, z), ident, (depth / 2, t, SHELF_CELL / 2)))
    height = SHELF_ROWS * SHELF_CELL
    width = SHELF_COLS * SHELF_CELL
    entries.append((PRIM_CUBOID, (SHELF_FRONT_X + depth + t, 0.0, SHELF_Z0 + height / 2), ident,
                    (t, width / 2, height / 2)))
    entries.append((PRIM_CUBOID, (xc, 0.0, SHELF_Z0 / 2 - t / 2), ident,
                    (depth / 2, width / 2, SHELF_Z0 / 2 - t / 2)))
    assert len(entries) == 40
    prims = make_prims(entries)
    if n_random_spheres:
        rnd = _random_spheres_outside_shelf(seed, robot, n_random_spheres)
        prims = np.concatenate([prims, rnd])
    return prims


APPROACH_LO = np.array([0.0, -SCENE_HALF, 0.0])            # region kept free of random spheres
APPROACH_HI = np.array([SHELF_FRONT_X, SCENE_HALF, SHELF_Z0 + 0.9])


def _random_spheres_outside_shelf(seed, robot, n):
    rng = np.random.default_rng(seed)
    fixed = _fixed_sphere_world(robot)
    bases = [robot["base_pose"][c].astype(np.float64).reshape(3, 4)[:, 3]
             for c in range(robot["n_chains"])]
    shelf_lo = np.array([SHELF_FRONT_X, SHELF_Y0, 0.0])
    shelf_hi = np.array([SHELF_FRONT_X + SHELF_CELL + SHELF_WALL, -SHELF_Y0, SHELF_Z0 + 0.9 + SHELF_WALL])
    entries = []
    while len(entries) < n:
        c = rng.uniform(-SCENE_HALF, SCENE_HALF, 3)
        c[2] = abs(c[2]) + 0.0  # keep random clutter above the floor plane
        r = rng.uniform(0.05, 0.15)
        if any(np.linalg.norm(c - b) < r + BASE_BALL for b in bases):
            continue
        if any(np.linalg.norm(c - p) < r + rs for p, rs in fixed):
            continue
        # keep the shelf cells themselves clear so goals inside them stay reachable
        if np.all(c > shelf_lo - r) and np.all(c < shelf_hi + r):
            continue
        # and the approach to the opening: the slab between the arm bases and
        # the shelf front, across the shelf's width and height
        if np.all(c > APPROACH_LO - r) and np.all(c < APPROACH_HI + r):
            continue
        entries.append((PRIM_SPHERE, c, np.eye(3), (r, 0.0, 0.0)))
    return make_prims(entries)


# ---- edges and queries -------------------------------------------------------------
def random_edges(robot: dict, n: int, seed: int = SEED_EDGES, length=(0.05, 1.0)):
    """n edges: a uniform within the limits, direction uniform on the sphere,
    length uniform in ``length``; the direction is redrawn (up to 64 times) if
    b leaves the limits, then a is redrawn.  Returns float32 (a, b), each (n, dof)."""
    rng = np.random.default_rng(seed)
    lo = robot["q_lo"].astype(np.float64)
    hi = robot["q_hi"].astype(np.float64)
    dof = lo.shape[0]
    a = np.empty((n, dof))
    b = np.empty((n, dof))
    todo = np.arange(n)
    while todo.size:
        m = todo.size
        aa = rng.uniform(lo, hi, (m, dof))
        ln = rng.uniform(length[0], length[1], m)
        bb = np.empty_like(aa)
        ok = np.zeros(m, bool)
        for _ in range(64):
            pend = np.nonzero(~ok)[0]
            if pend.size == 0:
                break
            d = rng.standard_normal((pend.size, dof))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            cand = aa[pend] + ln[pend, None] * d
            inside = np.all((cand >= lo) & (cand <= hi), axis=1)
            bb[pend[inside]] = cand[inside]
            ok[pend[inside]] = True
        a[todo[ok]] = aa[ok]
        b[todo[ok]] = bb[ok]
        todo = todo[~ok]
    return a.astype(np.float32), b.astype(np.float32)


def query_candidates(robot: dict, seed: int, n: int, min_dist: float = 1.0):
    """Candidate (start, goal) pairs uniform in the limits, ||goal - start|| >= min_dist.

    The caller keeps the first candidate whose endpoints its own collision
    check accepts (the generator never tests collisions).
    """
    rng = np.random.default_rng(seed)
    lo = robot["q_lo"].astype(np.float64)
    hi = robot["q_hi"].astype(np.float64)
    out = []
    while len(out) < n:
        s = rng.uniform(lo, hi)
        g = rng.uniform(lo, hi)
        if np.linalg.norm(g - s) >= min_dist:
            out.append((s.astype(np.float32), g.astype(np.float32)))
    return out


# ---- shelf queries (14-DoF workload) ------------------------------------------------
HAND_SPHERES = slice(52, 60)   # the 8 hand-bar spheres of one arm (R7 sphere order)
SHELF_MARGIN = 0.03


def hand_cell(hand_xyz: np.ndarray, margin: float = SHELF_MARGIN) -> int:
    """Index of the shelf cell whose interior (shrunk by ``margin``) holds the
    centre of the hand bar (the mean of the hand spheres' centres), or -1.
    Positions come from the caller's own forward kinematics; whether the hand
    then fits between the walls is left to the caller's collision check."""
    centre = np.mean(np.asarray(hand_xyz, np.float64), axis=0)
    for k, (lo, hi) in enumerate(shelf_cells()):
        if np.all(centre >= lo + SHELF_WALL / 2 + margin) and np.all(centre <= hi - SHELF_WALL / 2 - margin):
            return k
    return -1


def shelf_query_candidates(seed: int, n: int, dof_arm: int = 7, limit: float = R7_LIMIT):
    """Per-arm candidate configurations for one 14-DoF shelf query: ``n``
    uniform start candidates for the whole robot and ``n`` uniform goal
    candidates for each arm.  The caller keeps a start whose hands are outside
    the shelf and, per arm, the first goal candidate whose hand is inside a
    cell on the arm's own side (y < 0 for arm A, y > 0 for arm B), then checks
    the combined configurations with its own collision checker."""
    rng = np.random.default_rng(seed)
    starts = rng.uniform(-limit, limit, (n, 2 * dof_arm)).astype(np.float32)
    goals_a = rng.uniform(-limit, limit, (n, dof_arm)).astype(np.float32)
    goals_b = rng.uniform(-limit, limit, (n, dof_arm)).astype(np.float32)
    return starts, goals_a, goals_b
