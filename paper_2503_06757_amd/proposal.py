"""Learned sampling proposal: weight initialisation, blob packing and the
training driver.  Every arithmetic step of the model runs in libprrtc's
kernels; this module only prepares arrays and calls the C ABI."""
from __future__ import annotations

import math
import struct
import time

import numpy as np

N_COMP = 8
HIDDEN = 256
VOX = 16
MAGIC, VERSION = 0x31505250, 1
PARAM_ORDER = ("Wv", "bv", "W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")
HEADER = struct.Struct("<IIiiiiqii")


def param_shapes(dof: int) -> dict:
    c = N_COMP * (1 + 2 * dof)
    return dict(Wv=(VOX ** 3, HIDDEN), bv=(HIDDEN,), W1=(2 * dof + HIDDEN, HIDDEN), b1=(HIDDEN,),
                W2=(HIDDEN, HIDDEN), b2=(HIDDEN,), W3=(HIDDEN, HIDDEN), b3=(HIDDEN,), W4=(HIDDEN, c), b4=(c,))


def init_params(dof: int, seed: int) -> dict:
    """He-normal hidden weights (GELU), a small head, zero biases; seeded."""
    rng = np.random.default_rng(seed)
    out = {}
    for k, shp in param_shapes(dof).items():
        if len(shp) == 1:
            out[k] = np.zeros(shp, np.float32)
        else:
            std = math.sqrt(2.0 / shp[0]) * (0.1 if k == "W4" else 1.0)
            if k == "Wv":
                std = math.sqrt(1.0 / 64.0)  # sparse binary input: ~64 occupied cells
            out[k] = (rng.standard_normal(shp) * std).astype(np.float32)
    return out


def pack(params: dict, dof: int, m: dict | None = None, v: dict | None = None, adam_t: int = 0) -> bytes:
    has = m is not None and v is not None
    parts = [HEADER.pack(MAGIC, VERSION, dof, HIDDEN, N_COMP, VOX, adam_t, int(has), 0)]
    for group in ([params] + ([m, v] if has else [])):
        for k in PARAM_ORDER:
            parts.append(np.ascontiguousarray(group[k], np.float32).tobytes())
    return b"".join(parts)


def unpack(blob: bytes):
    magic, ver, dof, hid, nc, vox, adam_t, has, _ = HEADER.unpack_from(blob, 0)
    assert magic == MAGIC and ver == VERSION and hid == HIDDEN and nc == N_COMP and vox == VOX
    shapes = param_shapes(dof)
    off = HEADER.size
    groups = []
    for _ in range(3 if has else 1):
        g = {}
        for k in PARAM_ORDER:
            n = int(np.prod(shapes[k]))
            g[k] = np.frombuffer(blob, np.float32, n, off).reshape(shapes[k]).copy()
            off += 4 * n
        groups.append(g)
    return dof, adam_t, groups


def resample_path(path: np.ndarray, step: float = 0.25, tail: float = 1.0) -> np.ndarray:
    """Waypoints every `step` rad of arclength along a path, endpoints excluded
    (training targets); with tail < 1 only those in the last `tail` fraction
    of the arclength (the approach to the goal)."""
    p = np.asarray(path, np.float64)
    seg = np.linalg.norm(np.diff(p, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    total = cum[-1]
    out = []
    t = step
    while t < (1.0 - tail) * total:
        t += step
    while t < total - 1e-9:
        i = min(int(np.searchsorted(cum, t, side="right")) - 1, len(seg) - 1)
        f = (t - cum[i]) / seg[i] if seg[i] > 0 else 0.0
        out.append(p[i] + f * (p[i + 1] - p[i]))
        t += step
    return np.array(out, np.float32).reshape(-1, p.shape[1])


# ---- training data, training and evaluation (drives the C ABI; needs a GPU) ----------
SEED_TRAIN = 0x54000000      # + scene index: training scenes
SEED_EVAL = 0x55000000       # + scene index: held-out scenes


def scene(robot: dict, index: int, base: int = SEED_TRAIN) -> np.ndarray:
    """Scene `index` of a family: U{8..128} obstacles, spheres/cuboids/cylinders 6:4:2."""
    from . import workloads as W
    n = int(np.random.default_rng(base + index).integers(8, 129))
    return W.scene_mixed(base + index, robot, n)


def free_query(P, ctx, torch, rid: int, sid: int, robot: dict, seed: int, n_cand: int = 64):
    """First generated (start, goal) whose endpoints the GPU collision check
    accepts (each configuration checked as a zero-length edge), or None."""
    from . import workloads as W
    cands = W.query_candidates(robot, seed, n_cand)
    q = torch.from_numpy(np.stack([c for pair in cands for c in pair]).astype(np.float32)).cuda()
    ok = torch.zeros(q.shape[0], dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, q.data_ptr(), q.data_ptr(), q.shape[0], 32.0, ok.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    ok = ok.cpu().numpy().reshape(-1, 2)
    for (s, g), (a, b) in zip(cands, ok):
        if a and b:
            return s, g
    return None


class Dataset:
    """Waypoint targets grouped by scene: vox [S][4096] (host uint8), and per
    sample scene index, start, goal and waypoint."""

    def __init__(self, dof):
        self.dof = dof
        self.vox, self.queries, self.paths = [], [], []
        self.scene_of, self.start, self.goal, self.waypoint = [], [], [], []

    def finish(self):
        d = self.dof
        self.vox = np.stack(self.vox) if self.vox else np.zeros((0, VOX ** 3), np.uint8)
        self.scene_of = np.asarray(self.scene_of, np.int32)
        self.start = np.asarray(self.start, np.float32).reshape(-1, d)
        self.goal = np.asarray(self.goal, np.float32).reshape(-1, d)
        self.waypoint = np.asarray(self.waypoint, np.float32).reshape(-1, d)
        return self


def generate(P, ctx, torch, rid: int, robot: dict, n_scenes: int, base: int = SEED_TRAIN, max_rounds: int = 1000,
             budget_ms: float = 50.0, log=None, chunk: int = 1024, workers: int = 64) -> Dataset:
    """Solve one query per scene with the uniform planner and keep the path's
    waypoints every 0.25 rad (endpoints excluded).  Scenes are taken `chunk`
    at a time: each scene's first free query, then one batched launch plans
    them all (seed base + i, `workers` workers per query).  Scenes without a
    free query or a solution within the round and time budget contribute no
    samples."""
    dof = int(np.asarray(robot["q_lo"]).shape[0])
    ds = Dataset(dof)
    stream = torch.cuda.current_stream().cuda_stream
    vox = torch.zeros((chunk, VOX ** 3), dtype=torch.uint8, device="cuda")
    p = P.prrtc_plan_params_default()
    p.workers, p.tile, p.max_rounds, p.time_budget_ms = workers, 16, max_rounds, budget_ms
    for c0 in range(0, n_scenes, chunk):
        idx = list(range(c0, min(n_scenes, c0 + chunk)))
        sids = [P.prrtc_load_scene(ctx, scene(robot, i, base)) for i in idx]
        qs = [free_query(P, ctx, torch, rid, sid, robot, base + i) for i, sid in zip(idx, sids)]
        live = [k for k, q in enumerate(qs) if q is not None]
        batch = [(rid, sids[k], qs[k][0], qs[k][1], base + idx[k], 0) for k in live]
        res = P.prrtc_plan_batch(ctx, batch, p, path_cap=512)[1] if batch else []
        solved = [(k, r[1]) for k, r in zip(live, res) if r[0] == P.PRRTC_OK]
        for j, (k, _) in enumerate(solved):
            P.prrtc_voxelize(ctx, sids[k], vox[j].data_ptr(), stream)
        grids = vox[:len(solved)].cpu().numpy()
        for j, (k, path) in enumerate(solved):
            n_vox = len(ds.vox)
            ds.vox.append(grids[j].copy())
            ds.queries.append(qs[k])
            ds.paths.append(path)
            for w in resample_path(path):
                ds.scene_of.append(n_vox)
                ds.start.append(qs[k][0])
                ds.goal.append(qs[k][1])
                ds.waypoint.append(w)
        for sid in sids:
            P.prrtc_unload_scene(ctx, sid)
        if log:
            log("  %d/%d scenes, %d solved, %d samples" % (idx[-1] + 1, n_scenes, len(ds.vox), len(ds.scene_of)))
    return ds.finish()


def train(P, ctx, torch, mid: int, rid: int, ds: Dataset, epochs: int, batch: int = 256, lr: float = 1e-3,
          seed: int = 0, log=None) -> np.ndarray:
    """Adam on the mean NLL.  Each epoch shuffles the scenes and cuts them into
    batches of whole scenes holding at least `batch` samples; every batch is
    a contiguous slice of arrays uploaded once per epoch.  Returns the mean
    loss of each epoch."""
    rng = np.random.default_rng(seed)
    n_sc = ds.vox.shape[0]
    counts = np.bincount(ds.scene_of, minlength=n_sc)
    first = np.concatenate([[0], np.cumsum(counts)])
    order_in = np.argsort(ds.scene_of, kind="stable")
    stream = torch.cuda.current_stream().cuda_stream
    out = []
    for ep in range(epochs):
        perm = rng.permutation(np.nonzero(counts)[0])
        idx = np.concatenate([order_in[first[s]:first[s + 1]] for s in perm])
        # batches: consecutive scenes of perm
        cuts, acc = [0], 0
        for j, s in enumerate(perm):
            acc += counts[s]
            if acc >= batch:
                cuts.append(j + 1)
                acc = 0
        if cuts[-1] != len(perm):
            cuts.append(len(perm))
        local = np.empty(len(idx), np.int32)
        starts = []
        pos = 0
        for b in range(len(cuts) - 1):
            cs = counts[perm[cuts[b]:cuts[b + 1]]]
            local[pos:pos + cs.sum()] = np.repeat(np.arange(len(cs), dtype=np.int32), cs)
            starts.append(np.concatenate([[0], np.cumsum(cs)]).astype(np.int32))
            pos += cs.sum()
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in dict(
            vox=ds.vox[perm], local=local, s=ds.start[idx], g=ds.goal[idx], w=ds.waypoint[idx],
            starts=np.concatenate(starts)).items()}
        losses = torch.zeros(len(cuts) - 1, dtype=torch.float32, device="cuda")
        a0, st0 = 0, 0
        for b in range(len(cuts) - 1):
            n_sb = cuts[b + 1] - cuts[b]
            n_b = int(starts[b][-1])
            tb = P.prrtc_train_batch(
                vox=dev["vox"].data_ptr() + cuts[b] * VOX ** 3, n_scenes=n_sb,
                scene_start=dev["starts"].data_ptr() + 4 * st0, scene_of=dev["local"].data_ptr() + 4 * a0,
                start=dev["s"].data_ptr() + 4 * a0 * ds.dof, goal=dev["g"].data_ptr() + 4 * a0 * ds.dof,
                waypoint=dev["w"].data_ptr() + 4 * a0 * ds.dof, n=n_b)
            P.prrtc_train_proposal(ctx, mid, rid, tb, lr, losses.data_ptr() + 4 * b, stream)
            a0 += n_b
            st0 += n_sb + 1
        l = losses.cpu().numpy()
        out.append(float(l.mean()))
        if log:
            log("  epoch %d: %d steps, mean NLL %.4f" % (ep, len(l), out[-1]))
    return np.asarray(out)


def mean_nll(P, ctx, torch, mid: int, rid: int, ds: Dataset, lo, hi) -> float:
    """Held-out mean NLL of the waypoints (mixture from the GPU forward pass;
    the log-sum-exp is evaluated here in FP64)."""
    if len(ds.scene_of) == 0:
        return float("nan")
    d = ds.dof
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in dict(
        vox=ds.vox, so=ds.scene_of, s=ds.start, g=ds.goal).items()}
    n = len(ds.scene_of)
    gmm = torch.zeros((n, N_COMP * (1 + 2 * d)), dtype=torch.float32, device="cuda")
    P.prrtc_proposal_forward(ctx, mid, rid, dev["vox"].data_ptr(), ds.vox.shape[0], dev["so"].data_ptr(),
                             dev["s"].data_ptr(), dev["g"].data_ptr(), n, gmm.data_ptr(),
                             torch.cuda.current_stream().cuda_stream)
    o = gmm.cpu().numpy().astype(np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    x = 2.0 * (ds.waypoint.astype(np.float64) - lo) / (hi - lo) - 1.0
    logits = o[:, :N_COMP]
    mu = o[:, N_COMP:N_COMP * (1 + d)].reshape(n, N_COMP, d)
    ls = o[:, N_COMP * (1 + d):].reshape(n, N_COMP, d)
    z = (x[:, None, :] - mu) * np.exp(-ls)
    a = logits - logits.max(1, keepdims=True)
    a = a - np.log(np.exp(a).sum(1, keepdims=True))
    a = a + np.sum(-0.5 * z * z - ls - 0.5 * math.log(2 * math.pi), axis=2)
    m = a.max(1, keepdims=True)
    return float(-(m[:, 0] + np.log(np.exp(a - m).sum(1))).mean())


SCREEN_SEED = 0x0A000000    # added to a query's seed for its screening runs


def compare(P, ctx, torch, mid: int, rid: int, robot: dict, n_scenes: int, base: int = SEED_EVAL,
            mix: float = 0.5, max_rounds: int = 1 << 30, budget_ms: float = 1000.0,
            screen_ms: float = 1000.0, log=None) -> dict:
    """Uniform against learned sampling on held-out scenes, one query each,
    same seed, round limit and time budget: wall time of the prrtc_plan call
    and success.

    Many generated queries have no solution at all (start and goal in
    different free regions of a crowded scene).  A screening pass first plans
    every query with both samplers under other seeds (one batched launch per
    sampler, screen_ms each); queries that neither solves are dropped, so the
    comparison runs on queries known to be solvable, chosen without favouring
    either sampler."""
    sids, queries = [], []
    for i in range(n_scenes):
        sid = P.prrtc_load_scene(ctx, scene(robot, i, base))
        q = free_query(P, ctx, torch, rid, sid, robot, base + i)
        if q is None:
            P.prrtc_unload_scene(ctx, sid)
            continue
        sids.append(sid)
        queries.append((i, q))
    solvable = np.zeros(len(queries), bool)
    for sampler in (0, 1):
        p = P.prrtc_plan_params_default()
        p.workers, p.tile, p.max_rounds, p.time_budget_ms = 64, 16, max_rounds, screen_ms
        p.sampler, p.model_id, p.mix = sampler, mid, mix
        batch = [(rid, sid, q[0], q[1], SCREEN_SEED + base + i, i) for sid, (i, q) in zip(sids, queries)]
        if batch:
            _, res = P.prrtc_plan_batch(ctx, batch, p)
            solvable |= np.array([r[0] == P.PRRTC_OK for r in res])
    if log:
        log("  screening: %d of %d free queries solvable" % (int(solvable.sum()), len(queries)))
    res = {"plain": [], "learned": []}
    for k, (sid, (i, q)) in enumerate(zip(sids, queries)):
        if not solvable[k]:
            continue
        for name, sampler in (("plain", 0), ("learned", 1)):
            p = P.prrtc_plan_params_default()
            p.seed, p.max_rounds, p.sampler, p.model_id, p.mix = base + i, max_rounds, sampler, mid, mix
            p.time_budget_ms = budget_ms
            t0 = time.perf_counter()
            st, _, stats = P.prrtc_plan(ctx, rid, sid, q[0], q[1], p)
            ms = (time.perf_counter() - t0) * 1e3
            res[name].append((st == P.PRRTC_OK, ms, stats["rounds"], stats["gpu_ms"]))
    for sid in sids:
        P.prrtc_unload_scene(ctx, sid)
    out = {"free_queries": len(queries), "solvable_queries": int(solvable.sum()), "time_budget_ms": budget_ms,
           "screen_ms": screen_ms}
    for name, rows in res.items():
        a = np.array(rows, np.float64).reshape(-1, 4)
        ok = a[:, 0] > 0
        t = np.where(ok, a[:, 1], np.inf)
        pct = {}
        for qq in (50, 90, 99):
            with np.errstate(invalid="ignore"):   # interpolating between two failures
                v = float(np.percentile(t, qq)) if len(t) else float("inf")
            pct["p%d_ms" % qq] = v if np.isfinite(v) else None
        out[name] = dict(queries=int(len(a)), success=float(ok.mean()) if len(a) else 0.0, **pct,
                         p50_rounds=float(np.median(a[ok, 2])) if ok.any() else None,
                         p50_gpu_ms=float(np.median(a[ok, 3])) if ok.any() else None)
        if log:
            log("  %s: %s" % (name, out[name]))
    return out


def main(argv=None):
    import argparse
    import sys
    import torch
    from . import prrtc as P
    from . import workloads as W
    ap = argparse.ArgumentParser(description="Generate data with the uniform planner, train the 7-DoF "
                                             "proposal, compare learned and uniform sampling")
    ap.add_argument("--scenes", type=int, default=10000)
    ap.add_argument("--eval-scenes", type=int, default=500)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--mix", type=float, default=0.5)
    ap.add_argument("--out", default=None, help="write the trained model blob here")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    robot = W.robot_r7()
    ctx = P.prrtc_create(0)
    rid = P.prrtc_load_robot(ctx, robot)
    t0 = time.perf_counter()
    ds = generate(P, ctx, torch, rid, robot, a.scenes, log=log)
    log("data: %d scenes solved, %d samples, %.1f s" % (ds.vox.shape[0], len(ds.scene_of), time.perf_counter() - t0))
    ev = generate(P, ctx, torch, rid, robot, a.eval_scenes, base=SEED_EVAL)
    mid = P.prrtc_load_proposal(ctx, pack(init_params(7, 1), 7))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = train(P, ctx, torch, mid, rid, ds, a.epochs, a.batch, a.lr, log=log)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("train: %.1f s, %.0f samples/s" % (dt, a.epochs * len(ds.scene_of) / dt))
    log("held-out NLL %.4f" % mean_nll(P, ctx, torch, mid, rid, ev, robot["q_lo"], robot["q_hi"]))
    compare(P, ctx, torch, mid, rid, robot, a.eval_scenes, mix=a.mix, log=log)
    if a.out:
        with open(a.out, "wb") as f:
            f.write(P.prrtc_save_proposal(ctx, mid))
    P.prrtc_destroy(ctx)



# ---- the dual-arm shelf: queries from the library's own FK and checks, training, comparison -----
def _valid_configs(P, ctx, torch, rid, sid, q):
    """uint8 [n]: each configuration collision-free (a zero-length edge)."""
    qd = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    ok = torch.zeros(qd.shape[0], dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, qd.data_ptr(), qd.data_ptr(), qd.shape[0], 32.0, ok.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    return ok.cpu().numpy().astype(bool)


def _valid_edges(P, ctx, torch, rid, sid, a, b):
    ad = torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    bd = torch.from_numpy(np.ascontiguousarray(b, np.float32)).cuda()
    ok = torch.zeros(ad.shape[0], dtype=torch.uint8, device="cuda")
    P.prrtc_check_edges(ctx, rid, sid, ad.data_ptr(), bd.data_ptr(), ad.shape[0], 32.0, ok.data_ptr(),
                        torch.cuda.current_stream().cuda_stream)
    return ok.cpu().numpy().astype(bool)


def _fk(P, ctx, torch, rid, q, n_spheres):
    """Sphere centres [n][n_spheres][3] (device tensor) from the library's FK."""
    qd = torch.from_numpy(np.ascontiguousarray(q, np.float32)).cuda()
    xyz = torch.zeros((qd.shape[0], n_spheres, 3), dtype=torch.float32, device="cuda")
    P.prrtc_fk_spheres(ctx, rid, qd.data_ptr(), qd.shape[0], xyz.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return xyz


def _front(P, ctx, torch, rid, q, n_spheres):
    """Every sphere in front of the shelf (x < 0.4 m)?"""
    return (_fk(P, ctx, torch, rid, q, n_spheres)[..., 0].amax(1) < 0.4).cpu().numpy()


def _arm_goals(P, ctx, torch, rid, sid, robot, arm, rng, want, max_batches, parked):
    """Goals of one arm, with the other arm parked at collision-free start
    configurations (rows of `parked`): the hand-bar centre in a shelf cell on
    the arm's side and the configuration collision-free; kept if also
    collision-free together with 16 random 0.05 rad moves of the arm (room
    around the hand) and with a straight retreat of 0.5-2 rad that reaches
    the front of the shelf collision-free.  Uniform sampling finds few such
    poses (about 1 in 2000), so accepted and in-cell poses also seed random
    walks (steps of 0.15 rad in the arm's joints)."""
    from . import workloads as W
    lo, hi = robot["q_lo"].astype(np.float64), robot["q_hi"].astype(np.float64)
    dof = lo.shape[0]
    n_sph = robot["sphere_xyzr"].shape[0]
    j0, j1 = 7 * arm, 7 * arm + 7
    hand = np.arange(n_sph // 2)[W.HAND_SPHERES] + (n_sph // 2) * arm
    cells = W.shelf_cells()
    inset = W.SHELF_WALL / 2 + W.SHELF_MARGIN
    c_lo = np.array([c[0] + inset for c in cells])
    c_hi = np.array([c[1] - inset for c in cells])
    side = np.array([(c[1][1] <= 1e-9) if arm == 0 else (c[0][1] >= -1e-9) for c in cells])
    hand_t = torch.from_numpy(hand).cuda()

    def in_cell_valid(q):
        h = _fk(P, ctx, torch, rid, q, n_sph).index_select(1, hand_t).mean(1).cpu().numpy()
        ok = np.any(np.all((h[:, None, :] >= c_lo[None]) & (h[:, None, :] <= c_hi[None]), axis=2) & side[None], axis=1)
        idx = np.nonzero(ok)[0]
        if len(idx):
            idx = idx[_valid_configs(P, ctx, torch, rid, sid, q[idx])]
        return q[idx]

    def roomy(gs):
        """Which of the candidate goals gs [m][dof] have room and a retreat
        (three batched library calls for all of them)."""
        m = len(gs)
        d = np.zeros((m, 16, dof))
        d[:, :, j0:j1] = rng.standard_normal((m, 16, 7))
        d *= 0.05 / np.linalg.norm(d, axis=2, keepdims=True)
        moves = np.clip(gs[:, None] + d, lo, hi).astype(np.float32).reshape(-1, dof)
        ok = _valid_edges(P, ctx, torch, rid, sid, np.repeat(gs, 16, 0), moves).reshape(m, 16).all(1)
        d = np.zeros((m, 32, dof))
        d[:, :, j0:j1] = rng.standard_normal((m, 32, 7))
        d /= np.linalg.norm(d, axis=2, keepdims=True)
        back = np.clip(gs[:, None] + rng.uniform(0.5, 2.0, (m, 32, 1)) * d, lo, hi).astype(np.float32).reshape(-1, dof)
        fr = _front(P, ctx, torch, rid, back, n_sph)
        esc = fr & _valid_edges(P, ctx, torch, rid, sid, np.repeat(gs, 32, 0), back)
        return ok & esc.reshape(m, 32).any(1)

    seeds, out = [], []
    for _ in range(max_batches):
        if len(out) >= want:
            break
        if len(seeds) < 8:
            q = parked[rng.integers(0, len(parked), 16384)].astype(np.float32)
            q[:, j0:j1] = rng.uniform(lo[j0:j1], hi[j0:j1], (16384, 7))
        else:
            base = np.array(seeds, np.float32)[rng.integers(0, len(seeds), 4096)]
            q = base.copy()
            q[:, j0:j1] = np.clip(base[:, j0:j1] + rng.normal(0.0, 0.15, (4096, 7)), lo[j0:j1], hi[j0:j1])
        found = in_cell_valid(q)
        seeds.extend(list(found[:256]))
        if len(found):
            keep = found[:256][roomy(found[:256])]
            out.extend(list(keep[:, j0:j1]))
    return np.array(out[:want], np.float32).reshape(-1, 7)


def shelf_queries(P, ctx, torch, rid, sid, robot, n, seed, max_batches=200, log=None):
    """Dual-arm shelf queries built with the library's FK and collision checks
    (training data; the stored benchmark queries come from the oracle): each
    arm's goal as in _arm_goals, the two combined and checked together;
    start uniform, collision-free, every sphere in front of the shelf.  At
    most max_batches sampling rounds per arm, so fewer than n queries may
    come back."""
    rng = np.random.default_rng(seed)
    lo, hi = robot["q_lo"].astype(np.float64), robot["q_hi"].astype(np.float64)
    dof = lo.shape[0]
    n_sph = robot["sphere_xyzr"].shape[0]
    starts = []
    for _ in range(max_batches):
        if len(starts) >= n:
            break
        q = rng.uniform(lo, hi, (8192, dof)).astype(np.float32)
        cand = q[_front(P, ctx, torch, rid, q, n_sph)]
        if len(cand):
            cand = cand[_valid_configs(P, ctx, torch, rid, sid, cand)]
        starts.extend(list(cand[:n - len(starts)]))
    starts = np.array(starts, np.float32).reshape(-1, dof)
    if not len(starts):
        return starts, starts
    ga = _arm_goals(P, ctx, torch, rid, sid, robot, 0, rng, n, max_batches, starts)
    if log:
        log("  shelf goals, arm 0: %d" % len(ga))
    gb = _arm_goals(P, ctx, torch, rid, sid, robot, 1, rng, n, max_batches, starts)
    m = min(len(ga), len(gb))
    goals = np.concatenate([ga[:m], gb[:m]], axis=1).astype(np.float32)
    if m:
        goals = goals[_valid_configs(P, ctx, torch, rid, sid, goals)]
    if log:
        log("  shelf goals: arm 0 %d, arm 1 %d, together %d" % (len(ga), len(gb), len(goals)))
    k = min(len(starts), len(goals))
    return np.array(starts[:k], np.float32).reshape(-1, dof), goals[:k]


def shelf_dataset(P, ctx, torch, rid, sid, starts, goals, vox_row, workers=64, budget_ms=1000.0, seed=0x57000000,
                  tail=1.0):
    """Solve the queries with the uniform planner in one batched launch and
    keep the paths' waypoints every 0.25 rad; one voxel row per query (the
    scene is shared)."""
    prm = P.prrtc_plan_params_default()
    prm.workers, prm.tile, prm.max_rounds, prm.time_budget_ms = workers, 16, 1 << 30, budget_ms
    qs = [(rid, sid, s, g, seed + k, 0) for k, (s, g) in enumerate(zip(starts, goals))]
    _, out = P.prrtc_plan_batch(ctx, qs, prm, path_cap=512)
    ds = Dataset(starts.shape[1])
    for (st, path, _), s, g in zip(out, starts, goals):
        if st != P.PRRTC_OK:
            continue
        k = len(ds.vox)
        ds.vox.append(vox_row)
        ds.queries.append((s, g))
        ds.paths.append(path)
        for w in resample_path(path, tail=tail):
            ds.scene_of.append(k)
            ds.start.append(s)
            ds.goal.append(g)
            ds.waypoint.append(w)
    return ds.finish()


if __name__ == "__main__":
    main()
