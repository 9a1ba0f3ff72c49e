"""Thin ctypes binding of libprrtc.so (argument marshalling only).

Every function keeps the C name and argument order of include/prrtc.h.
Device buffers are passed as integer device addresses (e.g. a torch tensor's
``data_ptr()``); torch is used by callers only to own device memory and
streams.  There is no fallback: if the HIP library is missing, importing this
module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PRRTC_LIB may name another build of the same library (same ABI)
LIB_PATH = os.environ.get("PRRTC_LIB") or os.path.join(_HERE, "libprrtc.so")

PRRTC_OK = 0
PRRTC_E_ARG = -1
PRRTC_E_STATE = -2
PRRTC_E_CAPACITY = -3
PRRTC_E_INVALID_ENDPOINT = -4
PRRTC_E_NO_SOLUTION = -5
PRRTC_E_BUSY = -6
PRRTC_E_HIP = -7

MAX_DOF = 16

# hipStreamLegacy: the null stream named explicitly (a NULL stream argument
# means the context's own stream)
HIP_STREAM_LEGACY = 1


def _stream(stream: int | None):
    """A stream argument: None -> NULL (the context's stream); 0, the handle
    torch reports for its default (null) stream -> hipStreamLegacy, so the
    call is ordered with torch's work on that stream; other handles as given."""
    if stream is None:
        return None
    return HIP_STREAM_LEGACY if int(stream) == 0 else int(stream)


class prrtc_robot_desc(C.Structure):
    _fields_ = [
        ("n_chains", C.c_int32),
        ("chain_dof", C.c_int32 * 2),
        ("base_pose", (C.c_float * 12) * 2),
        ("dh", C.POINTER(C.c_float)),
        ("q_lo", C.POINTER(C.c_float)),
        ("q_hi", C.POINTER(C.c_float)),
        ("n_spheres", C.c_int32),
        ("sphere_frame", C.POINTER(C.c_int32)),
        ("sphere_xyzr", C.POINTER(C.c_float)),
        ("n_self_pairs", C.c_int32),
        ("self_pairs", C.POINTER(C.c_int32)),
        ("n_coarse", C.c_int32),
        ("coarse_frame", C.POINTER(C.c_int32)),
        ("coarse_xyzr", C.POINTER(C.c_float)),
        ("sphere_coarse", C.POINTER(C.c_int32)),
    ]


class prrtc_plan_params(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("query", C.c_uint32),
        ("workers", C.c_int32),
        ("delta", C.c_float),
        ("res", C.c_float),
        ("max_rounds", C.c_int32),
        ("tree_capacity", C.c_int32),
        ("time_budget_ms", C.c_float),
        ("validate_factor", C.c_int32),
        ("dds_radius", C.c_float),
        ("dds_tries", C.c_int32),
        ("sampler", C.c_int32),
        ("model_id", C.c_int32),
        ("mix", C.c_float),
        ("tile", C.c_int32),
    ]


class prrtc_plan_stats(C.Structure):
    _fields_ = [
        ("rounds", C.c_int32),
        ("nodes_a", C.c_int32),
        ("nodes_b", C.c_int32),
        ("edges_checked", C.c_int64),
        ("validation_failures", C.c_int32),
        ("connect_worker", C.c_int32),
        ("gpu_ms", C.c_float),
        ("fallback", C.c_int32),
        ("pad", C.c_int32),
        ("learned_samples", C.c_int64),
    ]


class prrtc_query(C.Structure):
    _fields_ = [
        ("robot_id", C.c_int32),
        ("scene_id", C.c_int32),
        ("start", C.c_float * 16),
        ("goal", C.c_float * 16),
        ("seed", C.c_uint64),
        ("query", C.c_uint32),
        ("model_id", C.c_int32),
    ]


class prrtc_query_result(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("path_len", C.c_int32),
        ("stats", prrtc_plan_stats),
    ]


class prrtc_esdf_desc(C.Structure):
    _fields_ = [
        ("origin", C.c_float * 3),
        ("voxel", C.c_float),
        ("dims", C.c_int32 * 3),
        ("values", C.c_void_p),
    ]


class prrtc_train_batch(C.Structure):
    _fields_ = [
        ("vox", C.c_void_p),
        ("n_scenes", C.c_int32),
        ("scene_start", C.c_void_p),
        ("scene_of", C.c_void_p),
        ("start", C.c_void_p),
        ("goal", C.c_void_p),
        ("waypoint", C.c_void_p),
        ("n", C.c_int32),
    ]


class PrrtcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"prrtc status {status}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2503_06757_amd/build.py "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, F, VP = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_void_p
    L.prrtc_create.argtypes = [C.POINTER(P), C.c_int]
    L.prrtc_create.restype = I32
    L.prrtc_destroy.argtypes = [P]
    L.prrtc_destroy.restype = None
    L.prrtc_last_error.argtypes = [P]
    L.prrtc_last_error.restype = C.c_char_p
    L.prrtc_load_robot.argtypes = [P, C.POINTER(prrtc_robot_desc), C.POINTER(I32)]
    L.prrtc_load_robot.restype = I32
    L.prrtc_load_scene.argtypes = [P, VP, I32, C.POINTER(I32)]
    L.prrtc_load_scene.restype = I32
    L.prrtc_unload_scene.argtypes = [P, I32]
    L.prrtc_unload_scene.restype = I32
    L.prrtc_scene_set_esdf.argtypes = [P, I32, C.POINTER(prrtc_esdf_desc)]
    L.prrtc_scene_set_esdf.restype = I32
    L.prrtc_esdf_from_scene.argtypes = [P, I32, VP, F, VP, VP, VP]
    L.prrtc_esdf_from_scene.restype = I32
    L.prrtc_check_edges.argtypes = [P, I32, I32, VP, VP, I64, F, VP, VP]
    L.prrtc_check_edges.restype = I32
    L.prrtc_edge_schedule.argtypes = [P, I32, I32, I32, C.POINTER(I32)]
    L.prrtc_edge_schedule.restype = I32
    L.prrtc_fk_spheres.argtypes = [P, I32, VP, I64, VP, VP]
    L.prrtc_fk_spheres.restype = I32
    L.prrtc_load_proposal.argtypes = [P, VP, C.c_size_t, C.POINTER(I32)]
    L.prrtc_load_proposal.restype = I32
    L.prrtc_save_proposal.argtypes = [P, I32, VP, C.c_size_t, C.POINTER(C.c_size_t)]
    L.prrtc_save_proposal.restype = I32
    L.prrtc_voxelize.argtypes = [P, I32, VP, VP]
    L.prrtc_voxelize.restype = I32
    L.prrtc_proposal_forward.argtypes = [P, I32, I32, VP, I32, VP, VP, VP, I32, VP, VP]
    L.prrtc_proposal_forward.restype = I32
    L.prrtc_proposal_forward_noalloc.argtypes = [P, I32, I32, VP, I32, VP, VP, VP, I32, VP, VP]
    L.prrtc_proposal_forward_noalloc.restype = I32
    L.prrtc_train_proposal.argtypes = [P, I32, I32, C.POINTER(prrtc_train_batch), F, VP, VP]
    L.prrtc_train_proposal.restype = I32
    L.prrtc_proposal_sample.argtypes = [P, I32, VP, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, I32, VP, VP,
                                        VP]
    L.prrtc_proposal_sample.restype = I32
    L.prrtc_tuned_launch.argtypes = [P, C.POINTER(prrtc_query), I32, VP, I32, VP, I32, C.POINTER(I32),
                                     C.POINTER(I32)]
    L.prrtc_tuned_launch.restype = I32
    L.prrtc_tuning_save.argtypes = [P, C.c_char_p]
    L.prrtc_tuning_save.restype = I32
    L.prrtc_tuning_load.argtypes = [P, C.c_char_p]
    L.prrtc_tuning_load.restype = I32
    if hasattr(L, "prrtc_plan"):
        L.prrtc_plan_params_default.argtypes = [C.POINTER(prrtc_plan_params)]
        L.prrtc_plan_params_default.restype = None
        L.prrtc_plan.argtypes = [P, I32, I32, VP, VP, C.POINTER(prrtc_plan_params), VP, I32,
                                 C.POINTER(I32), C.POINTER(prrtc_plan_stats)]
        L.prrtc_plan.restype = I32
        L.prrtc_plan_batch.argtypes = [P, C.POINTER(prrtc_query), I32, C.POINTER(prrtc_plan_params), I32, I64,
                                       VP, I32, C.POINTER(prrtc_query_result), C.POINTER(I32)]
        L.prrtc_plan_batch.restype = I32
        L.prrtc_tune_launch.argtypes = [P, C.POINTER(prrtc_query), I32, C.POINTER(prrtc_plan_params), VP, I32, VP,
                                        I32, I64, VP, C.POINTER(I32), C.POINTER(I32)]
        L.prrtc_tune_launch.restype = I32
        L.prrtc_serve_start.argtypes = [P, C.POINTER(prrtc_plan_params), I32, I32, I64, I32]
        L.prrtc_serve_start.restype = I32
        L.prrtc_submit.argtypes = [P, C.POINTER(prrtc_query), C.POINTER(C.c_uint64)]
        L.prrtc_submit.restype = I32
        L.prrtc_poll.argtypes = [P, C.c_uint64, C.POINTER(prrtc_query_result), VP, I32]
        L.prrtc_poll.restype = I32
        L.prrtc_serve_stop.argtypes = [P, C.POINTER(I64)]
        L.prrtc_serve_stop.restype = I32
    return L


lib = _load()

# the symbols include/prrtc.h declares (checked by the CPU test-suite)
EXPORTED = ("prrtc_create", "prrtc_destroy", "prrtc_last_error", "prrtc_load_robot",
            "prrtc_load_scene", "prrtc_unload_scene", "prrtc_scene_set_esdf", "prrtc_esdf_from_scene",
            "prrtc_check_edges", "prrtc_edge_schedule", "prrtc_fk_spheres",
            "prrtc_plan_params_default", "prrtc_plan", "prrtc_plan_batch", "prrtc_tune_launch",
            "prrtc_tuned_launch", "prrtc_tuning_save", "prrtc_tuning_load",
            "prrtc_serve_start", "prrtc_submit", "prrtc_poll", "prrtc_serve_stop", "prrtc_load_proposal", "prrtc_save_proposal",
            "prrtc_voxelize", "prrtc_proposal_forward", "prrtc_proposal_forward_noalloc", "prrtc_proposal_sample",
            "prrtc_train_proposal")


# ---- C-named wrappers ------------------------------------------------------------
def prrtc_create(device: int = 0) -> int:
    h = C.c_void_p()
    st = lib.prrtc_create(C.byref(h), int(device))
    if st != PRRTC_OK:
        raise PrrtcError(st, "prrtc_create failed")
    return h.value


def prrtc_destroy(ctx: int) -> None:
    lib.prrtc_destroy(ctx)


def prrtc_last_error(ctx: int) -> str:
    return lib.prrtc_last_error(ctx).decode()


def _check(ctx, st):
    if st != PRRTC_OK:
        raise PrrtcError(st, prrtc_last_error(ctx))
    return st


def robot_desc(robot: dict):
    """Build a prrtc_robot_desc from a workload dict; returns (desc, keepalive)."""
    keep = dict(
        dh=np.ascontiguousarray(robot["dh"], np.float32),
        lo=np.ascontiguousarray(robot["q_lo"], np.float32),
        hi=np.ascontiguousarray(robot["q_hi"], np.float32),
        frame=np.ascontiguousarray(robot["sphere_frame"], np.int32),
        xyzr=np.ascontiguousarray(robot["sphere_xyzr"], np.float32),
        pairs=np.ascontiguousarray(robot["self_pairs"], np.int32).reshape(-1, 2),
    )
    d = prrtc_robot_desc()
    d.n_chains = int(robot["n_chains"])
    for c in range(d.n_chains):
        d.chain_dof[c] = int(robot["chain_dof"][c])
        for i in range(12):
            d.base_pose[c][i] = float(robot["base_pose"][c][i])
    fp = C.POINTER(C.c_float)
    ip = C.POINTER(C.c_int32)
    d.dh = keep["dh"].ctypes.data_as(fp)
    d.q_lo = keep["lo"].ctypes.data_as(fp)
    d.q_hi = keep["hi"].ctypes.data_as(fp)
    d.n_spheres = keep["xyzr"].shape[0]
    d.sphere_frame = keep["frame"].ctypes.data_as(ip)
    d.sphere_xyzr = keep["xyzr"].ctypes.data_as(fp)
    d.n_self_pairs = keep["pairs"].shape[0]
    d.self_pairs = keep["pairs"].ctypes.data_as(ip)
    if "coarse_xyzr" in robot:     # two-stage checks
        keep["cframe"] = np.ascontiguousarray(robot["coarse_frame"], np.int32)
        keep["cxyzr"] = np.ascontiguousarray(robot["coarse_xyzr"], np.float32)
        keep["owner"] = np.ascontiguousarray(robot["sphere_coarse"], np.int32)
        d.n_coarse = keep["cxyzr"].shape[0]
        d.coarse_frame = keep["cframe"].ctypes.data_as(ip)
        d.coarse_xyzr = keep["cxyzr"].ctypes.data_as(fp)
        d.sphere_coarse = keep["owner"].ctypes.data_as(ip)
    return d, keep


def prrtc_load_robot(ctx: int, robot: dict) -> int:
    d, keep = robot_desc(robot)
    rid = C.c_int32(-1)
    _check(ctx, lib.prrtc_load_robot(ctx, C.byref(d), C.byref(rid)))
    del keep
    return rid.value


def prrtc_load_scene(ctx: int, prims: np.ndarray) -> int:
    prims = np.ascontiguousarray(prims)
    assert prims.dtype.itemsize == 64
    sid = C.c_int32(-1)
    _check(ctx, lib.prrtc_load_scene(ctx, prims.ctypes.data if prims.size else None,
                                     int(prims.shape[0]), C.byref(sid)))
    return sid.value


def prrtc_unload_scene(ctx: int, scene_id: int) -> None:
    _check(ctx, lib.prrtc_unload_scene(ctx, int(scene_id)))


def prrtc_scene_set_esdf(ctx: int, scene_id: int, origin=None, voxel: float = 0.0, values=None) -> None:
    """Attach an ESDF grid: values float32 [nz][ny][nx] (x fastest) at
    origin + voxel (i, j, k); origin None detaches the scene's grid."""
    if origin is None:
        _check(ctx, lib.prrtc_scene_set_esdf(ctx, int(scene_id), None))
        return
    v = np.ascontiguousarray(values, np.float32)
    nz, ny, nx = v.shape
    d = prrtc_esdf_desc((C.c_float * 3)(*[float(x) for x in origin]), float(voxel), (C.c_int32 * 3)(nx, ny, nz),
                        v.ctypes.data)
    _check(ctx, lib.prrtc_scene_set_esdf(ctx, int(scene_id), C.byref(d)))


def prrtc_esdf_from_scene(ctx: int, scene_id: int, origin, voxel: float, dims, values_dev: int,
                          stream: int | None = None) -> None:
    o = np.ascontiguousarray(origin, np.float32)
    d = np.ascontiguousarray(dims, np.int32)
    _check(ctx, lib.prrtc_esdf_from_scene(ctx, int(scene_id), o.ctypes.data, float(voxel), d.ctypes.data,
                                          values_dev, _stream(stream)))


def prrtc_check_edges(ctx: int, robot_id: int, scene_id: int, a_dev: int, b_dev: int, n_edges: int,
                      res: float, valid_dev: int, stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_check_edges(ctx, robot_id, scene_id, a_dev, b_dev, int(n_edges),
                                             float(res), valid_dev, _stream(stream)))


def prrtc_edge_schedule(ctx: int, robot_id: int, scene_id: int, set: int = -2) -> int:
    """Pin (0/1), forget (-1) or only read (-2) the check_edges schedule of a
    (robot, scene) pair; returns the schedule in force (-1: none chosen)."""
    out = C.c_int32(0)
    _check(ctx, lib.prrtc_edge_schedule(ctx, int(robot_id), int(scene_id), int(set), C.byref(out)))
    return out.value


def prrtc_fk_spheres(ctx: int, robot_id: int, q_dev: int, n: int, xyz_dev: int,
                     stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_fk_spheres(ctx, robot_id, q_dev, int(n), xyz_dev, _stream(stream)))


def prrtc_plan_params_default() -> prrtc_plan_params:
    p = prrtc_plan_params()
    lib.prrtc_plan_params_default(C.byref(p))
    return p


def prrtc_plan(ctx: int, robot_id: int, scene_id: int, start: np.ndarray, goal: np.ndarray,
               params: prrtc_plan_params, path_cap: int = 4096):
    """Returns (status, path ndarray (len, dof) or None, stats).  Status codes
    E_NO_SOLUTION / E_INVALID_ENDPOINT are returned, not raised."""
    s = np.ascontiguousarray(start, np.float32)
    g = np.ascontiguousarray(goal, np.float32)
    path = np.zeros((path_cap, s.shape[0]), np.float32)
    ln = C.c_int32(0)
    st = prrtc_plan_stats()
    status = lib.prrtc_plan(ctx, robot_id, scene_id, s.ctypes.data, g.ctypes.data, C.byref(params),
                            path.ctypes.data, int(path_cap), C.byref(ln), C.byref(st))
    if status in (PRRTC_E_ARG, PRRTC_E_STATE, PRRTC_E_HIP):
        raise PrrtcError(status, prrtc_last_error(ctx))
    stats = {f: getattr(st, f) for f, _ in prrtc_plan_stats._fields_}
    stats["path_len"] = ln.value
    return status, (path[: ln.value].copy() if status == PRRTC_OK else None), stats


_QUERY_DT = np.dtype(prrtc_query)
_RESULT_DT = np.dtype(prrtc_query_result)


def prrtc_plan_batch(ctx: int, queries, params, groups: int = 0, memory_budget: int = 0, path_cap: int = 256):
    """queries: list of (robot_id, scene_id, start, goal, seed, query[, model_id]).
    Returns (groups used, [(status, path or None, stats dict)])."""
    n = len(queries)
    arr = _query_array(queries)
    paths = np.zeros((max(n, 1), path_cap, 16), np.float32)
    res = np.zeros(max(n, 1), _RESULT_DT)
    used = C.c_int32(0)
    _check(ctx, lib.prrtc_plan_batch(ctx, arr.ctypes.data_as(C.POINTER(prrtc_query)), n, C.byref(params),
                                     int(groups), int(memory_budget), paths.ctypes.data, int(path_cap),
                                     res.ctypes.data_as(C.POINTER(prrtc_query_result)), C.byref(used)))
    out = []
    names = [f for f, _ in prrtc_plan_stats._fields_]
    for k, q in enumerate(queries):
        r = res[k]
        dof = len(q[2])
        stats = {f: r["stats"][f].item() for f in names}
        stats["path_len"] = int(r["path_len"])
        path = None
        st = int(r["status"])
        if st == PRRTC_OK:
            path = paths[k].reshape(-1)[: stats["path_len"] * dof].reshape(-1, dof).copy()
        out.append((st, path, stats))
    return used.value, out


def _query_array(queries):
    n = len(queries)
    arr = np.zeros(max(n, 1), _QUERY_DT)
    if n:
        arr["robot_id"][:n] = [q[0] for q in queries]
        arr["scene_id"][:n] = [q[1] for q in queries]
        arr["seed"][:n] = [q[4] for q in queries]
        arr["query"][:n] = [q[5] for q in queries]
        arr["model_id"][:n] = [q[6] if len(q) > 6 else -1 for q in queries]
        for k, q in enumerate(queries):
            d = len(q[2])
            arr["start"][k, :d] = q[2]
            arr["goal"][k, :d] = q[3]
    return arr


def prrtc_tune_launch(ctx: int, queries, params, workers=(16, 32, 64, 128, 256), tiles=(16, 64),
                      memory_budget: int = 0):
    """((best workers, best tile), {(workers, tile): queries/s})."""
    arr = _query_array(queries)
    wk = np.asarray(workers, np.int32)
    tl = np.asarray(tiles, np.int32)
    rates = np.zeros((len(wk), len(tl)), np.float32)
    bw, bt = C.c_int32(0), C.c_int32(0)
    _check(ctx, lib.prrtc_tune_launch(ctx, arr.ctypes.data_as(C.POINTER(prrtc_query)), len(queries),
                                      C.byref(params), wk.ctypes.data, len(wk), tl.ctypes.data, len(tl),
                                      int(memory_budget), rates.ctypes.data, C.byref(bw), C.byref(bt)))
    return (bw.value, bt.value), {(int(w), int(t)): float(rates[i, j]) for i, w in enumerate(wk)
                                  for j, t in enumerate(tl)}


def prrtc_tuned_launch(ctx: int, queries, workers=(16, 32, 64, 128, 256), tiles=(16, 64)):
    """(workers, tile) stored by prrtc_tune_launch for these queries and
    candidates, or None without a record."""
    arr = _query_array(queries)
    wk = np.asarray(workers, np.int32)
    tl = np.asarray(tiles, np.int32)
    bw, bt = C.c_int32(0), C.c_int32(0)
    st = lib.prrtc_tuned_launch(ctx, arr.ctypes.data_as(C.POINTER(prrtc_query)), len(queries), wk.ctypes.data,
                                len(wk), tl.ctypes.data, len(tl), C.byref(bw), C.byref(bt))
    if st == PRRTC_E_STATE:
        return None
    _check(ctx, st)
    return bw.value, bt.value


def prrtc_tuning_save(ctx: int, path: str) -> None:
    _check(ctx, lib.prrtc_tuning_save(ctx, os.fsencode(path)))


def prrtc_tuning_load(ctx: int, path: str) -> None:
    _check(ctx, lib.prrtc_tuning_load(ctx, os.fsencode(path)))


def prrtc_serve_start(ctx: int, params, slots: int = 256, max_pending: int = 1024, memory_budget: int = 0,
                      path_cap: int = 256) -> None:
    _check(ctx, lib.prrtc_serve_start(ctx, C.byref(params), int(slots), int(max_pending), int(memory_budget),
                                      int(path_cap)))


def prrtc_submit(ctx: int, robot_id: int, scene_id: int, start, goal, seed: int, query: int = 0,
                 model_id: int = -1):
    """Ticket, or None when admission is refused (E_BUSY)."""
    q = prrtc_query()
    q.robot_id, q.scene_id, q.seed, q.query = int(robot_id), int(scene_id), int(seed), int(query)
    q.model_id = int(model_id)
    for j, v in enumerate(np.asarray(start, np.float32)):
        q.start[j] = float(v)
    for j, v in enumerate(np.asarray(goal, np.float32)):
        q.goal[j] = float(v)
    t = C.c_uint64(0)
    st = lib.prrtc_submit(ctx, C.byref(q), C.byref(t))
    if st == PRRTC_E_BUSY:
        return None
    if st != PRRTC_OK:   # the serving thread owns the error text: not read here
        raise PrrtcError(st, "prrtc_submit refused")
    return t.value


def prrtc_poll(ctx: int, ticket: int, dof: int, path_cap: int = 256):
    """None while the query is queued or running, else (status, path or None, stats)."""
    r = prrtc_query_result()
    path = np.zeros((path_cap, dof), np.float32)
    st = lib.prrtc_poll(ctx, int(ticket), C.byref(r), path.ctypes.data, int(path_cap))
    if st == PRRTC_E_BUSY:
        return None
    if st != PRRTC_OK:
        raise PrrtcError(st, "prrtc_poll failed")
    stats = {f: getattr(r.stats, f) for f, _ in prrtc_plan_stats._fields_}
    stats["path_len"] = r.path_len
    return r.status, (path[: r.path_len].copy() if r.status == PRRTC_OK else None), stats


def prrtc_serve_stop(ctx: int) -> int:
    n = C.c_int64(0)
    _check(ctx, lib.prrtc_serve_stop(ctx, C.byref(n)))
    return n.value


# ---- learned proposal ---------------------------------------------------------------
def prrtc_load_proposal(ctx: int, blob: bytes) -> int:
    buf = C.create_string_buffer(bytes(blob), len(blob))
    mid = C.c_int32(-1)
    _check(ctx, lib.prrtc_load_proposal(ctx, C.cast(buf, C.c_void_p), len(blob), C.byref(mid)))
    return mid.value


def prrtc_save_proposal(ctx: int, model_id: int) -> bytes:
    need = C.c_size_t(0)
    st = lib.prrtc_save_proposal(ctx, model_id, None, 0, C.byref(need))
    if st != PRRTC_E_CAPACITY:
        _check(ctx, st)
    buf = C.create_string_buffer(need.value)
    _check(ctx, lib.prrtc_save_proposal(ctx, model_id, C.cast(buf, C.c_void_p), need.value, C.byref(need)))
    return buf.raw[: need.value]


def prrtc_voxelize(ctx: int, scene_id: int, vox_dev: int, stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_voxelize(ctx, scene_id, vox_dev, _stream(stream)))


def prrtc_proposal_forward(ctx: int, model_id: int, robot_id: int, vox_dev: int, n_scenes: int,
                           scene_of_dev: int, start_dev: int, goal_dev: int, n: int, gmm_dev: int,
                           stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_proposal_forward(ctx, model_id, robot_id, vox_dev, n_scenes, scene_of_dev,
                                                  start_dev, goal_dev, n, gmm_dev, _stream(stream)))


def prrtc_proposal_forward_noalloc(ctx: int, model_id: int, robot_id: int, vox_dev: int, n_scenes: int,
                                   scene_of_dev: int, start_dev: int, goal_dev: int, n: int, gmm_dev: int,
                                   stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_proposal_forward_noalloc(ctx, model_id, robot_id, vox_dev, n_scenes, scene_of_dev,
                                                          start_dev, goal_dev, n, gmm_dev, _stream(stream)))


def prrtc_train_proposal(ctx: int, model_id: int, robot_id: int, batch: prrtc_train_batch, lr: float,
                         loss_dev: int, stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_train_proposal(ctx, model_id, robot_id, C.byref(batch), float(lr), loss_dev,
                                                _stream(stream)))


def prrtc_proposal_sample(ctx: int, robot_id: int, gmm_dev: int, seed: int, query: int, rnd: int, attempt: int,
                          n: int, q_dev: int, inside_dev: int, stream: int | None = None) -> int:
    return _check(ctx, lib.prrtc_proposal_sample(ctx, robot_id, gmm_dev, int(seed), int(query), int(rnd),
                                                 int(attempt), int(n), q_dev, inside_dev, _stream(stream)))
