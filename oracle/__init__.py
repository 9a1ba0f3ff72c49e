"""ctypes front end of the serial C oracle (``prrtc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the product package never imports
it.  Shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "prrtc_oracle.c")
# ORACLE_LIB may name another build of the same source (e.g. with sanitizers)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

FLAG_BAND = 1e-5
MAX_DOF = 16


def build(force: bool = True, out: str | None = None, extra=()) -> str:
    """Compile liboracle.so with gcc (FP contraction off, OpenMP on); `out`
    and `extra` flags build another copy (e.g. with sanitizers)."""
    out = out or _LIB
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fopenmp", "-shared",
               "-fPIC", *extra, "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(out + ".tmp", out)
    return out


class Robot(C.Structure):
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
    ]


class PlanParams(C.Structure):
    _fields_ = [
        ("seed", C.c_uint64),
        ("query", C.c_uint32),
        ("workers", C.c_int32),
        ("delta", C.c_float),
        ("res", C.c_float),
        ("max_rounds", C.c_int32),
        ("tree_capacity", C.c_int32),
        ("validate_factor", C.c_int32),
        ("dds_radius", C.c_float),
        ("dds_tries", C.c_int32),
        ("sampler", C.c_int32),
    ]


class Esdf(C.Structure):
    _fields_ = [
        ("origin", C.c_float * 3),
        ("voxel", C.c_float),
        ("dims", C.c_int32 * 3),
        ("values", C.c_void_p),
    ]


class TreeDump(C.Structure):
    _fields_ = [
        ("nodes_a", C.c_void_p),
        ("nodes_b", C.c_void_p),
        ("parent_a", C.c_void_p),
        ("parent_b", C.c_void_p),
        ("blocked_a", C.c_void_p),
        ("blocked_b", C.c_void_p),
    ]


class PlanStats(C.Structure):
    _fields_ = [
        ("rounds", C.c_int32),
        ("nodes_a", C.c_int32),
        ("nodes_b", C.c_int32),
        ("edges_checked", C.c_int64),
        ("flagged_edges", C.c_int32),
        ("validation_failures", C.c_int32),
        ("connect_worker", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_dof.argtypes = [P]
        L.orc_n_frames.argtypes = [P]
        L.orc_fk_frames.argtypes = [P, P, P]
        L.orc_fk_spheres.argtypes = [P, P, P]
        L.orc_fk_spheres_batch.argtypes = [P, P, C.c_int64, P, C.c_int32]
        L.orc_fk_spheres_batch.restype = None
        L.orc_esdf_attach.argtypes = [P]
        L.orc_esdf_attach.restype = None
        L.orc_esdf_value.argtypes = [P, P]
        L.orc_esdf_value.restype = C.c_double
        L.orc_esdf_from_prims.argtypes = [P, C.c_int32, P, C.c_float, P, P, C.c_int32]
        L.orc_esdf_from_prims.restype = None
        L.orc_radical_inverse.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_radical_inverse.restype = C.c_float
        L.orc_halton_config.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                        C.c_uint32, P, P, C.c_int32, P]
        L.orc_halton_config.restype = None
        L.orc_clearance.argtypes = [P, C.c_double, P]
        L.orc_clearance.restype = C.c_double
        L.orc_config_clearance.argtypes = [P, P, C.c_int32, P]
        L.orc_config_clearance.restype = C.c_double
        L.orc_edge_count.argtypes = [P, P, C.c_int32, C.c_float]
        L.orc_edge_count.restype = C.c_int32
        L.orc_edge_clearance.argtypes = [P, P, C.c_int32, P, P, C.c_float, C.c_int32, C.c_int32]
        L.orc_edge_clearance.restype = C.c_double
        L.orc_check_edges.argtypes = [P, P, C.c_int32, P, P, C.c_int64, C.c_float, P, P, P,
                                      C.c_int32, C.c_int32]
        L.orc_nearest.argtypes = [P, C.c_int32, C.c_int32, P, P, C.c_int32]
        L.orc_nearest.restype = C.c_int32
        L.orc_steer.argtypes = [P, P, C.c_int32, C.c_float, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_sample_config.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, P, P,
                                        C.c_int32, P]
        L.orc_sample_config_try.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                            P, P, C.c_int32, P]
        L.orc_plan.argtypes = [P, P, C.c_int32, P, P, P, P, C.c_int32, P, P, C.c_int32]
        L.orc_plan.restype = C.c_int32
        L.orc_plan_dump.argtypes = [P, P, C.c_int32, P, P, P, P, C.c_int32, P, P, C.c_int32, P]
        L.orc_plan_dump.restype = C.c_int32
        L.orc_path_clearance.argtypes = [P, P, C.c_int32, P, C.c_int32, C.c_float, P]
        L.orc_path_clearance.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleRobot:
    """Keeps the numpy arrays referenced by the C struct alive."""

    def __init__(self, robot: dict):
        self.dof = int(sum(robot["chain_dof"]))
        self._dh = np.ascontiguousarray(robot["dh"], np.float32)
        self._lo = np.ascontiguousarray(robot["q_lo"], np.float32)
        self._hi = np.ascontiguousarray(robot["q_hi"], np.float32)
        self._frame = np.ascontiguousarray(robot["sphere_frame"], np.int32)
        self._xyzr = np.ascontiguousarray(robot["sphere_xyzr"], np.float32)
        self._pairs = np.ascontiguousarray(robot["self_pairs"], np.int32).reshape(-1, 2)
        s = Robot()
        s.n_chains = int(robot["n_chains"])
        for c in range(s.n_chains):
            s.chain_dof[c] = int(robot["chain_dof"][c])
            for i in range(12):
                s.base_pose[c][i] = float(robot["base_pose"][c][i])
        s.dh = self._dh.ctypes.data_as(C.POINTER(C.c_float))
        s.q_lo = self._lo.ctypes.data_as(C.POINTER(C.c_float))
        s.q_hi = self._hi.ctypes.data_as(C.POINTER(C.c_float))
        s.n_spheres = self._xyzr.shape[0]
        s.sphere_frame = self._frame.ctypes.data_as(C.POINTER(C.c_int32))
        s.sphere_xyzr = self._xyzr.ctypes.data_as(C.POINTER(C.c_float))
        s.n_self_pairs = self._pairs.shape[0]
        s.self_pairs = self._pairs.ctypes.data_as(C.POINTER(C.c_int32))
        self.struct = s
        self.n_frames = lib().orc_n_frames(C.byref(s))

    @property
    def ref(self):
        return C.byref(self.struct)


def _prims(prims: np.ndarray):
    prims = np.ascontiguousarray(prims)
    assert prims.dtype.itemsize == 64
    return prims


def fk_frames(rob: OracleRobot, q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros((rob.n_frames, 12))
    lib().orc_fk_frames(rob.ref, _ptr(q), _ptr(out))
    return out


def fk_spheres(rob: OracleRobot, q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float32)
    out = np.zeros((rob.struct.n_spheres, 3))
    lib().orc_fk_spheres(rob.ref, _ptr(q), _ptr(out))
    return out


def fk_spheres_batch(rob: OracleRobot, q, n_threads: int = 0) -> np.ndarray:
    """fk_spheres of every row of q [n][dof] -> [n][n_spheres][3] (FP64)."""
    q = np.ascontiguousarray(q, np.float32)
    out = np.zeros((q.shape[0], rob.struct.n_spheres, 3))
    lib().orc_fk_spheres_batch(rob.ref, _ptr(q), q.shape[0], _ptr(out), int(n_threads))
    return out


def clearance(c, r: float, prim) -> float:
    c = np.ascontiguousarray(c, np.float64)
    p = _prims(np.asarray(prim).reshape(1))
    return lib().orc_clearance(_ptr(c), float(r), _ptr(p))


def config_clearance(rob: OracleRobot, prims, q) -> float:
    p = _prims(prims)
    q = np.ascontiguousarray(q, np.float64)
    return lib().orc_config_clearance(rob.ref, _ptr(p), p.shape[0], _ptr(q))


def edge_count(a, b, res: float) -> int:
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    return lib().orc_edge_count(_ptr(a), _ptr(b), a.shape[0], float(res))


def edge_clearance(rob: OracleRobot, prims, a, b, res: float, i_first: int = 0,
                   early_exit: bool = False) -> float:
    p = _prims(prims)
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    return lib().orc_edge_clearance(rob.ref, _ptr(p), p.shape[0], _ptr(a), _ptr(b), float(res),
                                    int(i_first), int(early_exit))


def check_edges(rob: OracleRobot, prims, a, b, res: float, early_exit: bool = True,
                n_threads: int = 0, want_m: bool = False):
    """Returns (valid uint8[n], flagged uint8[n], m float64[n] or None)."""
    p = _prims(prims)
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    n = a.shape[0]
    valid = np.zeros(n, np.uint8)
    flagged = np.zeros(n, np.uint8)
    m = np.zeros(n) if want_m else None
    lib().orc_check_edges(rob.ref, _ptr(p), p.shape[0], _ptr(a), _ptr(b), n, float(res),
                          _ptr(valid), _ptr(flagged), _ptr(m) if m is not None else None,
                          int(early_exit), int(n_threads))
    return valid, flagged, m


def nearest(tree, size: int, x, blocked=None) -> int:
    tree = np.ascontiguousarray(tree, np.float32)  # [dof][cap]
    x = np.ascontiguousarray(x, np.float32)
    bl = None if blocked is None else np.ascontiguousarray(blocked, np.uint8)
    return lib().orc_nearest(_ptr(tree), tree.shape[1], int(size),
                             _ptr(bl) if bl is not None else None, _ptr(x), tree.shape[0])


def steer(frm, to, delta: float) -> np.ndarray:
    frm = np.ascontiguousarray(frm, np.float32)
    to = np.ascontiguousarray(to, np.float32)
    out = np.zeros_like(frm)
    lib().orc_steer(_ptr(frm), _ptr(to), frm.shape[0], float(delta), _ptr(out))
    return out


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample_config(seed: int, query: int, rnd: int, worker: int, lo, hi) -> np.ndarray:
    lo = np.ascontiguousarray(lo, np.float32)
    hi = np.ascontiguousarray(hi, np.float32)
    out = np.zeros_like(lo)
    lib().orc_sample_config(C.c_uint64(seed), query, rnd, worker, _ptr(lo), _ptr(hi),
                            lo.shape[0], _ptr(out))
    return out


class EsdfGrid:
    """An ESDF grid for the oracle: node values [nz][ny][nx] (x fastest) at
    origin + voxel (i, j, k).  attach() makes every clearance of the oracle
    take it into account (one grid at a time; detach() ends it)."""

    def __init__(self, origin, voxel, values):
        self.values = np.ascontiguousarray(values, np.float32)
        nz, ny, nx = self.values.shape
        self.struct = Esdf((C.c_float * 3)(*[float(x) for x in origin]), float(voxel),
                           (C.c_int32 * 3)(nx, ny, nz), self.values.ctypes.data)

    def value(self, p) -> float:
        p = np.ascontiguousarray(p, np.float64)
        return lib().orc_esdf_value(C.byref(self.struct), _ptr(p))

    def attach(self):
        lib().orc_esdf_attach(C.byref(self.struct))
        return self

    def detach(self):
        lib().orc_esdf_attach(None)

    def __enter__(self):
        return self.attach()

    def __exit__(self, *exc):
        self.detach()


def esdf_of_scene(prims, origin, voxel, dims, n_threads: int = 0) -> np.ndarray:
    """Node values of the signed distance to the union of the primitives
    (the least signed clearance at radius 0), FP64 rounded to FP32,
    [nz][ny][nx] for dims = (nx, ny, nz)."""
    p = _prims(prims)
    nx, ny, nz = (int(d) for d in dims)
    out = np.zeros((nz, ny, nx), np.float32)
    o = np.ascontiguousarray(origin, np.float32)
    d = np.array([nx, ny, nz], np.int32)
    lib().orc_esdf_from_prims(_ptr(p), p.shape[0], _ptr(o), float(voxel), _ptr(d), _ptr(out), int(n_threads))
    return out


def radical_inverse(i: int, base: int) -> float:
    return float(lib().orc_radical_inverse(int(i) & 0xFFFFFFFF, int(base)))


def halton_config(seed: int, query: int, rnd: int, worker: int, workers: int, tries: int, attempt: int,
                  lo, hi) -> np.ndarray:
    lo = np.ascontiguousarray(lo, np.float32)
    hi = np.ascontiguousarray(hi, np.float32)
    out = np.zeros(lo.shape[0], np.float32)
    lib().orc_halton_config(int(seed), int(query), int(rnd), int(worker), int(workers), int(tries), int(attempt),
                            _ptr(lo), _ptr(hi), lo.shape[0], _ptr(out))
    return out


def plan(rob: OracleRobot, prims, start, goal, seed=1, query=0, workers=256, delta=0.5, res=32.0,
         max_rounds=200, tree_capacity=1 << 16, validate_factor=4, dds_radius=0.0, dds_tries=1,
         n_threads=0, sampler=0):
    """Round replay of the planner.  Returns (status, path (K, dof) or None, stats dict)."""
    p = _prims(prims)
    s = np.ascontiguousarray(start, np.float32)
    g = np.ascontiguousarray(goal, np.float32)
    pp = PlanParams(seed=seed, query=query, workers=workers, delta=delta, res=res,
                    max_rounds=max_rounds, tree_capacity=tree_capacity,
                    validate_factor=validate_factor, dds_radius=dds_radius, dds_tries=dds_tries,
                    sampler=sampler)
    st = PlanStats()
    cap = 4096
    path = np.zeros((cap, rob.dof), np.float32)
    ln = C.c_int32(0)
    status = lib().orc_plan(rob.ref, _ptr(p), p.shape[0], _ptr(s), _ptr(g), C.byref(pp),
                            _ptr(path), cap, C.byref(ln), C.byref(st), int(n_threads))
    stats = {f: getattr(st, f) for f, _ in PlanStats._fields_}
    return status, (path[: ln.value].copy() if status == 0 else None), stats


def plan_trees(rob: OracleRobot, prims, start, goal, seed=1, query=0, workers=256, delta=0.5,
               res=32.0, max_rounds=200, tree_capacity=4096, validate_factor=4, dds_radius=0.0,
               dds_tries=1, n_threads=1, sampler=0):
    """As plan(), also returning the final trees: (status, path, stats, trees) with
    trees = {"a": (nodes (n, dof), parent (n,), blocked (n,)), "b": (...)}."""
    p = _prims(prims)
    s = np.ascontiguousarray(start, np.float32)
    g = np.ascontiguousarray(goal, np.float32)
    pp = PlanParams(seed=seed, query=query, workers=workers, delta=delta, res=res,
                    max_rounds=max_rounds, tree_capacity=tree_capacity,
                    validate_factor=validate_factor, dds_radius=dds_radius, dds_tries=dds_tries,
                    sampler=sampler)
    st = PlanStats()
    cap = 4096
    path = np.zeros((cap, rob.dof), np.float32)
    ln = C.c_int32(0)
    na = np.zeros((tree_capacity, rob.dof), np.float32)
    nb = np.zeros_like(na)
    pa = np.zeros(tree_capacity, np.int32)
    pb = np.zeros_like(pa)
    ba = np.zeros(tree_capacity, np.uint8)
    bb = np.zeros_like(ba)
    dump = TreeDump(na.ctypes.data, nb.ctypes.data, pa.ctypes.data, pb.ctypes.data,
                    ba.ctypes.data, bb.ctypes.data)
    status = lib().orc_plan_dump(rob.ref, _ptr(p), p.shape[0], _ptr(s), _ptr(g), C.byref(pp),
                                 _ptr(path), cap, C.byref(ln), C.byref(st), int(n_threads),
                                 C.byref(dump))
    stats = {f: getattr(st, f) for f, _ in PlanStats._fields_}
    ka, kb = stats["nodes_a"], stats["nodes_b"]
    trees = {"a": (na[:ka].copy(), pa[:ka].copy(), ba[:ka].copy()),
             "b": (nb[:kb].copy(), pb[:kb].copy(), bb[:kb].copy())}
    return status, (path[: ln.value].copy() if status == 0 else None), stats, trees


def path_clearance(rob: OracleRobot, prims, path, res: float):
    p = _prims(prims)
    path = np.ascontiguousarray(path, np.float32)
    nf = C.c_int32(0)
    m = lib().orc_path_clearance(rob.ref, _ptr(p), p.shape[0], _ptr(path), path.shape[0],
                                 float(res), C.byref(nf))
    return m, nf.value
