"""Configurations and edges built to lie within 1e-6 .. 1e-3 m of contact
(either side), for checking FP32 verdicts against the FP64 oracle where the
1e-5 m flag band matters.

From a configuration q0 with clearance above 2 mm, the robot moves along a
random joint-space direction d until it penetrates by more than 2 mm; for
each target clearance c, bisection on t in FP64 finds q0 + t d whose oracle
clearance is c, and the configuration is rounded to FP32 (which moves the
clearance by up to about a micrometre; the oracle's value at the rounded
configuration is what the tests use).  Test infrastructure only: it calls
the oracle's clearance and nothing of the HIP path.
"""
import numpy as np

TARGETS = np.array([1e-6, 3e-6, 9e-6, 1.2e-5, 2e-5, 5e-5, 1e-4, 3e-4, 1e-3])
TARGETS = np.concatenate([-TARGETS[::-1], TARGETS])


def graze_configs(orc, robot, prims, n_dirs, seed, targets=TARGETS, iters=64):
    """[(q float32 [dof], target c, oracle clearance of q, direction, t)] for
    n_dirs random (q0, d) pairs times every target."""
    rob = orc.OracleRobot(robot)
    rng = np.random.default_rng(seed)
    lo, hi = robot["q_lo"].astype(np.float64), robot["q_hi"].astype(np.float64)
    dof = lo.size
    clear = lambda q: orc.config_clearance(rob, prims, q)
    out = []
    found = 0
    for _ in range(200 * n_dirs):
        if found == n_dirs:
            break
        q0 = rng.uniform(lo, hi)
        if clear(q0) < 2e-3:
            continue
        d = rng.standard_normal(dof)
        d /= np.linalg.norm(d)
        t_hit = None
        for t in np.arange(0.02, 4.0, 0.02):
            if clear(q0 + t * d) < -2e-3:
                t_hit = t
                break
        if t_hit is None:
            continue
        found += 1
        for c in targets:
            a, b = 0.0, t_hit          # clear(q0 + a d) > c > clear(q0 + b d)
            for _ in range(iters):
                m = 0.5 * (a + b)
                if clear(q0 + m * d) > c:
                    a = m
                else:
                    b = m
            q = (q0 + 0.5 * (a + b) * d).astype(np.float32)
            out.append((q, float(c), clear(q.astype(np.float64)), d, 0.5 * (a + b)))
    return out


def graze_edges(configs, back=0.05):
    """Two edges per configuration q: zero length (a = b = q) and an approach
    edge ending at q from `back` rad earlier along its direction."""
    a, b = [], []
    for q, _, _, d, t in configs:
        a.append(q)
        b.append(q)
        a.append((q.astype(np.float64) - back * d).astype(np.float32))
        b.append(q)
    return np.array(a, np.float32), np.array(b, np.float32)


def graze_scenes(W, r7, r14):
    """(name, robot, prims): one primitive type at a time, thin shelf boards,
    and the dual arm's inter-arm pairs alone."""
    s64 = W.scene_s64(r7)
    out = [("spheres", r7, s64[s64["type"] == W.PRIM_SPHERE]),
           ("cuboids", r7, s64[s64["type"] == W.PRIM_CUBOID]),
           ("cylinders", r7, s64[s64["type"] == W.PRIM_CYLINDER]),
           ("shelf", r14, W.scene_shelf(r14)),
           ("self pairs", r14, np.zeros(0, W.PRIM_DTYPE))]
    return out
