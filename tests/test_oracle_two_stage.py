"""Pins of two-stage sphere checking (Sec. III-A: a low-resolution pass over
coarse spheres flags the links that may collide; only their fine spheres are
then checked) on the synthetic coarse layout, independent of the GPU: every
coarse sphere encloses its fine spheres, and the two-stage decision equals
the fine-sphere decision on every configuration, which fails as soon as the
coarse spheres are made too small."""
import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W


def _world(frames, f, p):
    F = frames[f].reshape(3, 4)
    return F[:, :3] @ np.asarray(p, np.float64) + F[:, 3]


def two_stage_collides(orc, rob, robot, prims, q, shrink=1.0):
    """The two-stage decision from the oracle's clearances: coarse spheres
    that meet an obstacle flag their fine spheres, and a flagged fine sphere
    that meets one (or any self pair) is a collision."""
    frames = orc.fk_frames(rob, q)
    xyz = orc.fk_spheres(rob, np.asarray(q, np.float32))
    cx = robot["coarse_xyzr"]
    flagged = []
    for c in range(cx.shape[0]):
        centre = _world(frames, robot["coarse_frame"][c], cx[c, :3])
        flagged.append(any(orc.clearance(centre, float(cx[c, 3]) * shrink, pr) < 0 for pr in prims))
    for k in range(xyz.shape[0]):
        if flagged[robot["sphere_coarse"][k]]:
            r = float(robot["sphere_xyzr"][k, 3])
            if any(orc.clearance(xyz[k], r, pr) < 0 for pr in prims):
                return True
    for i, j in robot["self_pairs"]:
        ri, rj = robot["sphere_xyzr"][i, 3], robot["sphere_xyzr"][j, 3]
        if np.linalg.norm(xyz[i] - xyz[j]) - (ri + rj) < 0:
            return True
    return False


@pytest.mark.parametrize("name", ["r7", "r14"])
def test_coarse_spheres_enclose_their_fine_spheres(name):
    robot = W.with_coarse_spheres(W.robot_r7() if name == "r7" else W.robot_r14())
    f, c = robot["sphere_xyzr"].astype(np.float64), robot["coarse_xyzr"].astype(np.float64)
    own = robot["sphere_coarse"]
    assert np.all(robot["coarse_frame"][own] == robot["sphere_frame"])
    reach = np.linalg.norm(f[:, :3] - c[own, :3], axis=1) + f[:, 3]
    assert np.all(reach <= c[own, 3])
    assert c.shape[0] < f.shape[0] / 4        # coarse: far fewer spheres


@pytest.mark.parametrize("scene", ["s12", "s64", "shelf"])
def test_two_stage_decision_equals_fine_decision(orc, scene):
    robot = W.with_coarse_spheres(W.robot_r14() if scene == "shelf" else W.robot_r7())
    prims = {"s12": lambda: W.scene_s12(robot, 1), "s64": lambda: W.scene_s64(robot),
             "shelf": lambda: W.scene_shelf(robot)}[scene]()
    rob = orc.OracleRobot(robot)
    rng = np.random.default_rng(7)
    qs = rng.uniform(robot["q_lo"], robot["q_hi"], (150, len(robot["q_lo"])))
    both = 0
    for q in qs:
        fine = orc.config_clearance(rob, prims, q) < 0
        assert two_stage_collides(orc, rob, robot, prims, q) == fine
        both += fine
    assert 0 < both < len(qs)


def test_too_small_coarse_spheres_miss_collisions(orc):
    """The equivalence rests on enclosure: coarse spheres shrunk by 40% let
    colliding configurations through."""
    robot = W.with_coarse_spheres(W.robot_r7())
    prims = W.scene_s64(robot)
    rob = orc.OracleRobot(robot)
    qs = np.random.default_rng(8).uniform(-2.8, 2.8, (150, 7))
    missed = sum(orc.config_clearance(rob, prims, q) < 0 and not two_stage_collides(orc, rob, robot, prims, q, 0.6)
                 for q in qs)
    assert missed > 0
