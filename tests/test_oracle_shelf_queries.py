"""The stored dual-arm shelf queries (tests/golden/shelf_queries_r14.txt,
written by oracle/make_shelf_queries.py): every start is collision-free and
in front of the shelf, every goal is collision-free with each hand-bar centre
inside a shelf cell on its arm's side, and the first rows regenerate
bit for bit."""
import os

import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W

PATH = os.path.join(os.path.dirname(__file__), "golden", "shelf_queries_r14.txt")


@pytest.fixture(scope="module")
def rows():
    return np.loadtxt(PATH, dtype=np.float32)


def test_fixture_shape(rows):
    assert rows.shape == (500, 28)
    assert np.all(np.abs(rows) <= W.R7_LIMIT)


def test_queries_valid(orc, rows):
    r14 = W.robot_r14()
    rob = orc.OracleRobot(r14)
    prims = W.scene_shelf(r14)
    cells = W.shelf_cells()
    for row in rows[::5]:
        s, g = row[:14].astype(np.float64), row[14:].astype(np.float64)
        assert orc.config_clearance(rob, prims, s) > 1e-3
        assert np.all(orc.fk_spheres(rob, row[:14])[:, 0] < 0.4)
        assert orc.config_clearance(rob, prims, g) > 1e-3
        xyz = orc.fk_spheres(rob, row[14:])
        for arm in (0, 1):
            hand = xyz[60 * arm:60 * (arm + 1)][W.HAND_SPHERES]
            c = W.hand_cell(hand)
            assert c >= 0
            lo, hi = cells[c]
            assert (hi[1] <= 1e-9) if arm == 0 else (lo[1] >= -1e-9)


def test_first_rows_regenerate(orc, rows):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "mk", os.path.join(os.path.dirname(os.path.dirname(__file__)), "oracle", "make_shelf_queries.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    for i in range(2):
        assert np.array_equal(mk._one(i), rows[i])
