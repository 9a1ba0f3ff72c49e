import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def wl():
    from paper_2503_06757_amd import workloads
    return workloads


@pytest.fixture(scope="session")
def r7(wl):
    return wl.robot_r7()


@pytest.fixture(scope="session")
def r14(wl):
    return wl.robot_r14()


@pytest.fixture(scope="session")
def gpu():
    """(binding module, context handle, torch) on cuda:0; the HIP library must be built."""
    import torch
    from paper_2503_06757_amd import prrtc as P
    assert torch.cuda.is_available(), "GPU test needs a visible MI355X"
    ctx = P.prrtc_create(0)
    yield P, ctx, torch
    torch.cuda.synchronize()
    P.prrtc_destroy(ctx)


def free_query(orc, rob, prims, robot, seed, n=200, margin=1e-4):
    """First generated (start, goal) whose endpoints the oracle finds clear."""
    import numpy as np
    from paper_2503_06757_amd import workloads as W
    for s, g in W.query_candidates(robot, seed, n):
        if (orc.config_clearance(rob, prims, s.astype(np.float64)) > margin and
                orc.config_clearance(rob, prims, g.astype(np.float64)) > margin):
            return s, g
    raise RuntimeError("no free query among the candidates")


def path_ok(orc, robot, prims, path, s, g, delta=0.5, res=32.0):
    """A planned path is exact at both ends, has segments of at most delta and
    is collision-free for the oracle at 4x the planning resolution."""
    rob = orc.OracleRobot(robot)
    assert np.array_equal(path[0], s) and np.array_equal(path[-1], g)
    seg = np.linalg.norm(np.diff(path.astype(np.float64), axis=0), axis=1)
    assert np.all(seg <= delta * (1 + 1e-6))
    m, _ = orc.path_clearance(rob, prims, path, 4 * res)
    assert m >= -orc.FLAG_BAND, m


def replay_equal(orc, robot, prims, s, g, gst, gpath, gstats, **kw):
    """The oracle replays the query's rounds with the same parameters; when it
    met no edge within the 1e-5 m flag band, status, rounds, tree sizes,
    edge count, re-check failures, the connecting worker and the path must
    equal the GPU's.  Returns whether the comparison was made."""
    rob = orc.OracleRobot(robot)
    ost, opath, ostats = orc.plan(rob, prims, s, g, n_threads=16, **kw)
    print("   oracle:", ost, ostats, " gpu:", gst, {k: gstats[k] for k in
                                                 ("rounds", "nodes_a", "nodes_b", "edges_checked",
                                                  "validation_failures", "connect_worker")}, flush=True)
    if ostats["flagged_edges"] == 0:
        assert gst == ost
        assert gstats["rounds"] == ostats["rounds"]
        assert gstats["nodes_a"] == ostats["nodes_a"] and gstats["nodes_b"] == ostats["nodes_b"]
        assert gstats["edges_checked"] == ostats["edges_checked"]
        assert gstats["validation_failures"] == ostats["validation_failures"]
        if gst == 0:
            assert gstats["connect_worker"] == ostats["connect_worker"]
            assert np.array_equal(gpath, opath)
        return True
    return False
