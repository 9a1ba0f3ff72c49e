import os
import sys

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
