"""Host-side logic that needs no GPU: path resampling for the proposal's
training targets, the proposal blob layout, the shelf workload's placement
rules and the benchmark's percentile reporting."""
import numpy as np

from paper_2503_06757_amd import proposal as PR
from paper_2503_06757_amd import workloads as W


def test_resample_path_spacing_and_tail():
    path = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0]], np.float32)   # arclength 2
    w = PR.resample_path(path, step=0.25)
    # every 0.25 rad of arclength, both endpoints excluded
    assert w.shape == (7, 2)
    arc = np.concatenate([[0.0], np.cumsum(np.linalg.norm(np.diff(np.vstack([path[:1], w]), axis=0), axis=1))])
    assert np.allclose(np.diff(arc), 0.25, atol=1e-6)
    # only the last half of the arclength (from t = 1 on)
    t = PR.resample_path(path, step=0.25, tail=0.5)
    assert np.allclose(t, w[3:])
    # a path shorter than one step has no interior target
    assert PR.resample_path(path[:2] * 0.1, step=0.25).shape == (0, 2)


def test_proposal_blob_roundtrip():
    dof = 7
    params = PR.init_params(dof, 5)
    blob = PR.pack(params, dof)
    got_dof, adam_t, groups = PR.unpack(blob)
    assert got_dof == dof and adam_t == 0 and len(groups) == 1
    p2 = groups[0]
    for k in PR.PARAM_ORDER:
        assert np.array_equal(np.asarray(p2[k]), params[k]), k
    shapes = PR.param_shapes(dof)
    n = sum(int(np.prod(s)) for s in shapes.values())
    assert len(blob) == PR.HEADER.size + 4 * n


def test_shelf_spheres_keep_out_of_the_approach_slab():
    r14 = W.robot_r14()
    prims = W.scene_shelf(r14)
    assert prims.shape[0] == 64 and int((prims["type"] == 1).sum()) == 40
    sph = prims[prims["type"] == 0]
    assert sph.shape[0] == 24
    for p in sph:
        c, r = p["c"].astype(np.float64), float(p["dims"][0])
        assert 0.05 <= r <= 0.15 and c[2] >= 0.0
        inside_slab = np.all(c > W.APPROACH_LO - r) and np.all(c < W.APPROACH_HI + r)
        assert not inside_slab
    # the same seed gives the same scene
    assert np.array_equal(W.scene_shelf(r14), prims)


def test_bench_percentiles_report_failures_as_null():
    import bench
    t = np.array([1.0, 2.0, 3.0, np.inf])
    p = bench.pcts(t)
    assert p["p50_ms"] == 2.5 and p["p90_ms"] is None and p["p99_ms"] is None
    assert bench.pcts(np.array([]))["p50_ms"] is None


def test_served_shape_most_workers_with_headroom():
    """Serving takes the most workers per query whose tuned rate keeps the
    headroom over the arrival rate; with none, the tuner's fastest shape."""
    import bench
    rates = {(16, 16): 2484.0, (16, 64): 2116.0, (32, 16): 2422.0, (32, 64): 1721.0, (64, 16): 2219.0,
             (64, 64): 1196.0, (128, 16): 2043.0, (128, 64): 1255.0, (256, 16): 1508.0, (256, 64): 655.0}
    assert bench.served_shape(rates, 2000.0, (16, 16)) == (64, 16)
    assert bench.served_shape(rates, 1000.0, (16, 16)) == (256, 16)
    assert bench.served_shape(rates, 1450.0, (16, 16)) == (128, 16)   # 1508 < 1.05 x 1450
    assert bench.served_shape(rates, 600.0, (16, 16)) == (256, 16)    # both tiles keep up: the faster one
    assert bench.served_shape(rates, 5000.0, (16, 16)) == (16, 16)    # nothing keeps up: the fastest
