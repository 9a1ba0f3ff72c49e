"""Pins of the proposal oracle: bfloat16 rounding against an independent
implementation, GELU and Gaussian closed forms, mixture invariances,
analytic gradients against central finite differences, Adam's first step,
and the voxel grid on a box aligned with the cells."""
import math

import numpy as np
import pytest

from paper_2503_06757_amd import workloads as W


@pytest.fixture(scope="module")
def prop(orc):
    from oracle import proposal
    return proposal


def test_bf16_rounding_matches_torch(prop):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.140625, 0.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(prop.bf16(x), ref)
    assert prop.bf16(1.0 + 2 ** -8) == 1.0                 # tie -> even
    assert prop.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7


def test_gelu_closed_forms(prop):
    # GELU(x) = x * Phi(x); Phi(1) = 0.8413447460685429, Phi(-2) = 0.022750131948179195
    assert prop.gelu(np.array([0.0]))[0] == 0.0
    assert prop.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-14)
    assert prop.gelu(np.array([-2.0]))[0] == pytest.approx(-2 * 0.022750131948179195, rel=1e-12)
    x = np.linspace(-4, 4, 81)
    fd = (prop.gelu(x + 1e-6) - prop.gelu(x - 1e-6)) / 2e-6
    np.testing.assert_allclose(prop.gelu_grad(x), fd, atol=1e-8)
    assert prop.gelu_grad(np.array([0.0]))[0] == 0.5


def _one_component(mu, logsig, k=0):
    logits = np.full((1, prop_n()), -1e9)
    logits[0, k] = 0.0
    return logits


def prop_n():
    from oracle import proposal
    return proposal.N_COMP


def test_nll_single_component_is_gaussian(prop):
    rng = np.random.default_rng(1)
    dof = 7
    mu = rng.standard_normal((1, prop.N_COMP, dof))
    logsig = rng.uniform(-2, 1, (1, prop.N_COMP, dof))
    q = rng.standard_normal((1, dof))
    logits = _one_component(mu, logsig, 3)
    z = (q[0] - mu[0, 3]) / np.exp(logsig[0, 3])
    exp = np.sum(0.5 * z * z + logsig[0, 3] + 0.5 * math.log(2 * math.pi))
    assert prop.nll((logits, mu, logsig), q)[0] == pytest.approx(exp, rel=1e-12)


def test_nll_invariances(prop):
    rng = np.random.default_rng(2)
    B, dof = 5, 7
    logits = rng.standard_normal((B, prop.N_COMP))
    mu = rng.standard_normal((B, prop.N_COMP, dof))
    logsig = rng.uniform(-1, 0.5, (B, prop.N_COMP, dof))
    q = rng.standard_normal((B, dof))
    base = prop.nll((logits, mu, logsig), q)
    np.testing.assert_allclose(prop.nll((logits + 3.7, mu, logsig), q), base, rtol=1e-12)
    perm = rng.permutation(prop.N_COMP)
    np.testing.assert_allclose(prop.nll((logits[:, perm], mu[:, perm], logsig[:, perm]), q), base, rtol=1e-12)
    # two identical components with equal weights = one component
    l2 = np.full((B, prop.N_COMP), -1e9)
    l2[:, :2] = 0.0
    mu2 = mu.copy()
    mu2[:, 1] = mu2[:, 0]
    ls2 = logsig.copy()
    ls2[:, 1] = ls2[:, 0]
    l1 = np.full((B, prop.N_COMP), -1e9)
    l1[:, 0] = 0.0
    np.testing.assert_allclose(prop.nll((l2, mu2, ls2), q), prop.nll((l1, mu, logsig), q), rtol=1e-12)


def _tiny_model(prop, dof, seed):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal(shp) * (0.5 / math.sqrt(shp[0]) if len(shp) == 2 else 0.1)
            for k, shp in prop.dims(dof).items()}


def test_gradients_match_finite_differences(prop):
    dof = 3
    params = _tiny_model(prop, dof, 3)
    rng = np.random.default_rng(4)
    S, B = 2, 5
    vox = (rng.random((S, 4096)) < 0.1).astype(np.float64)
    scene_of = np.array([0, 0, 1, 1, 1])
    lo, hi = -np.ones(dof) * 2.8, np.ones(dof) * 2.8
    s = rng.uniform(-2.8, 2.8, (B, dof))
    g = rng.uniform(-2.8, 2.8, (B, dof))
    q = rng.uniform(-0.9, 0.9, (B, dof))

    def loss(p):
        gm, _ = prop.forward(p, vox, scene_of, s, g, lo, hi, rounding=False)
        return prop.nll(gm, q).mean()

    gm, cache = prop.forward(params, vox, scene_of, s, g, lo, hi, rounding=False)
    G = prop.backward(params, cache, gm, q, rounding=False)
    for k in prop.PARAM_ORDER:
        flat = params[k].reshape(-1)
        for idx in rng.choice(flat.size, 4, replace=False):
            p2 = {kk: vv.copy() for kk, vv in params.items()}
            h = 1e-6
            p2[k].reshape(-1)[idx] += h
            up = loss(p2)
            p2[k].reshape(-1)[idx] -= 2 * h
            dn = loss(p2)
            fd = (up - dn) / (2 * h)
            an = G[k].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (k, idx)


def test_adam_first_step_closed_form(prop):
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -0.25, 2.0])}
    z = {"w": np.zeros(3)}
    p1, m1, v1 = prop.adam(p, g, z, z, 1, lr=0.01)
    # bias-corrected first step: lr * g / (|g| + eps) = lr * sign(g)
    np.testing.assert_allclose(p1["w"], p["w"] - 0.01 * np.sign(g["w"]), rtol=1e-7)
    np.testing.assert_allclose(m1["w"], 0.1 * g["w"])
    np.testing.assert_allclose(v1["w"], 0.001 * g["w"] ** 2)


def test_voxel_grid_box_aligned_with_cells(prop):
    # a box 1 mm inside the cell block x: cells 8..11, y: 8..9, z: 8 (4 x 2 x 1 cells);
    # face and edge neighbours (0.051 m, 0.072 m) are within the half diagonal
    # 0.0866 m, corner neighbours (0.088 m) are not: (4+2)(2+2)(1+2) - 8 cells.
    lo = np.array([0.0, 0.0, 0.0]) + 0.001
    hi = np.array([0.4, 0.2, 0.1]) - 0.001
    box = W.make_prims([(W.PRIM_CUBOID, (lo + hi) / 2, np.eye(3), (hi - lo) / 2)])
    occ, margin = prop.voxelize(box)
    assert int(occ.sum()) == 6 * 4 * 3 - 8
    assert np.all(np.abs(margin) > 1e-3)
    idx = (8 * 16 + 8) * 16 + 8          # cell (8, 8, 8) holds the box corner region
    assert occ[idx] == 1


def _row(prop, dof, logits, mu, ls):
    return np.concatenate([logits, np.broadcast_to(mu, (prop.N_COMP, dof)).ravel(),
                           np.broadcast_to(ls, (prop.N_COMP, dof)).ravel()])


def test_mixture_draw_normals(prop):
    """One component at mu = 0, sigma = 1 over [-1, 1] limits: q is a standard
    normal draw (Box-Muller); mean, variance, an independence check across the
    pair and a Kolmogorov-Smirnov test against the normal CDF."""
    from scipy import stats
    dof = 4
    logits = np.full(prop.N_COMP, -1e30)
    logits[2] = 0.0
    row = _row(prop, dof, logits, 0.0, 0.0)
    lo, hi = -np.ones(dof), np.ones(dof)
    Z = np.array([prop.mixture_draw(row, dof, lo, hi, 7, 1, 2, w, 0)[0] for w in range(6000)])
    assert abs(Z.mean()) < 0.05
    np.testing.assert_allclose(Z.var(axis=0), 1.0, atol=0.08)
    assert abs(np.corrcoef(Z[:, 0], Z[:, 1])[0, 1]) < 0.05
    for j in range(dof):
        assert stats.kstest(Z[:, j], "norm").pvalue > 1e-3


def test_mixture_draw_components_and_scaling(prop):
    """Component frequencies follow softmax(logits) (chi-square); a component
    with sigma ~ 0 lands exactly on lo + (mu + 1)(hi - lo) / 2."""
    from scipy import stats
    dof = 3
    pw = np.array([0.4, 0.2, 0.1, 0.1, 0.05, 0.05, 0.05, 0.05])
    mu = np.linspace(-0.7, 0.7, prop.N_COMP)[:, None] * np.ones(dof)
    row = _row(prop, dof, np.log(pw) + 1.3, mu, -60.0)
    lo, hi = np.array([-2.0, 0.0, -1.0]), np.array([2.0, 3.0, 0.5])
    n = 8000
    counts = np.zeros(prop.N_COMP)
    for w in range(n):
        q, k, _ = prop.mixture_draw(row, dof, lo, hi, 3, 0, 0, w, 5)
        counts[k] += 1
        np.testing.assert_allclose(q, lo + 0.5 * (mu[k] + 1.0) * (hi - lo), atol=1e-12)
    assert stats.chisquare(counts, pw * n).pvalue > 1e-3
    # the mixing uniform and the component uniform are distinct words
    us = [prop.mix_uniform(3, 0, 0, w, 5) for w in range(2000)]
    assert 0.45 < np.mean(us) < 0.55 and min(us) >= 0.0 and max(us) < 1.0
