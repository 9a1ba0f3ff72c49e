"""Oracle of the learned sampling proposal: voxel grid, MLP, Gaussian mixture.

TEST INFRASTRUCTURE ONLY (tests, smoke, benchmark CPU baseline); shares no
code with the HIP library.  Plain numpy in FP64.  The paper samples uniformly
(Halton, Sec. IV-A); this proposal is an addition whose definition is fixed
here and implemented identically on the GPU:

  * scene encoding: a 16^3 occupancy grid over [-0.8, 0.8]^3 (0.1 m cells); a
    cell is occupied iff some obstacle lies closer than the cell's half
    diagonal (0.05 * sqrt(3) m) to the cell centre;
  * MLP: e = vox W_v + b_v (4096 -> 256); x0 = [s_hat, g_hat, e] with start and
    goal scaled to [-1, 1] by the joint limits; three Linear(256) + GELU
    (erf form) layers; a head Linear(256 -> K (1 + 2 dof)) giving K = 8 mixture
    logits, means and log standard deviations (clamped to [-5, 2]) in the same
    scaled coordinates;
  * every matrix product rounds both operands to bfloat16 (round to nearest
    even) and accumulates in high precision, as the kernels do;
  * loss: negative log-likelihood of a scaled waypoint under the mixture,
    averaged over the batch; Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8);
  * drawing from the mixture (the learned RANDOM_CONFIG): Philox4x32-10 words
    with counter (0x80000000 | attempt << 8 | slot, worker, round, query) and
    key = seed; slot 255 word 0 decides mixture against uniform, word 1 picks
    the component by inverse CDF of the softmax weights; slot 1 + j // 2 gives
    the Box-Muller pair of joints j, j + 1.
"""
from __future__ import annotations

import math

import numpy as np

from . import clearance as _clearance
from . import philox as _philox

N_COMP = 8
HIDDEN = 256
VOX = 16
VOX_LO, VOX_CELL = -0.8, 0.1
LOGSIG_LO, LOGSIG_HI = -5.0, 2.0
PARAM_ORDER = ("Wv", "bv", "W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) through float32; returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def voxelize(prims) -> tuple[np.ndarray, np.ndarray]:
    """(occupancy uint8 [4096] in x-fastest order, min clearance - half diagonal
    per cell (for flagging cells at the threshold))."""
    half = 0.5 * VOX_CELL * math.sqrt(3.0)
    occ = np.zeros(VOX ** 3, np.uint8)
    margin = np.full(VOX ** 3, np.inf)
    for z in range(VOX):
        for y in range(VOX):
            for x in range(VOX):
                c = VOX_LO + VOX_CELL * (np.array([x, y, z]) + 0.5)
                i = (z * VOX + y) * VOX + x
                m = min((_clearance(c, 0.0, p) for p in prims), default=np.inf)
                margin[i] = m - half
                occ[i] = m < half
    return occ, margin


def dims(dof: int) -> dict:
    return dict(Wv=(VOX ** 3, HIDDEN), bv=(HIDDEN,), W1=(2 * dof + HIDDEN, HIDDEN), b1=(HIDDEN,),
                W2=(HIDDEN, HIDDEN), b2=(HIDDEN,), W3=(HIDDEN, HIDDEN), b3=(HIDDEN,),
                W4=(HIDDEN, N_COMP * (1 + 2 * dof)), b4=(N_COMP * (1 + 2 * dof),))


def gelu(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def scale(q, lo, hi):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    return 2.0 * (np.asarray(q, np.float64) - lo) / (hi - lo) - 1.0


def _mm(a, b, rounding):
    return (bf16(a) @ bf16(b)) if rounding else (np.asarray(a, np.float64) @ np.asarray(b, np.float64))


def forward(params, vox, scene_of, s, g, lo, hi, rounding=True):
    """Mixture parameters for each sample and the cache for backward.
    vox: [S, 4096]; scene_of: [B] row of vox per sample; s, g: [B, dof]."""
    P = {k: np.asarray(v, np.float64) for k, v in params.items()}
    dof = np.asarray(s).shape[1]
    E = _mm(vox, P["Wv"], rounding) + P["bv"]
    x0 = np.concatenate([scale(s, lo, hi), scale(g, lo, hi), E[np.asarray(scene_of)]], axis=1)
    z1 = _mm(x0, P["W1"], rounding) + P["b1"]
    h1 = gelu(z1)
    z2 = _mm(h1, P["W2"], rounding) + P["b2"]
    h2 = gelu(z2)
    z3 = _mm(h2, P["W3"], rounding) + P["b3"]
    h3 = gelu(z3)
    o = _mm(h3, P["W4"], rounding) + P["b4"]
    logits = o[:, :N_COMP]
    mu = o[:, N_COMP:N_COMP * (1 + dof)].reshape(-1, N_COMP, dof)
    raw = o[:, N_COMP * (1 + dof):].reshape(-1, N_COMP, dof)
    logsig = np.clip(raw, LOGSIG_LO, LOGSIG_HI)
    cache = dict(E=E, x0=x0, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3, raw=raw, vox=vox,
                 scene_of=np.asarray(scene_of))
    return (logits, mu, logsig), cache


def log_softmax(a):
    m = a.max(axis=-1, keepdims=True)
    return a - m - np.log(np.exp(a - m).sum(axis=-1, keepdims=True))


def nll(gmm, q_hat):
    """Per-sample negative log-likelihood of q_hat [B, dof] under the mixture."""
    logits, mu, logsig = gmm
    z = (q_hat[:, None, :] - mu) / np.exp(logsig)
    comp = np.sum(-0.5 * z * z - logsig - 0.5 * math.log(2.0 * math.pi), axis=2)
    a = log_softmax(logits) + comp
    m = a.max(axis=1, keepdims=True)
    return -(m[:, 0] + np.log(np.exp(a - m).sum(axis=1)))


def backward(params, cache, gmm, q_hat, rounding=True):
    """Gradients of the batch-mean NLL with respect to every parameter."""
    P = {k: np.asarray(v, np.float64) for k, v in params.items()}
    logits, mu, logsig = gmm
    B, K, dof = mu.shape
    sig = np.exp(logsig)
    z = (q_hat[:, None, :] - mu) / sig
    comp = np.sum(-0.5 * z * z - logsig - 0.5 * math.log(2.0 * math.pi), axis=2)
    lp = log_softmax(logits)
    a = lp + comp
    r = np.exp(a - a.max(axis=1, keepdims=True))
    r /= r.sum(axis=1, keepdims=True)                          # responsibilities
    d_logits = (np.exp(lp) - r) / B
    d_mu = -(r[:, :, None] * z / sig) / B
    d_logsig = -(r[:, :, None] * (z * z - 1.0)) / B
    inside = (cache["raw"] >= LOGSIG_LO) & (cache["raw"] <= LOGSIG_HI)
    d_raw = d_logsig * inside
    do = np.concatenate([d_logits, d_mu.reshape(B, -1), d_raw.reshape(B, -1)], axis=1)
    G = {}
    G["W4"] = _mm(cache["h3"].T, do, rounding)
    G["b4"] = do.sum(axis=0)
    dz3 = _mm(do, P["W4"].T, rounding) * gelu_grad(cache["z3"])
    G["W3"] = _mm(cache["h2"].T, dz3, rounding)
    G["b3"] = dz3.sum(axis=0)
    dz2 = _mm(dz3, P["W3"].T, rounding) * gelu_grad(cache["z2"])
    G["W2"] = _mm(cache["h1"].T, dz2, rounding)
    G["b2"] = dz2.sum(axis=0)
    dz1 = _mm(dz2, P["W2"].T, rounding) * gelu_grad(cache["z1"])
    G["W1"] = _mm(cache["x0"].T, dz1, rounding)
    G["b1"] = dz1.sum(axis=0)
    dx0 = _mm(dz1, P["W1"].T, rounding)
    dE = np.zeros_like(cache["E"])
    np.add.at(dE, cache["scene_of"], dx0[:, 2 * dof:])
    G["Wv"] = _mm(np.asarray(cache["vox"], np.float64).T, dE, rounding)
    G["bv"] = dE.sum(axis=0)
    return G


def adam(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (params, m, v)."""
    out_p, out_m, out_v = {}, {}, {}
    for k in params:
        mk = b1 * m[k] + (1.0 - b1) * grads[k]
        vk = b2 * v[k] + (1.0 - b2) * grads[k] * grads[k]
        mh = mk / (1.0 - b1 ** t)
        vh = vk / (1.0 - b2 ** t)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v


def mixture_moments(gmm_one):
    """Mean and per-joint variance of one sample's mixture (scaled coords)."""
    logits, mu, logsig = gmm_one
    w = np.exp(log_softmax(logits))
    mean = np.sum(w[:, None] * mu, axis=0)
    second = np.sum(w[:, None] * (np.exp(2 * logsig) + mu * mu), axis=0)
    return mean, second - mean * mean


def _unit(word) -> float:
    return float(int(word) >> 8) * 2.0 ** -24


def _words(seed, query, rnd, worker, attempt, slot):
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return _philox([0x80000000 | (attempt << 8) | slot, worker, rnd, query], key)


def mix_uniform(seed, query, rnd, worker, attempt) -> float:
    """The uniform compared with the mixing probability (slot 255, word 0)."""
    return _unit(_words(seed, query, rnd, worker, attempt, 255)[0])


def mixture_draw(gmm_row, dof, lo, hi, seed, query, rnd, worker, attempt):
    """One draw from one sample's mixture, in FP64 after the Philox words.
    gmm_row = [K logits | K x dof means | K x dof log sigmas] (scaled
    coordinates).  Returns (q in joint units, component, distance of the
    component uniform from the nearest inner CDF boundary)."""
    g = np.asarray(gmm_row, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    logits = g[:N_COMP]
    mu = g[N_COMP:N_COMP * (1 + dof)].reshape(N_COMP, dof)
    ls = g[N_COMP * (1 + dof):N_COMP * (1 + 2 * dof)].reshape(N_COMP, dof)
    w = np.exp(logits - logits.max())
    cdf = np.cumsum(w / w.sum())
    uc = _unit(_words(seed, query, rnd, worker, attempt, 255)[1])
    comp = next((k for k in range(N_COMP) if uc < cdf[k]), N_COMP - 1)
    gap = float(np.min(np.abs(uc - cdf[:-1])))
    q = np.empty(dof)
    for j in range(dof):
        wn = _words(seed, query, rnd, worker, attempt, 1 + j // 2)
        u1 = (float(int(wn[0]) >> 8) + 1.0) * 2.0 ** -24
        u2 = _unit(wn[1])
        r = math.sqrt(-2.0 * math.log(u1))
        z = r * (math.sin(2.0 * math.pi * u2) if j % 2 else math.cos(2.0 * math.pi * u2))
        x = mu[comp, j] + math.exp(ls[comp, j]) * z
        q[j] = lo[j] + 0.5 * (x + 1.0) * (hi[j] - lo[j])
    return q, comp, gap
