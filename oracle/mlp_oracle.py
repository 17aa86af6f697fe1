"""CPU oracle of the learned insertion proposal -- TEST INFRASTRUCTURE ONLY.

Not part of the paper's method: an extension that keeps its statistics.  A
multilayer perceptron maps the 16^3 occupancy grid of a configuration to a
4096-bin categorical over insertion voxels; a trial position is a voxel drawn from
it plus a uniform offset inside the voxel (mixed with uniform insertion), and the
proposal density enters the Metropolis-Hastings acceptance:
    insertion  A = min[1, z exp(-beta dE) / ((N+1) q(r | X))],
    removal    A = min[1, N q(r_i | X without i) exp(-beta dE) / z],
    q(r | X) = alpha P(v(r) | occ(X)) / V_vox + (1 - alpha) / V.
Network: occ (4096) -> 128 -> 128 -> 128 -> 4096, GELU (erf form) after the three
hidden layers, log-softmax output.  Training: cross-entropy of the voxel of a
removed particle given the occupancy of the other particles; Adam.

Two arithmetic paths:
  fp64 -- everything in double (the reference for gradients and probabilities);
  bf16 -- the rounding points of the GPU kernels: weights and hidden activations
          rounded to bfloat16 (round to nearest even) before each product, sums and
          softmax in float32.
Only tests and benchmark baselines use this module.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

GRID = 16
NV = GRID ** 3
H = 128


# ---------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def voxel_of(xyz, lx, ly, zlo, zhi, g: int = GRID) -> np.ndarray:
    """Voxel index (iz * g + iy) * g + ix of positions, cells of the gas region
    [0,lx) x [0,ly) x [zlo,zhi] cut g ways per axis, indices clamped to the grid."""
    p = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    ix = np.clip(np.floor(p[:, 0] * (g / lx)).astype(np.int64), 0, g - 1)
    iy = np.clip(np.floor(p[:, 1] * (g / ly)).astype(np.int64), 0, g - 1)
    iz = np.clip(np.floor((p[:, 2] - zlo) * (g / (zhi - zlo))).astype(np.int64), 0, g - 1)
    return (iz * g + iy) * g + ix


# ---------------------------------------------------------------------------
def forward(params, voxels, n, excl, mode: str = "fp64"):
    """Batch forward.  voxels [B][nmax] (voxel of each particle), n [B], excl [B]
    (index of the particle left out of the occupancy, -1 for none).  Returns a dict
    of pre-activations a1..a3, activations h1..h3 and logits [B][NV]."""
    f = np.float64 if mode == "fp64" else np.float32
    rd = (lambda x: np.asarray(x, np.float64)) if mode == "fp64" else bf16_round
    W1, W2, W3, W4 = (rd(params[k]) for k in ("W1", "W2", "W3", "W4"))
    b1, b2, b3, b4 = (np.asarray(params[k], f) for k in ("b1", "b2", "b3", "b4"))
    B = len(n)
    a1 = np.zeros((B, H), f)
    for b in range(B):
        acc = b1.astype(f).copy()
        for j in range(n[b]):
            if j != excl[b]:
                acc = (acc + W1[voxels[b][j]].astype(f)).astype(f)
        a1[b] = acc
    h1 = rd(gelu(a1).astype(f))
    a2 = (h1.astype(f) @ W2.T.astype(f) + b2).astype(f)
    h2 = rd(gelu(a2).astype(f))
    a3 = (h2.astype(f) @ W3.T.astype(f) + b3).astype(f)
    h3 = rd(gelu(a3).astype(f))
    logits = (h3.astype(f) @ W4.T.astype(f) + b4).astype(f)
    return {"a1": a1, "h1": h1, "a2": a2, "h2": h2, "a3": a3, "h3": h3, "logits": logits}


def log_softmax(logits):
    m = logits.max(axis=1, keepdims=True)
    return logits - m - np.log(np.exp(logits - m).sum(axis=1, keepdims=True))


def loss_and_grads(params, voxels, n, excl, target, mode: str = "fp64"):
    """Mean cross-entropy of the target voxels and its gradient with respect to every
    parameter (same shapes as params)."""
    f = np.float64 if mode == "fp64" else np.float32
    rd = (lambda x: np.asarray(x, np.float64)) if mode == "fp64" else bf16_round
    fw = forward(params, voxels, n, excl, mode)
    B = len(n)
    lp = log_softmax(fw["logits"].astype(f)).astype(f)
    loss = float(-lp[np.arange(B), target].mean())
    p = np.exp(lp).astype(f)
    d = p.copy()
    d[np.arange(B), target] -= 1.0
    d = (d / B).astype(f)
    g = {"b4": d.sum(0).astype(f)}
    dq = rd(d)
    W2, W3, W4 = (rd(params[k]) for k in ("W2", "W3", "W4"))
    g["W4"] = (dq.T.astype(f) @ fw["h3"].astype(f)).astype(f)
    dh3 = (dq.astype(f) @ W4.astype(f)).astype(f)
    da3 = (dh3 * gelu_grad(fw["a3"]).astype(f)).astype(f)
    g["b3"] = da3.sum(0).astype(f)
    da3q = rd(da3)
    g["W3"] = (da3q.T.astype(f) @ fw["h2"].astype(f)).astype(f)
    dh2 = (da3q.astype(f) @ W3.astype(f)).astype(f)
    da2 = (dh2 * gelu_grad(fw["a2"]).astype(f)).astype(f)
    g["b2"] = da2.sum(0).astype(f)
    da2q = rd(da2)
    g["W2"] = (da2q.T.astype(f) @ fw["h1"].astype(f)).astype(f)
    dh1 = (da2q.astype(f) @ W2.astype(f)).astype(f)
    da1 = (dh1 * gelu_grad(fw["a1"]).astype(f)).astype(f)
    g["b1"] = da1.sum(0).astype(f)
    W1g = np.zeros((NV, H), f)
    for b in range(B):
        for j in range(n[b]):
            if j != excl[b]:
                W1g[voxels[b][j]] += da1[b]
    g["W1"] = W1g
    return loss, g


def adam(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) with bias correction, in place; state holds
    m, v per parameter and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] * grads[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def log_q(params, voxels, n, excl, query_voxel, alpha, v_total, mode: str = "fp64"):
    """ln q of a position in query_voxel for each example: the mixture
    alpha P(v | occ) / V_vox + (1 - alpha) / V."""
    fw = forward(params, voxels, n, excl, mode)
    lp = log_softmax(fw["logits"].astype(np.float64))
    v_vox = v_total / NV
    pv = np.exp(lp[np.arange(len(n)), query_voxel])
    return np.log(alpha * pv / v_vox + (1.0 - alpha) / v_total), lp
