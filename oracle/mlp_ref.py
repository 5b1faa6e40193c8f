"""Float64 reference of the warm-start network (test infrastructure only).

Network: 4 -> 32 -> 32 -> 1, ReLU after every layer (so the predicted dual is
nonnegative).  Loss: mean squared error of the output, where the output
ReLU passes the gradient for rows with a positive target (so that a unit
clamped at zero can still learn a positive dual); a row with target 0 is
fitted by any output <= 0.  Parameters are one flat float32 vector:
W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3[1] (1249 values).

Rounding points (the GPU multiplies bf16 operands and accumulates in fp32;
this reference takes the same bf16 roundings and accumulates in float64):
forward   phi, W1, h1, W2, h2, W3 are rounded to bf16 before they multiply;
backward  delta2 is rounded to bf16 before it meets W2 and h1 (the matrix
          products); delta1 multiplies the rounded phi; biases stay fp32.
With round=False every rounding is skipped (for finite-difference checks).

Features of a metric row (the reading of "3 edge weights + endpoint
degrees"): for the row x_ab <= x_ac + x_bc of triplet (a,b,c) with long side
(a,b): (s_ab w_ab, s_ac w_ac, s_bc w_bc, (deg_a + deg_b) / (2 mean deg)),
s = +1 for a positive pair (d = 0) and -1 for a negative one.
"""
from __future__ import annotations

import numpy as np

NPARAM = 32 * 4 + 32 + 32 * 32 + 32 + 32 + 1


def bf16(a):
    """Round float64/float32 values to the nearest bfloat16 (ties to even),
    returned as float64.  bfloat16 keeps the top 16 bits of an IEEE float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == NPARAM
    o = 0
    W1 = p[o:o + 128].reshape(32, 4); o += 128
    b1 = p[o:o + 32]; o += 32
    W2 = p[o:o + 1024].reshape(32, 32); o += 1024
    b2 = p[o:o + 32]; o += 32
    W3 = p[o:o + 32]; o += 32
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, W3, [b3]])


def forward(params, phi, round=True):
    """phi: [N, 4].  Returns y [N] and the intermediates."""
    rb = bf16 if round else (lambda v: np.asarray(v, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(params)
    phib = rb(phi)
    z1 = phib @ rb(W1).T + b1
    h1 = rb(np.maximum(z1, 0.0))
    z2 = h1 @ rb(W2).T + b2
    h2 = rb(np.maximum(z2, 0.0))
    z3 = h2 @ rb(W3) + b3
    y = np.maximum(z3, 0.0)
    return y, dict(phib=phib, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3)


def loss_and_grad(params, phi, target, weight=None, round=True):
    """Mean squared error over N samples (sample weights optional, each
    sample's term scaled by weight / N) and its gradient with respect to
    the float32 master parameters."""
    rb = bf16 if round else (lambda v: np.asarray(v, dtype=np.float64))
    phi = np.asarray(phi, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    N = phi.shape[0]
    wgt = np.ones(N) if weight is None else np.asarray(weight, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(params)
    y, c = forward(params, phi, round)
    # squared error of the ReLU output; the output ReLU passes the gradient
    # where the target is positive
    pos = t > 0
    r = np.where(pos, c["z3"] - t, y)
    loss = float(np.sum(wgt * r ** 2) / N)
    d3 = wgt * 2.0 * r / N * (pos | (c["z3"] > 0))
    gW3 = d3 @ c["h2"]
    gb3 = d3.sum()
    d2 = np.outer(d3, rb(W3)) * (c["z2"] > 0)
    d2b = rb(d2)
    gW2 = d2b.T @ c["h1"]
    gb2 = d2.sum(0)
    dh1 = d2b @ rb(W2)
    d1 = dh1 * (c["z1"] > 0)
    gW1 = d1.T @ c["phib"]
    gb1 = d1.sum(0)
    return loss, pack(gW1, gb1, gW2, gb2, gW3, gb3)


def features(d, w, deg, i, j, k, o):
    """Features of metric rows: triplets (i<j<k) and orientations o (arrays)."""
    d = np.asarray(d)
    w = np.asarray(w, dtype=np.float64)
    deg = np.asarray(deg, dtype=np.float64)
    i, j, k, o = (np.asarray(v, dtype=np.int64) for v in (i, j, k, o))
    pid = lambda a, b: b * (b - 1) // 2 + a
    pij, pik, pjk = pid(i, j), pid(i, k), pid(j, k)
    # long side, then the sides at its first and second endpoint
    L = np.select([o == 0, o == 1], [pij, pik], pjk)
    S1 = np.select([o == 0, o == 1], [pik, pij], pij)
    S2 = np.select([o == 0, o == 1], [pjk, pjk], pik)
    a = np.select([o == 0, o == 1], [i, i], j)
    bnode = np.select([o == 0, o == 1], [j, k], k)
    sgn = lambda p: np.where(d[p] == 0, 1.0, -1.0) * w[p]
    mean_deg = deg.mean() if deg.size else 1.0
    f3 = (deg[a] + deg[bnode]) / (2.0 * mean_deg) if mean_deg > 0 else np.zeros(i.shape)
    return np.stack([sgn(L), sgn(S1), sgn(S2), f3], axis=1)


def init_params(seed):
    """He-style initialisation (used by tests that need a generic network)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, np.sqrt(2 / 4), (32, 4))
    W2 = rng.normal(0, np.sqrt(2 / 32), (32, 32))
    W3 = rng.normal(0, np.sqrt(2 / 32), 32)
    return pack(W1, rng.normal(0, 0.1, 32), W2, rng.normal(0, 0.1, 32), W3, 0.1).astype(np.float32)
