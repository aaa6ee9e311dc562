"""Oracle: the segment-rank predictor (features, MLP forward / backward,
Adam), FP64 NumPy.  TEST INFRASTRUCTURE ONLY (see the package docstring).

The predictor replaces the adaptive sample count of the hybrid sampling
(Section 4.2.3 takes h = k + p with k unknown): from 12 features of a
segment it predicts the rank fraction k/n, and the sampler starts with
h = ceil(margin * n * yhat) + p samples; the a-posteriori check of the ID
still judges the result and falls back to doubling h.

Features of segment c at level l (current DOFs before its ID):
  f0  log2(n + 1)                  n: current size
  f1  log2(span)                   span: longest bounding-box side (vertices)
  f2  span * sqrt(kh2) / (2 pi)    wavelengths across the segment, where
                                   kh2 = max(0, max_v (S_v - a_vv) * m_v / S_v),
                                   S_v = sum |a_vj| (j != v), m_v = #those j
  f3  log2(nV + 1)                 nV: current DOFs of all coupled segments
  f4  near fraction                near rows / all 2 nV stacked rows
  f5  l / L
  f6  log10(1 / eps) / 16           eps: the ID tolerance
  f7  1 if the segment lies on a level-l separator
  f8  1 if its bounding box touches the grid boundary
  f9  mean of g_v = log(a_vv h^2 / (2 dim)) over its current DOFs
  f10 standard deviation of g_v
  f11 mean over its DOFs of sum_j |a_vj - a_jv| / sum_j (|a_vj| + |a_jv|)

Parameter vector (float): mu[12], sd[12] (input standardisation), then
W1[64x12], b1[64], W2[64x64], b2[64], w3[64], b3[1].
"""
from __future__ import annotations

import math

import numpy as np

NF = 12
H = 64
OFF_MU = 0
OFF_SD = 12
OFF_W1 = 24
OFF_B1 = OFF_W1 + H * NF
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
NPARAM = OFF_B3 + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    return dict(mu=p[OFF_MU:OFF_MU + NF], sd=p[OFF_SD:OFF_SD + NF],
                W1=p[OFF_W1:OFF_B1].reshape(H, NF), b1=p[OFF_B1:OFF_W2],
                W2=p[OFF_W2:OFF_B2].reshape(H, H), b2=p[OFF_B2:OFF_W3],
                w3=p[OFF_W3:OFF_B3], b3=p[OFF_B3])


def init_params(mu, sd, seed=0):
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    p[OFF_MU:OFF_MU + NF] = mu
    p[OFF_SD:OFF_SD + NF] = sd
    p[OFF_W1:OFF_B1] = rng.standard_normal(H * NF) * math.sqrt(2.0 / NF)
    p[OFF_W2:OFF_B2] = rng.standard_normal(H * H) * math.sqrt(2.0 / H)
    p[OFF_W3:OFF_B3] = rng.standard_normal(H) * math.sqrt(1.0 / H)
    return p


def forward(p, X):
    """yhat for the rows of X (B x 12) and the intermediate activations."""
    q = unpack(p)
    Xn = (np.asarray(X, np.float64) - q["mu"]) / q["sd"]
    Z1 = Xn @ q["W1"].T + q["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ q["W2"].T + q["b2"]
    H2 = np.maximum(Z2, 0.0)
    z = H2 @ q["w3"] + q["b3"]
    y = 1.0 / (1.0 + np.exp(-z))
    return y, dict(Xn=Xn, H1=H1, H2=H2, y=y)


def loss_and_grad(p, X, t):
    """Mean squared error of yhat against targets t, and its gradient with
    respect to the trainable parameters (mu, sd entries of the gradient are 0)."""
    q = unpack(p)
    y, c = forward(p, X)
    B = len(t)
    r = y - t
    loss = float(np.mean(r * r))
    dz = (2.0 / B) * r * y * (1.0 - y)
    g = np.zeros_like(np.asarray(p, np.float64))
    g[OFF_W3:OFF_B3] = c["H2"].T @ dz
    g[OFF_B3] = dz.sum()
    dH2 = np.outer(dz, q["w3"]) * (c["H2"] > 0)
    g[OFF_W2:OFF_B2] = (dH2.T @ c["H1"]).ravel()
    g[OFF_B2:OFF_W3] = dH2.sum(axis=0)
    dH1 = (dH2 @ q["W2"]) * (c["H1"] > 0)
    g[OFF_W1:OFF_B1] = (dH1.T @ c["Xn"]).ravel()
    g[OFF_B1:OFF_W2] = dH1.sum(axis=0)
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) of the trainable entries."""
    mask = np.ones_like(p)
    mask[:OFF_W1] = 0.0
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - mask * lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def segment_features(nd, A, lev, c, cur, eps):
    """The 12 features of segment c of level lev given the current DOF lists
    ``cur`` (segment -> vertex ids) of that level (see the module docstring)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    lvl = nd.levels[lev]
    seg = lvl.segs[c]
    dofs = np.asarray(cur[c], dtype=np.int64)
    n = len(dofs)
    lo, hi = np.array(seg.bbox_lo), np.array(seg.bbox_hi)
    span = int((hi - lo + 1).max())
    dims = np.array(nd.dims)
    h = 1.0 / (max(nd.dims) + 1)
    kh2 = 0.0
    g = []
    asym = []
    for v in dofs:
        row = A.getrow(v)
        S, m, diag = 0.0, 0, 0.0
        num, den = 0.0, 0.0
        for j, a in zip(row.indices, row.data):
            if j == v:
                diag = a
            else:
                S += abs(a)
                m += 1
                at = A[j, v]
                num += abs(a - at)
                den += abs(a) + abs(at)
        if S > 0:
            kh2 = max(kh2, (S - diag) * m / S)
        g.append(math.log(abs(diag) * h * h / (2 * nd.dim)) if diag != 0 else 0.0)
        asym.append(num / den if den > 0 else 0.0)
    nbrs = [d for (a, d) in lvl.pairs if a == c and d != c]
    nV = sum(len(cur[d]) for d in nbrs)
    thr = None
    near = 0
    if nV:
        from .spalu import _cheb_to_box, _coords
        thr = max(1, int(math.ceil(0.5 * span)))
        for d in nbrs:
            if len(cur[d]):
                near += 2 * int((_cheb_to_box(_coords(nd, cur[d]), lo, hi) <= thr).sum())
    touches = bool(np.any(lo[:nd.dim] == 0) or np.any(hi[:nd.dim] == dims[:nd.dim] - 1))
    L = nd.L
    gm = float(np.mean(g)) if g else 0.0
    gs = float(np.std(g)) if g else 0.0
    return np.array([math.log2(n + 1), math.log2(span), span * math.sqrt(kh2) / (2 * math.pi),
                     math.log2(nV + 1), near / (2 * nV) if nV else 0.0, lev / L,
                     math.log10(1.0 / eps) / 16.0,
                     1.0 if seg.is_sep else 0.0, 1.0 if touches else 0.0, gm, gs,
                     float(np.mean(asym)) if asym else 0.0])
