"""Pins of the rank-predictor oracle: gradients against central finite
differences in FP64, Adam against its defining recurrences, and features
against closed forms of the stencils (Laplace: no wavelengths, zero
asymmetry, unit scaled diagonal; Helmholtz: span * k h / 2 pi)."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from oracle.nd import nd_order
from workloads import make_config
from workloads.pde import helmholtz_2d
import scipy.sparse as sp


def _params(seed=1):
    rng = np.random.default_rng(seed)
    p = M.init_params(rng.standard_normal(M.NF), 1.0 + rng.random(M.NF), seed)
    p[M.OFF_B1:M.OFF_W2] = 0.1 * rng.standard_normal(M.H)
    p[M.OFF_B2:M.OFF_W3] = 0.1 * rng.standard_normal(M.H)
    return p


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = _params()
    X = rng.standard_normal((17, M.NF))
    t = rng.random(17)
    loss, g = M.loss_and_grad(p, X, t)
    idx = list(range(M.OFF_W1, M.OFF_W1 + 20)) + list(range(M.OFF_B1, M.OFF_B1 + 5)) + \
        list(range(M.OFF_W2, M.OFF_W2 + 20)) + list(range(M.OFF_W3, M.NPARAM))
    for i in idx:
        hstep = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += hstep
        pm[i] -= hstep
        fd = (M.loss_and_grad(pp, X, t)[0] - M.loss_and_grad(pm, X, t)[0]) / (2 * hstep)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9
    assert np.all(g[:M.OFF_W1] == 0.0)


def test_adam_recurrence_and_frozen_normalisation():
    p = _params()
    g = np.random.default_rng(0).standard_normal(M.NPARAM)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    p1, m1, v1 = M.adam_step(p, g, m, v, 1, lr=1e-2, eps=0.0)
    # first step of Adam moves every trainable entry by lr * sign(g)
    d = (p1 - p)[M.OFF_W1:]
    assert np.allclose(d, -1e-2 * np.sign(g[M.OFF_W1:]), rtol=1e-6)
    assert np.array_equal(p1[:M.OFF_W1], p[:M.OFF_W1])


def test_forward_closed_form():
    """A hand-set network: standardisation, the orientation of W1 and W2
    (row = output unit), both ReLUs, the output weights and the sigmoid each
    change the value in a way that is written out here."""
    p = np.zeros(M.NPARAM)
    mu = np.arange(M.NF, dtype=float)
    sd = np.full(M.NF, 2.0)
    p[M.OFF_MU:M.OFF_MU + M.NF] = mu
    p[M.OFF_SD:M.OFF_SD + M.NF] = sd
    W1 = np.zeros((M.H, M.NF))
    W1[1, 3] = 1.0          # hidden unit 1 reads feature 3
    W1[2, 5] = -1.0         # hidden unit 2 reads minus feature 5
    b1 = np.zeros(M.H)
    b1[2] = 0.25
    W2 = np.zeros((M.H, M.H))
    W2[4, 1] = 2.0          # unit 4 of layer 2 reads unit 1 of layer 1
    W2[4, 2] = 1.0
    W2[6, 1] = -1.0         # unit 6 is negative whenever unit 1 is positive
    b2 = np.zeros(M.H)
    b2[6] = 0.5
    w3 = np.zeros(M.H)
    w3[4] = 3.0
    w3[6] = -2.0
    p[M.OFF_W1:M.OFF_B1] = W1.ravel()
    p[M.OFF_B1:M.OFF_W2] = b1
    p[M.OFF_W2:M.OFF_B2] = W2.ravel()
    p[M.OFF_B2:M.OFF_W3] = b2
    p[M.OFF_W3:M.OFF_B3] = w3
    p[M.OFF_B3] = -1.0
    X = np.tile(mu, (4, 1))
    X[0, 3] = mu[3] + 2.0     # xn3 = 1: h1 = 1, h2 = relu(0.25) = .25
    X[0, 5] = mu[5] + 0.0     #          z2_4 = 2.25, z2_6 = -0.5 -> 0
    X[1, 3] = mu[3] - 2.0     # xn3 = -1: h1 = 0; xn5 = 0: h2 = .25
    X[2, 5] = mu[5] + 1.0     # xn5 = .5: h2 = relu(-.25) = 0, h1 = 0
    X[3, 3] = mu[3] + 0.5     # xn3 = .25: h1 = .25, h2 = .25; z2_6 = .25
    z = np.array([3 * 2.25 - 1.0,
                  3 * 0.25 - 2 * 0.5 - 1.0,
                  -2 * 0.5 - 1.0,
                  3 * 0.75 - 2 * 0.25 - 1.0])
    y, _ = M.forward(p, X)
    assert np.allclose(y, 1.0 / (1.0 + np.exp(-z)), rtol=1e-15, atol=0)
    assert np.all((y > 0) & (y < 1))


def test_features_closed_forms():
    P = make_config(0, side=31)
    nd = nd_order(P.dims)
    lev = nd.L
    cur = {c: sg.verts for c, sg in enumerate(nd.levels[lev].segs)}
    A = P.scipy()
    for c, sg in enumerate(nd.levels[lev].segs):
        f = M.segment_features(nd, A, lev, c, cur, 1e-6)
        assert f[0] == math.log2(len(sg.verts) + 1)
        assert f[2] == 0.0 and f[11] == 0.0
        assert abs(f[9]) < 1e-12 and abs(f[10]) < 1e-12
        assert f[5] == 1.0 and abs(f[6] - 6.0 / 16.0) < 1e-15
    # Helmholtz: an interior vertex gives kh2 = (kh)^2 exactly
    n = 31
    k = 2 * math.pi / (10 / (n + 1))
    ip, ix, dv = helmholtz_2d(n, k=k)
    A = sp.csr_matrix((dv, ix, ip), shape=(n * n, n * n))
    h = 1.0 / (n + 1)
    sg = nd.levels[lev].segs[0]
    c = 0
    f = M.segment_features(nd, A, lev, c, cur, 1e-6)
    span = max(b - a + 1 for a, b in zip(sg.bbox_lo, sg.bbox_hi))
    assert abs(f[2] - span * k * h / (2 * math.pi)) <= 1e-9 * f[2]
