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


def test_sigmoid_output_range():
    p = _params()
    y, _ = M.forward(p, np.random.default_rng(2).standard_normal((50, M.NF)) * 10)
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
