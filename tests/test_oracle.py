"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: printed
worked examples (Figs. 2 and 5), closed forms (separator counts and
lengths of the grid bisection), textbook routines (LAPACK LU, SciPy's
pivoted QR, dense solves), exact invariants (remainder decoupling, exact
zero couplings between segments of one separator), and the error bounds of
the method (Section 4.4)."""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import dense, philox, spalu
from oracle.nd import nd_order
from workloads import make_config, laplacian_2d, laplacian_3d, helmholtz_2d, convection_diffusion_2d

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(t, n):
    return sp.csr_matrix((t[2], t[1], t[0]), shape=(n, n))


# ----------------------------------------------------------------- Philox
def test_philox_known_answers():
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert philox.philox4x32_10(w[0:4], w[4:6]) == tuple(w[6:10])
        out = philox.philox4x32_10_np(*[np.array([x], dtype=np.uint64) for x in w[0:6]])
        assert tuple(int(o[0]) for o in out) == tuple(w[6:10])


def test_gaussian_moments():
    g = philox.gaussian(7, 3, 0, np.arange(64), np.arange(4000), 5, np.zeros(4000, np.int64))
    assert abs(g.mean()) < 0.01
    assert abs(g.std() - 1.0) < 0.01
    # entries depend only on their coordinates
    g2 = philox.gaussian(7, 3, 0, np.arange(8, 16), np.arange(100, 200), 5, np.zeros(100, np.int64))
    assert np.array_equal(g2, g[8:16, 100:200])


# ----------------------------------------------------------------- ND
def test_fig2a_level1_separator():
    nd = nd_order((7, 7), 1)
    sep = nd.perm[nd.node_begin[2]:nd.node_begin[2] + nd.node_size[2]]
    assert sorted(sep % 7) == [3] * 7
    left = nd.perm[:nd.node_size[0]]
    right = nd.perm[nd.node_size[0]:nd.node_size[0] + nd.node_size[1]]
    assert set(left % 7) == {0, 1, 2} and set(right % 7) == {4, 5, 6}


def test_fig5_nd_7x7_L3():
    nd = nd_order((7, 7), 3)
    lv = nd.node_level
    sizes = {l: int(nd.node_size[lv == l].sum()) for l in (1, 2, 3, 4)}
    assert sizes == {1: 7, 2: 6, 3: 12, 4: 24}
    assert (lv == 4).sum() == 8 and set(nd.node_size[lv == 4]) == {3}
    def verts(l):
        out = []
        for k in np.nonzero(lv == l)[0]:
            out += list(nd.perm[nd.node_begin[k]:nd.node_begin[k] + nd.node_size[k]])
        return np.array(out)
    v1, v2, v3 = verts(1), verts(2), verts(3)
    assert set(v1 % 7) == {3}
    assert set(v2 // 7) == {3} and set(v2 % 7) == {0, 1, 2, 4, 5, 6}
    assert set(v3 % 7) == {1, 5} and set(v3 // 7) == {0, 1, 2, 4, 5, 6}


@pytest.mark.parametrize("m", [4, 6, 8])
def test_bisection_closed_form_2d(m):
    n = 2 ** m - 1
    nd = nd_order((n, n))
    assert nd.L == 2 * (m - 3)
    for l in range(1, nd.L + 1):
        k = np.nonzero(nd.node_level == l)[0]
        assert len(k) == 2 ** (l - 1)
        assert set(nd.node_size[k]) == {2 ** (m - l // 2) - 1}
    leaves = nd.node_level == nd.L + 1
    assert leaves.sum() == 2 ** nd.L and set(nd.node_size[leaves]) == {49}
    assert np.array_equal(np.sort(nd.perm), np.arange(n * n))


def test_bisection_closed_form_3d():
    nd = nd_order((15, 15, 15))
    assert nd.L == 3
    assert list(nd.node_size[nd.node_level == 1]) == [225]
    assert list(nd.node_size[nd.node_level == 2]) == [105, 105]
    assert list(nd.node_size[nd.node_level == 3]) == [49] * 4
    assert np.array_equal(np.sort(nd.perm), np.arange(15 ** 3))


def test_etree_parents():
    nd = nd_order((31, 31))
    for k, p in enumerate(nd.node_parent):
        if p < 0:
            assert nd.node_level[k] == 1
        else:
            assert nd.node_level[p] == (nd.node_level[k] - 1 if nd.node_level[k] <= nd.L else nd.L)


def test_segment_split_of_a_separator():
    """Section 2.3.1 / Fig. 3: a lower-level separator cuts a separator into
    two regular segments and one junction."""
    nd = nd_order((63, 63))
    lv = nd.levels[2]
    root = [s for s in lv.segs if s.sep_level == 1]
    assert sorted(len(s.verts) for s in root) == [1, 31, 31]
    assert sum(s.regular for s in root) == 2


@pytest.mark.parametrize("dims", [(15, 15), (31, 15), (15, 15, 7)])
def test_segment_couplings_cover_exact_schur(dims):
    """Every nonzero of the exact level-l Schur complement lies in a block
    listed as coupled, and two regular segments of one separator are not
    coupled (Section 2.3.1)."""
    if len(dims) == 2:
        A = _csr(laplacian_2d(*dims), dims[0] * dims[1]).toarray()
    else:
        A = _csr(laplacian_3d(*dims), int(np.prod(dims))).toarray()
    nd = nd_order(dims)
    for l in range(nd.L, 0, -1):
        lvl = nd.levels[l]
        keep = np.nonzero(lvl.seg_of >= 0)[0]
        elim = np.nonzero(lvl.seg_of < 0)[0]
        S = A[np.ix_(keep, keep)] - A[np.ix_(keep, elim)] @ np.linalg.solve(
            A[np.ix_(elim, elim)], A[np.ix_(elim, keep)])
        seg = lvl.seg_of[keep]
        pairs = set(lvl.pairs)
        nz = np.abs(S) > 1e-9 * np.abs(S).max()
        ii, jj = np.nonzero(nz)
        for a, b in set(zip(seg[ii].tolist(), seg[jj].tolist())):
            assert (a, b) in pairs
        for a, sa in enumerate(lvl.segs):
            for b, sb in enumerate(lvl.segs):
                if a != b and sa.sep_node == sb.sep_node and sa.regular and sb.regular:
                    assert (a, b) not in pairs


# ----------------------------------------------------------------- dense
def test_lu_window_matches_lapack():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((23, 23))
    LU, piv = dense.lu_window(M)
    lu2, piv2 = sla.lu_factor(M)
    assert np.array_equal(piv, piv2)
    assert np.allclose(LU, lu2, rtol=1e-12, atol=1e-13)
    X = rng.standard_normal((23, 3))
    assert np.allclose(dense.lu_solve(LU, piv, X), np.linalg.solve(M, X), rtol=1e-10)


def test_lu_window_keeps_remainder_rows():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((12, 12))
    LU, piv = dense.lu_window(M, split=5)
    assert all(piv[j] < 5 for j in range(5)) and all(piv[j] >= j for j in range(12))
    P = dense.apply_row_pivots(piv, np.eye(12))
    L = np.tril(LU, -1) + np.eye(12)
    U = np.triu(LU)
    assert np.allclose(P @ M, L @ U, atol=1e-12)


def test_cpqr_matches_scipy_pivots():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((40, 15)) * np.logspace(0, -3, 15)[None, :] @ rng.standard_normal((15, 15))
    k, perm, T, r11 = dense.cpqr_id(Y, 0.0)
    _, R, p = sla.qr(Y, pivoting=True, mode="economic")
    assert np.array_equal(perm, p)
    assert abs(r11 - abs(R[0, 0])) < 1e-12 * r11


def test_cpqr_exact_rank():
    rng = np.random.default_rng(3)
    for k0 in (1, 4, 9):
        Y = rng.standard_normal((30, k0)) @ rng.standard_normal((k0, 14))
        k, perm, T, r11 = dense.cpqr_id(Y, 1e-10)
        assert k == k0
        err = Y[:, perm[k:]] - Y[:, perm[:k]] @ T
        assert np.abs(err).max() <= 1e-12 * np.abs(Y).max()


def test_cpqr_gu_eisenstat_bracket():
    """|R_{k+1,k+1}| brackets sigma_{k+1} within sqrt(1 + n k (n-k))
    (eq. (4.15)); sigma_k(R_11) >= sigma_k / sqrt(1 + n k (n-k))."""
    rng = np.random.default_rng(4)
    n = 20
    U, _ = np.linalg.qr(rng.standard_normal((50, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -12, n)
    Y = U @ np.diag(s) @ V.T
    eps = 1e-6
    k, perm, T, r11 = dense.cpqr_id(Y, eps)
    bound = math.sqrt(1 + n * k * (n - k))
    Q, R = np.linalg.qr(Y[:, perm])
    assert abs(R[k, k]) <= bound * s[k]
    assert np.linalg.svd(R[:k, :k], compute_uv=False)[-1] >= s[k - 1] / bound


# ----------------------------------------------------------------- factor
def _solve_dense(P):
    A = P.scipy().toarray()
    return np.linalg.solve(A, P.rhs)


@pytest.mark.parametrize("cfg,side", [(0, 7), (0, 15), (0, 31), (1, 31), (2, 31), (4, 31), (3, 7), (3, 15)])
def test_eps0_equals_dense_lu(cfg, side):
    """Compression off: spaLU is exact block LU along the ND tree and must
    reproduce a dense LU solve to 1e-12."""
    P = make_config(cfg, side=side, nrhs=2)
    nd = nd_order(P.dims)
    F = spalu.factor(nd, P.scipy(), spalu.Opts(eps=0.0))
    x = spalu.apply_inverse(F, P.rhs)
    xe = _solve_dense(P)
    assert np.linalg.norm(x - xe) <= 1e-12 * np.linalg.norm(xe)


def test_single_level_is_block_schur():
    """L = 1: one separator, two leaves: the textbook 2x2 block Schur solve."""
    P = make_config(0, side=7, nrhs=1)
    nd = nd_order(P.dims, 1)
    A = P.scipy().toarray()
    F = spalu.factor(nd, P.scipy(), spalu.Opts(eps=1e-3))
    x = spalu.apply_inverse(F, P.rhs)
    s = nd.levels[1].segs[0].verts
    i = np.setdiff1d(np.arange(49), s)
    S = A[np.ix_(s, s)] - A[np.ix_(s, i)] @ np.linalg.solve(A[np.ix_(i, i)], A[np.ix_(i, s)])
    b = P.rhs[:, 0]
    xs = np.linalg.solve(S, b[s] - A[np.ix_(s, i)] @ np.linalg.solve(A[np.ix_(i, i)], b[i]))
    assert np.allclose(x[s, 0], xs, rtol=1e-12)


@pytest.mark.parametrize("eps", [1e-4, 1e-6, 1e-8])
def test_compressed_residual_within_10_eps(eps):
    """With compression on, the direct solve loses about one digit
    (Section 6): R_es <= 10 eps on the 63 x 63 Laplacian."""
    P = make_config(0)
    F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=eps))
    x, it, hist = spalu.solve(F, P.rhs)
    assert hist[0].max() <= 10 * eps


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_compressed_other_families(cfg):
    P = make_config(cfg, side=63, nrhs=2)
    F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=P.eps))
    x, it, hist = spalu.solve(F, P.rhs, tol=1e-10, max_iter=30)
    assert hist[-1].max() <= 1e-10
    if cfg != 4:
        assert hist[0].max() <= 100 * P.eps


def test_remainder_decoupled_and_locality():
    """After sparsification the remainder DOFs of a segment have no
    coupling left (eq. (2.7)), and blocks that do not touch the segment are
    unchanged (A_ff, A_nf stay as they are)."""
    P = make_config(0, side=31)
    nd = nd_order(P.dims)
    F = spalu.factor(nd, P.scipy(), spalu.Opts(eps=1e-6))
    for lev, rec in F.levels.items():
        for s, lst in rec.sep_coup.items():
            for (d, Ads, Asd) in lst:
                assert Ads.shape == (len(rec.segs[d].skel), len(rec.segs[s].skel))
                assert Asd.shape == (len(rec.segs[s].skel), len(rec.segs[d].skel))


def test_error_bound_eq_4_14():
    """||A - W~^{-1} V~^{-1}|| <= prod_l (1+||T_l||)^2 eps ||A|| on a tiny grid."""
    P = make_config(0, side=15)
    A = P.scipy().toarray()
    eps = 1e-4
    F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=eps))
    Minv = spalu.apply_inverse(F, np.eye(A.shape[0]))
    Aapprox = np.linalg.inv(Minv)
    prod = 1.0
    for lev, rec in F.levels.items():
        t = max([np.linalg.norm(r.T, 2) for r in rec.segs if r.sparsified and r.T.size] + [0.0])
        prod *= (1 + t) ** 2
    assert np.linalg.norm(A - Aapprox, 2) <= prod * eps * np.linalg.norm(A, 2)


def test_symmetric_input_symmetric_solution_operator():
    """For symmetric A the stacked ID (eq. (4.12)) uses the same skeleton for
    rows and columns; the inverse operator is then close to symmetric."""
    P = make_config(0, side=15)
    F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=1e-8))
    M = spalu.apply_inverse(F, np.eye(225))
    assert np.linalg.norm(M - M.T) <= 1e-6 * np.linalg.norm(M)


def _dense_work(F):
    w = 0.0
    for (I, LU, piv) in F.leaves:
        w += len(I) ** 3
    for rec in F.levels.values():
        for r in rec.segs:
            w += len(r.dofs) ** 3
        for s, lst in rec.sep_coup.items():
            ks = len(rec.segs[s].skel)
            kd = sum(len(rec.segs[d].skel) for d, _, _ in lst)
            w += 2.0 * kd * kd * ks
    return w


@pytest.mark.slow
def test_factor_cost_near_linear():
    """O(N) factor cost (Section 5.2): with compression the log-log slope of
    the dense work is <= 1.15 and falls as N grows, while plain nested
    dissection (eps = 0) climbs toward its O(N^{3/2})."""
    def slopes(eps):
        ns, ws = [], []
        for side in (63, 127, 255):
            P = make_config(0, side=side)
            F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=eps))
            ns.append(side * side)
            ws.append(_dense_work(F))
        return np.diff(np.log(ws)) / np.diff(np.log(ns))
    s = slopes(1e-4)
    assert s[-1] <= 1.15 and s[-1] < s[0]
    s0 = slopes(0.0)
    assert s0[-1] >= 1.35 and s0[-1] > s0[0]
