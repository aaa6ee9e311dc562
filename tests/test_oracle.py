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


def test_uniform53_bit_window():
    """The uniform of two Philox words uses bits 63..11 of hi:lo: bit 11 is
    the lowest counted bit (one step of 2^-53), bits 10..0 are dropped, the
    top bit is worth 1/2, and half a step keeps the value away from 0."""
    u = philox.uniform53
    assert u(0, 0) == 2.0 ** -54
    assert u(0, (1 << 11) - 1) == 2.0 ** -54
    assert u(0, 1 << 11) == 2.0 ** -53 + 2.0 ** -54
    assert u(1 << 31, 0) == 0.5 + 2.0 ** -54
    assert u(1, 0) == 2.0 ** -32 + 2.0 ** -54
    assert u(0xFFFFFFFF, 0xFFFFFFFF) == 1.0          # 1 - 2^-54 rounds to 1


def test_gaussian_law():
    """Entries of G follow N(0, 1) (Kolmogorov-Smirnov, also for even and odd
    rows apart); the two entries of one draw are independent normals, so
    their squared radius / 2 is Exp(1) and their angle is uniform; entries
    depend only on their coordinates."""
    from scipy import stats
    g = philox.gaussian(7, 3, 0, np.arange(64), np.arange(4000), 5, np.zeros(4000, np.int64))
    assert stats.kstest(g.ravel(), "norm").pvalue > 1e-3
    assert stats.kstest(g[0::2].ravel(), "norm").pvalue > 1e-3
    assert stats.kstest(g[1::2].ravel(), "norm").pvalue > 1e-3
    ev, od = g[0::2].ravel(), g[1::2].ravel()
    assert stats.kstest((ev ** 2 + od ** 2) / 2, "expon").pvalue > 1e-3
    assert stats.kstest(np.arctan2(od, ev), stats.uniform(-math.pi, 2 * math.pi).cdf).pvalue > 1e-3
    assert abs(np.corrcoef(ev, od)[0, 1]) < 0.01
    # the other half, segment, stream and level give independent entries
    for args in ((7, 3, 0, 5, 1), (7, 3, 0, 6, 0), (7, 3, 1, 5, 0), (7, 4, 0, 5, 0), (8, 3, 0, 5, 0)):
        s_, l_, st_, c_, h_ = args
        g2 = philox.gaussian(s_, l_, st_, np.arange(64), np.arange(4000), c_, np.full(4000, h_))
        assert abs(np.corrcoef(g.ravel(), g2.ravel())[0, 1]) < 0.01
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


def test_cpqr_tie_rule():
    """Column norms within TIE_REL of the maximum are tied and the smallest
    original column wins, also when that column sits at a later position
    after an earlier swap."""
    a = np.array([1.0, 2.0, 2.0, 0.0, 0.0])
    b = np.array([2.0, 1.0, 0.0, 2.0, 0.0])
    c = np.array([0.0, 0.0, 0.0, 0.0, 9.0])
    # step 0: columns 1 and 3 tie (norm 3), column 1 wins
    Y = np.stack([0.1 * c, a, 0.2 * c, b], axis=1)
    k, perm, T, r11 = dense.cpqr_id(Y, 0.0, max_rank=1)
    assert perm[0] == 1
    # step 0 takes column 3 (norm 9), which moves column 0 to position 3;
    # step 1: columns 0 (position 3) and 2 (position 2) tie, column 0 wins
    Y = np.stack([a, 0.01 * c + 0.0 * a, b, c], axis=1)
    Y[:, 1] = np.array([0.0, 0.0, 0.0, 0.5, 0.0])
    k, perm, T, r11 = dense.cpqr_id(Y, 0.0, max_rank=2)
    assert perm[0] == 3 and perm[1] == 0
    # one part in 1e9 is not a tie: the larger column wins
    Y = np.stack([a, b * (1 + 1e-9)], axis=1)
    k, perm, T, r11 = dense.cpqr_id(Y, 0.0, max_rank=1)
    assert perm[0] == 1


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
    """The loss of about one digit (Section 6) as a normwise backward error
    ||b - A x|| / (||A||_2 ||x||) <= 10 eps for every family, and as the
    relative residual R_es <= 10 eps for the well-conditioned ones (the
    indefinite Helmholtz operator at 10 points per wavelength multiplies
    the residual by its condition number); refinement then reaches 1e-10."""
    P = make_config(cfg, side=63, nrhs=2)
    A = P.scipy()
    F = spalu.factor(nd_order(P.dims), A, spalu.Opts(eps=P.eps))
    x, it, hist = spalu.solve(F, P.rhs, tol=1e-10, max_iter=30)
    assert hist[-1].max() <= 1e-10
    x0 = spalu.apply_inverse(F, P.rhs)
    normA = np.linalg.norm(A.toarray(), 2)
    back = np.linalg.norm(P.rhs - A @ x0, axis=0) / (normA * np.linalg.norm(x0, axis=0))
    assert back.max() <= 10 * P.eps
    if cfg != 4:
        assert hist[0].max() <= 10 * P.eps


def test_compression_stats():
    """q~ = max_l e'_l / e_l (Section 6): no segment is sparsified with
    eps = 0; with compression the per-level maximum sizes satisfy the
    sparsity assumption e'_l <= q e_l + sigma_e with q = 2^(-1/3) and
    sigma_e = 7 (one leaf side: segments that small may stay whole), the
    largest segments shrink, and q~ is the largest ratio."""
    P = make_config(0, side=127)
    nd = nd_order(P.dims)
    F0 = spalu.factor(nd, P.scipy(), spalu.Opts(eps=0.0))
    assert spalu.compression_stats(F0) == ({}, 0.0)
    F = spalu.factor(nd, P.scipy(), spalu.Opts(eps=1e-4))
    st, q = spalu.compression_stats(F)
    for lev, (e, e2) in st.items():
        sizes = [F.levels[lev].n_before[i] for i, r in enumerate(F.levels[lev].segs) if r.sparsified]
        kept = [len(r.skel) for r in F.levels[lev].segs if r.sparsified]
        assert (e, e2) == (max(sizes), max(kept))
        assert e2 <= 2 ** (-1 / 3) * e + 7
    top = max(st, key=lambda l: st[l][0])
    assert st[top][1] < st[top][0]
    assert q == max(e2 / e for e, e2 in st.values())


# ----------------------------------------------------------------- sampled ID
def _id_rows(rng, m_near, m_far, n, k0):
    """Near and far rows of an exact rank-k0 coupling matrix, with far-row
    keys (vertex ids and halves) for the Gaussian entries."""
    C = rng.standard_normal((k0, n)) * np.logspace(0, -1, n)[None, :]
    BN = rng.standard_normal((m_near, k0)) @ C
    BF = rng.standard_normal((m_far, k0)) @ C
    vf = rng.permutation(10 * m_far)[:m_far]
    hf = rng.integers(0, 2, m_far)
    return BN, BF, vf, hf


@pytest.mark.parametrize("m_near", [0, 6])
def test_sampled_id_range_finder(m_near):
    """Randomised range finder (Section 4.2.3; Halko, Martinsson, Tropp
    2011): when the far rows have rank k0 < h, G B_F has the row space of
    B_F, so one pass finds k = k0 and T reconstructs the true far rows (not
    only the sampled ones) and the near rows to rounding."""
    rng = np.random.default_rng(11)
    BN, BF, vf, hf = _id_rows(rng, m_near, 120, 18, 5)
    o = spalu.Opts(eps=1e-10)
    k, perm, T, h, passes, _ = spalu.sampled_id(BN, BF, vf, hf, 3, 7, 8, o)
    assert (k, h, passes) == (5, 8, 1)
    for B in (BF, BN):
        if len(B):
            E = B[:, perm[k:]] - B[:, perm[:k]] @ T
            assert np.abs(E).max() <= 1e-11 * np.abs(B).max()


def test_sampled_id_doubles_until_the_check_passes():
    """Far rows of rank 20 sampled with h = 8 cannot pass the probe check;
    h doubles (8, 16, 32) and the accepted ID reconstructs the far rows."""
    rng = np.random.default_rng(12)
    BN, BF, vf, hf = _id_rows(rng, 0, 200, 30, 20)
    o = spalu.Opts(eps=1e-10)
    k, perm, T, h, passes, _ = spalu.sampled_id(BN, BF, vf, hf, 2, 1, 8, o)
    assert (k, h, passes) == (20, 32, 3)
    E = BF[:, perm[k:]] - BF[:, perm[:k]] @ T
    assert np.abs(E).max() <= 1e-9 * np.abs(BF).max()


def _scipy_id(Y, eps):
    """Pivoted QR ID by LAPACK (scipy): rank = first |R_jj| <= eps |R_00|."""
    _, R, p = sla.qr(Y, pivoting=True, mode="economic")
    d = np.abs(np.diag(R))
    small = np.nonzero(d <= eps * d[0])[0]
    k = int(small[0]) if len(small) else len(d)
    T = sla.solve_triangular(R[:k, :k], R[:k, k:])
    return k, p, T


def test_sampled_id_at_the_cap_is_the_exact_id():
    """With h at the cap (h >= |F|) the ID is taken on the exact rows
    [B_N; B_F], i.e. the unsampled ID: pivots, rank and T equal LAPACK's
    pivoted QR of the stacked matrix (tie-free input)."""
    rng = np.random.default_rng(13)
    BN = rng.standard_normal((9, 16)) * np.logspace(0, -8, 16)[None, :]
    BF = rng.standard_normal((14, 16)) * np.logspace(0, -8, 16)[None, :]
    vf = np.arange(14)
    hf = np.zeros(14, np.int64)
    eps = 1e-5
    k, perm, T, h, passes, _ = spalu.sampled_id(BN, BF, vf, hf, 1, 0, 14, spalu.Opts(eps=eps))
    ks, ps, Ts = _scipy_id(np.vstack([BN, BF]), eps)
    assert (h, passes) == (14, 1)
    assert k == ks and np.array_equal(perm, ps)
    assert np.allclose(T, Ts, rtol=1e-9, atol=1e-12)


def _level_schur(A, nd, lev):
    """Dense Schur complement onto the DOFs that are still present at the
    start of level lev when nothing is compressed (eps = 0): every vertex
    of the leaves and of separators of level > lev is eliminated."""
    A = A.toarray()
    lvl = nd.levels[lev]
    keep = np.nonzero(lvl.seg_of >= 0)[0]
    elim = np.nonzero(lvl.seg_of < 0)[0]
    S = A[np.ix_(keep, keep)] - A[np.ix_(keep, elim)] @ np.linalg.solve(
        A[np.ix_(elim, elim)], A[np.ix_(elim, keep)])
    pos = np.full(A.shape[0], -1)
    pos[keep] = np.arange(len(keep))
    return S, pos


@pytest.mark.parametrize("cfg", [1, 2])
def test_level_L_ids_are_ids_of_the_exact_stacked_couplings(cfg):
    """Stacking (eq. (4.12)): with every row near (rho large) each level-L ID
    is the pivoted QR ID of [S_{n,c}; S_{c,n}^T] taken from the dense Schur
    complement of the leaves (computed here with numpy), for the symmetric
    GRF diffusion and the non-symmetric convection-diffusion matrix (where
    the two halves differ, so a transposed or missing half shows)."""
    P = make_config(cfg, side=31)
    nd = nd_order(P.dims)
    A = P.scipy()
    seen = {}
    o = spalu.Opts(eps=P.eps, rho=1e9, trace=lambda lev, d: seen.setdefault(lev, d))
    spalu.factor(nd, A, o)
    L = nd.L
    S, pos = _level_schur(A, nd, L)
    lvl = nd.levels[L]
    tr = seen[L]
    checked = 0
    for c, sg in enumerate(lvl.segs):
        if c not in tr["ids"]:
            continue
        k, perm, T, h, passes, _ = tr["ids"][c]
        vc = pos[tr["cur"][c]]
        rows = []
        for (a, d) in lvl.pairs:
            if a == c and d != c:
                vd = pos[tr["cur"][d]]
                rows += [S[np.ix_(vd, vc)], S[np.ix_(vc, vd)].T]
        Y = np.vstack(rows)
        ks, ps, Ts = _scipy_id(Y, P.eps)
        assert (k, passes) == (ks, 1)
        _check_pivots(Y, perm, k, ps)
        if np.array_equal(perm, ps):
            assert np.allclose(T, Ts, rtol=1e-7, atol=1e-9)
        if k < len(perm):     # residual columns = those of R_22, each <= eps |R_11|
            E = Y[:, perm[k:]] - Y[:, perm[:k]] @ T
            assert np.linalg.norm(E, axis=0).max() <= P.eps * np.linalg.norm(Y, axis=0).max()
        checked += 1
    assert checked >= 8


def _check_pivots(Y, perm, k, lapack_perm):
    """Each pivot of the first k steps has the largest norm of the columns
    projected off the pivots before it (fresh norms, by an orthogonal
    projection computed here); where LAPACK's pivot order first departs,
    its choice is tied with the oracle's and the oracle took the smaller
    original column."""
    same = True
    for j in range(k):
        if j:
            Q, _ = np.linalg.qr(Y[:, perm[:j]])
            Z = Y - Q @ (Q.T @ Y)
        else:
            Z = Y
        nrm = np.linalg.norm(Z, axis=0)
        nrm[perm[:j]] = 0.0
        mx = nrm.max()
        assert nrm[perm[j]] >= mx * (1 - 1e-10)
        if same and lapack_perm[j] != perm[j]:
            assert nrm[lapack_perm[j]] >= mx * (1 - 1e-10)
            assert perm[j] < lapack_perm[j]
            same = False


def _transform(M, perm, k, T):
    """U_t M L_t of eq. (2.7) as dense products: L_t is the identity except
    (L_t)[s_i, r_j] = -T[i, j] (column r_j := r_j - sum_i T[i, j] s_i) and
    U_t = L_t^T; returned in [remainder; skeleton] order."""
    n = len(perm)
    Lt = np.eye(n)
    Lt[np.ix_(perm[:k], perm[k:])] = -T
    order = np.concatenate([perm[k:], perm[:k]])
    return (Lt.T @ M @ Lt)[np.ix_(order, order)]


@pytest.mark.parametrize("cfg", [2, 4])
def test_sparsify_decouples_the_remainder(cfg):
    """Schur sparsification (eq. (2.7), Section 2.3.2): after the transform
    every coupling of a segment's remainder DOFs to its neighbours is of
    the order of eps (what the method drops), the remainder DOFs never
    appear again (the next level holds skeletons only), and the two-stage
    LU of the transformed diagonal block keeps its pivots inside the
    remainder for the first n_r steps and reproduces the block."""
    P = make_config(cfg, side=63)
    nd = nd_order(P.dims)
    seen = {}
    spalu.factor(nd, P.scipy(), spalu.Opts(eps=P.eps, trace=lambda lev, d: seen.setdefault(lev, d)))
    nchecked = 0
    for lev, tr in seen.items():
        lvl = nd.levels[lev]
        B, cur = tr["blocks"], tr["cur"]
        dropped = set()
        for c, (k, perm, T, h, passes, _) in tr["ids"].items():
            nr = len(perm) - k
            rec = tr["recs"][c]
            assert rec.nr == nr
            nbr = [d for (a, d) in lvl.pairs if a == c and d != c and len(cur[d])]
            Y = np.vstack([np.vstack([B[(d, c)], B[(c, d)].T]) for d in nbr])
            scale = np.linalg.norm(Y, axis=0).max()
            worst = 0.0
            for d in nbr:
                Edc = B[(d, c)][:, perm[k:]] - B[(d, c)][:, perm[:k]] @ T
                Ecd = B[(c, d)][perm[k:], :] - T.T @ B[(c, d)][perm[:k], :]
                worst = max(worst, np.abs(Edc).max(initial=0.0), np.abs(Ecd).max(initial=0.0))
                assert tr["scaled"][(c, d)].shape == (k, len(tr["recs"][d].skel))
            assert worst <= 10 * P.eps * scale
            M2 = _transform(B[(c, c)], perm, k, T)
            LU, piv = rec.LU, rec.piv
            assert np.all(piv[:nr] < nr)
            L = np.tril(LU, -1) + np.eye(len(perm))
            U = np.triu(LU)
            PM = dense.apply_row_pivots(piv, M2)
            assert np.linalg.norm(PM - L @ U) <= 1e-12 * np.linalg.norm(M2)
            dropped |= set(rec.dofs[:nr].tolist())
            nchecked += nr > 0
        if lev - 1 in seen:
            nxt = set(np.concatenate([v for v in seen[lev - 1]["cur"].values()]).tolist())
            assert not (nxt & dropped)
    assert nchecked >= 10


def test_sparsification_is_local_and_simultaneous():
    """Sparsifying a segment changes only the blocks in its own row and
    column (A_ff and A_nf stay as they are, Section 2.3.2): with the ID of
    one segment switched off, every scaled coupling of that level between
    two other segments is bit-identical; every ID of the level sees the
    level-start matrix (the simultaneous reading), so the neighbours'
    skeletons are unchanged too."""
    P = make_config(2, side=63)
    nd = nd_order(P.dims)
    base, off = {}, {}
    spalu.factor(nd, P.scipy(), spalu.Opts(eps=P.eps, trace=lambda lev, d: base.setdefault(lev, d)))
    nr, lev, c0 = max((len(r[1]) - r[0], l, c) for l in base for c, r in base[l]["ids"].items())
    assert nr > 0
    o = spalu.Opts(eps=P.eps, no_id=frozenset({(lev, c0)}),
                   trace=lambda l, d: off.setdefault(l, d))
    spalu.factor(nd, P.scipy(), o)
    a, b = base[lev], off[lev]
    assert c0 in a["ids"] and c0 not in b["ids"]
    assert set(a["ids"]) - {c0} == set(b["ids"])
    for c in b["ids"]:
        assert np.array_equal(a["ids"][c][1], b["ids"][c][1])
    touched = 0
    for key in a["scaled"]:
        if c0 in key:
            touched += a["scaled"][key].shape != b["scaled"][key].shape
            continue
        assert np.array_equal(a["scaled"][key], b["scaled"][key])
    assert touched > 0


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


# ------------------------------------------- symmetric form (Section 4.4.2)
def test_cholesky_and_triangular_solves_match_lapack():
    """The LDL^T factor in Cholesky form and its triangular solves equal
    LAPACK's Cholesky and dense solves; a block that is not positive
    definite is refused."""
    rng = np.random.default_rng(21)
    G = rng.standard_normal((30, 30))
    M = G @ G.T + 30 * np.eye(30)
    C = dense.cholesky(M)
    assert np.allclose(C, np.linalg.cholesky(M), rtol=1e-13, atol=1e-13)
    X = rng.standard_normal((30, 4))
    assert np.allclose(dense.solve_lower(C, X), np.linalg.solve(C, X), rtol=1e-12)
    assert np.allclose(dense.solve_lower_transposed(C, X), np.linalg.solve(C.T, X), rtol=1e-12)
    Z = rng.standard_normal((5, 30))
    assert np.allclose(dense.right_solve_lower_transposed(C, Z), Z @ np.linalg.inv(C.T), rtol=1e-10)
    with pytest.raises(ValueError):
        dense.cholesky(-M)


@pytest.mark.parametrize("cfg,side", [(0, 15), (0, 31), (1, 31), (3, 7), (3, 15)])
def test_sym_eps0_equals_dense_lu(cfg, side):
    """Symmetric form with compression off: exact block LDL^T along the ND
    tree, a dense solve to 1e-12."""
    P = make_config(cfg, side=side, nrhs=2)
    F = spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=0.0, symmetric=1))
    x = spalu.apply_inverse(F, P.rhs)
    xe = _solve_dense(P)
    assert np.linalg.norm(x - xe) <= 1e-12 * np.linalg.norm(xe)


def _level_asymmetry(cfg, side, eps, symmetric):
    P = make_config(cfg, side=side)
    seen = {}
    spalu.factor(nd_order(P.dims), P.scipy(),
                 spalu.Opts(eps=eps, symmetric=symmetric, trace=lambda lev, d: seen.setdefault(lev, d)))
    out = {}
    for lev, d in seen.items():
        b = d["blocks"]
        big = max(np.abs(v).max() for v in b.values() if v.size)
        out[lev] = max((np.abs(v - b[(cd[1], cd[0])].T).max() for cd, v in b.items() if v.size),
                       default=0.0) / big
    return out


def test_sym_level_matrices_stay_symmetric():
    """W~ = V~^T (Section 4.4.2): with the LDL^T (Cholesky) scaling every
    level's matrix is symmetric to rounding, which is what lets one ID
    serve A_{s,n} and A_{n,s}^T; the LU scaling of the stacked form makes
    it unsymmetric after the first level (the contrast shows the check
    sees a one-sided scaling)."""
    a_sym = _level_asymmetry(1, 31, 1e-6, 1)
    a_lu = _level_asymmetry(1, 31, 1e-6, 0)
    assert len(a_sym) >= 4
    assert max(a_sym.values()) <= 1e-12
    assert max(a_lu.values()) >= 1e-3


def test_sym_level_L_ids_are_ids_of_the_exact_one_sided_couplings():
    """Symmetric form: with every row near (rho large) each level-L ID is
    LAPACK's pivoted QR ID of S_{n,c} alone, from the dense Schur
    complement of the leaves computed here with numpy."""
    P = make_config(1, side=31)
    nd = nd_order(P.dims)
    A = P.scipy()
    seen = {}
    o = spalu.Opts(eps=P.eps, rho=1e9, symmetric=1, trace=lambda lev, d: seen.setdefault(lev, d))
    spalu.factor(nd, A, o)
    L = nd.L
    S, pos = _level_schur(A, nd, L)
    lvl = nd.levels[L]
    tr = seen[L]
    checked = 0
    for c, sg in enumerate(lvl.segs):
        if c not in tr["ids"]:
            continue
        k, perm, T, h, passes, _ = tr["ids"][c]
        vc = pos[tr["cur"][c]]
        Y = np.vstack([S[np.ix_(pos[tr["cur"][d]], vc)] for (a, d) in lvl.pairs if a == c and d != c])
        ks, ps, Ts = _scipy_id(Y, P.eps)
        assert (k, passes) == (ks, 1)
        _check_pivots(Y, perm, k, ps)
        if np.array_equal(perm, ps):
            assert np.allclose(T, Ts, rtol=1e-7, atol=1e-9)
        checked += 1
    assert checked >= 8


@pytest.mark.parametrize("cfg,side", [(0, 63), (1, 63), (3, 15)])
def test_sym_compressed_within_10_eps(cfg, side):
    """Symmetric form, compression on: normwise backward error <= 10 eps,
    the relative residual <= 10 eps for the Laplacians, and refinement to
    1e-10."""
    P = make_config(cfg, side=side, nrhs=2)
    A = P.scipy()
    F = spalu.factor(nd_order(P.dims), A, spalu.Opts(eps=P.eps, symmetric=1))
    assert sum(r.sparsified for rec in F.levels.values() for r in rec.segs) > 0
    x, it, hist = spalu.solve(F, P.rhs, tol=1e-10, max_iter=30)
    assert hist[-1].max() <= 1e-10
    x0 = spalu.apply_inverse(F, P.rhs)
    normA = np.linalg.norm(A.toarray(), 2)
    back = np.linalg.norm(P.rhs - A @ x0, axis=0) / (normA * np.linalg.norm(x0, axis=0))
    assert back.max() <= 10 * P.eps
    if cfg != 1:
        assert hist[0].max() <= 10 * P.eps


def test_sym_solution_operator_is_symmetric():
    """W~ = V~^T: the symmetric form's approximate inverse is a symmetric
    matrix to rounding even with compression on, while the stacked form's
    is symmetric only to the truncation level."""
    P = make_config(1, side=31)
    nd = nd_order(P.dims)
    M1 = spalu.apply_inverse(spalu.factor(nd, P.scipy(), spalu.Opts(eps=1e-4, symmetric=1)), np.eye(961))
    M0 = spalu.apply_inverse(spalu.factor(nd, P.scipy(), spalu.Opts(eps=1e-4)), np.eye(961))
    assert np.linalg.norm(M1 - M1.T) <= 1e-13 * np.linalg.norm(M1)
    assert np.linalg.norm(M0 - M0.T) >= 1e-7 * np.linalg.norm(M0)


def test_sym_refuses_what_it_cannot_factor():
    """The symmetric form needs a symmetric matrix, and its LDL^T without
    pivoting needs positive pivots (a negative definite operator has none)."""
    P = make_config(2, side=15)
    with pytest.raises(ValueError):
        spalu.factor(nd_order(P.dims), P.scipy(), spalu.Opts(eps=1e-6, symmetric=1))
    P = make_config(0, side=15)
    with pytest.raises(ValueError):
        spalu.factor(nd_order(P.dims), -P.scipy(), spalu.Opts(eps=1e-6, symmetric=1))
