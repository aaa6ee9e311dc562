"""Oracle: spaLU factorization, solve and iterative refinement (FP64).

Follows Algorithm 2 and Section 4.3 step by step, on a dictionary of dense
blocks indexed by pairs of segments (the separator-graph Schur complement
A^(l) of eq. (4.9)).

  1. Leaf elimination (eq. (4.8)): LU of every leaf interior block A_II and
     the Schur update A_BB -= A_BI A_II^{-1} A_IB onto the level-L blocks.
  2. For l = L..1:
     a. Sparsify every regular segment with neighbours (eq. (4.9)): hybrid
        sampling Y = [A_{N,s}; A_{s,N}^T; G [A_{F,s}; A_{s,F}^T] / sqrt(h)]
        (eq. (4.6), stacked as in eq. (4.12)), column-pivoted QR ID of Y
        (eqs. (4.1)-(4.3)); all IDs of a level use the level-start matrix.
     b. Apply L_t and U_t = L_t^T to the diagonal block, drop the remainder
        rows/columns of every coupling (eq. (2.7)).
     c. LU of every segment diagonal block, remainder rows first; scale the
        couplings so every diagonal block becomes I (eq. (4.10)).
     d. Eliminate the level-l separators: A_ab -= A_{a,s} A_{s,b} (Z_l, Z_u).
     e. Merge surviving skeletons and junctions into the level-(l-1)
        segments (E_(l), eq. (4.11)).
  3. Solve: x = V~ W~ b with W, V of eqs. (4.12)-(4.13).

Symmetric form (Section 4.4.2, Opts.symmetric = 1, for symmetric positive
definite A): A_{s,n} and A_{n,s}^T share one ID, so the sampled matrix is
the one-sided Y = [A_{N,s}; G A_{F,s} / sqrt(h)], and every segment block
is factored as LDL^T, here in its Cholesky form C C^T with C = L D^{1/2}, in
place of the pivoted LU: the couplings are scaled as C_c^{-1} A_cd C_d^{-T},
which keeps every level's matrix symmetric, and W~ = V~^T.  The leaves keep
the pivoted LU (their Schur complement is symmetric either way).

Readings of points the paper leaves open (each is a documented choice):
  * near field N of a segment: neighbour DOFs within Chebyshev grid
    distance max(1, ceil(rho * span)) of the segment's bounding box, rho =
    0.5 by default; the rest is the far field F;
  * the rank test is relative: stop at the first |R_jj| <= eps |R_11|;
  * samples: h starts at h0 = 8 (or a predicted value), doubles while an
    a-posteriori test with 5 Gaussian probes of the far rows fails,
        max_i ||w_i^T E|| > tau * sqrt(n - k) * eps * |R_11|,
        E = B_F P_r - B_F P_s T,  tau = 1,
    and once h >= |F| the exact far rows are used.  For a standard Gaussian
    w, E ||w^T E||^2 = ||E||_F^2, so each probe estimates the Frobenius norm
    of the far-field residual; the unsampled ID accepted by the rank test
    leaves n - k residual columns of norm at most eps |R_11| each, i.e.
    ||E||_F <= sqrt(n - k) eps |R_11|, and the test holds the sampled ID to
    that same bound (by Halko, Martinsson and Tropp 2011, Section 4.3, the
    accepted ||E||_2 is then at most 10 sqrt(2/pi) times the bound with
    probability 1 - 10^-probes);
  * a rank hint (learned form) gives the first h; a negative hint keeps the
    segment whole (k = n, no ID): skipping compression is exact, it only
    gives up the reduction in size;
  * merged segments list their constituents' surviving DOFs one after
    another, constituents ordered by smallest original vertex id (ascending
    vertex ids along 2D separators), skeletons in pivot order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

from . import dense
from .philox import gaussian
from .nd import ND


@dataclasses.dataclass
class Opts:
    eps: float = 1e-6
    symmetric: int = 0         # 0: stacked ID + pivoted LU; 1: symmetric form (one-sided ID + LDL^T)
    seed: int = 1234
    rho: float = 0.5
    h0: int = 8
    probes: int = 5
    tau: float = 1.0
    rank_hint: object = None   # callable (level, seg, info) -> initial h (< 0: keep whole), or None
    no_id: frozenset = frozenset()   # (level, segment) pairs kept whole (locality checks)
    trace: object = None       # callable (level, dict) receiving each level's blocks (checks)


@dataclasses.dataclass
class SegRec:
    dofs: np.ndarray           # current DOF order [remainder; skeleton]
    nr: int                    # remainder size (0 if not sparsified)
    T: np.ndarray | None       # k x nr interpolation matrix
    LU: np.ndarray
    piv: np.ndarray
    sparsified: bool
    h: int = 0
    passes: int = 0
    margin: float = float("inf")   # closest rank / check decision to its threshold
    chol: bool = False         # symmetric form: LU holds the Cholesky factor C (lower), piv = identity

    @property
    def skel(self):
        return self.dofs[self.nr:]


@dataclasses.dataclass
class LevelRec:
    level: int
    segs: list
    sep_coup: dict             # sep index -> list of (d, A'_{d,s}, A'_{s,d})
    n_before: list
    k_after: list


@dataclasses.dataclass
class Factor:
    nd: ND
    A: sp.csr_matrix
    opts: Opts
    symmetric: bool
    leaves: list               # (interior verts, LU, piv)
    levels: dict
    interior_mask: np.ndarray
    flops: float = 0.0


def _cheb_to_box(coords, lo, hi):
    d = np.maximum(np.asarray(lo)[None, :] - coords, 0)
    d = np.maximum(d, coords - np.asarray(hi)[None, :])
    return d.max(axis=1)


def _coords(nd, verts):
    nx, ny, nz = nd.dims
    v = np.asarray(verts, dtype=np.int64)
    return np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=1)


def _dense(A, rows, cols):
    return A[rows][:, cols].toarray()


def coupling_rows(nd, lev, c, blocks, cur, opts, sym=False):
    """Rows of the stacked coupling matrix [A_{n,c}; A_{c,n}^T] of segment c
    (eq. (4.12)), split into near rows B_N and far rows B_F (Section 4.2.3,
    hybrid sampling); also the vertex id and half (0: a row of A_{n,c}, 1: a
    row of A_{c,n}^T) of every far row, which key its Gaussian entries.
    With sym (symmetric form, Section 4.4.2) only the rows of A_{n,c} are
    taken.  Returns None when the segment has no coupling rows."""
    lvl = nd.levels[lev]
    seg = lvl.segs[c]
    nbrs = [d for (a, d) in lvl.pairs if a == c and d != c]
    rows, verts, halves = [], [], []
    for d in nbrs:
        if len(cur[d]) == 0:
            continue
        rows.append(blocks[(d, c)])
        verts.append(cur[d]); halves.append(np.zeros(len(cur[d]), dtype=np.int64))
        if not sym:
            rows.append(blocks[(c, d)].T)
            verts.append(cur[d]); halves.append(np.ones(len(cur[d]), dtype=np.int64))
    if not rows or len(cur[c]) == 0:
        return None
    Bm = np.vstack(rows)
    verts = np.concatenate(verts)
    halves = np.concatenate(halves)
    lo, hi = np.array(seg.bbox_lo), np.array(seg.bbox_hi)
    span = int((hi - lo + 1).max())
    reach = opts.rho * span
    thr = max(1, int(math.ceil(reach))) if math.isfinite(reach) else math.inf
    near = _cheb_to_box(_coords(nd, verts), lo, hi) <= thr
    return Bm[near], Bm[~near], verts[~near], halves[~near]


def sampled_id(BN, BF, vf, hf, lev, c, h, opts):
    """Hybrid-sampled CPQR ID (Sections 4.1-4.2) of the columns of
    [B_N; B_F]: Y = [B_N; G B_F / sqrt(h)] with G Gaussian (h x |F|, entries
    keyed by (seed, level, row, vf, c, hf)), CPQR of Y, and the a-posteriori
    probe check of the far rows; h doubles until the check passes, and once
    h >= |F| the exact far rows are used (then no check is needed).  Returns
    (k, perm, T, h, passes, margin); margin is the closest of the rank and
    check decisions to its threshold (relative)."""
    passes = 0
    margins = []
    while True:
        passes += 1
        if h >= len(BF):
            Y = np.vstack([BN, BF])
            k, perm, T, r11 = dense.cpqr_id(Y, opts.eps, margins=margins)
            return k, perm, T, len(BF), passes, min(margins, default=float("inf"))
        G = gaussian(opts.seed, lev, 0, np.arange(h), vf, c, hf)
        Y = np.vstack([BN, (G @ BF) / math.sqrt(h)])
        k, perm, T, r11 = dense.cpqr_id(Y, opts.eps, margins=margins)
        Om = gaussian(opts.seed, lev, 1, np.arange(opts.probes), vf, c, hf)
        P = Om @ BF
        E = P[:, perm[k:]] - P[:, perm[:k]] @ T
        err = float(np.sqrt((E ** 2).sum(axis=1)).max()) if E.size else 0.0
        bound = opts.tau * math.sqrt(len(perm) - k) * opts.eps * r11
        if bound > 0:
            margins.append(abs(err / bound - 1.0))
        if err <= bound:
            return k, perm, T, h, passes, min(margins, default=float("inf"))
        h *= 2


def segment_id(nd, lev, c, blocks, cur, opts, sym):
    """ID of segment c of level lev against the level-start blocks; returns
    the result of sampled_id, or None when the segment has no coupling rows
    or a negative rank hint keeps it whole."""
    rows = coupling_rows(nd, lev, c, blocks, cur, opts, sym)
    if rows is None:
        return None
    BN, BF, vf, hf = rows
    h = opts.h0
    if opts.rank_hint is not None:
        h = int(opts.rank_hint(lev, c, dict(n=len(cur[c]), nnear=len(BN), nfar=len(BF))))
        if h < 0:
            return None
        if h == 0:
            h = opts.h0
    return sampled_id(BN, BF, vf, hf, lev, c, h, opts)


def _scale_block(X, rc, rd):
    """L_ss,c^{-1} P_s,c X U_ss,d^{-1} with the skeleton parts of the
    two-stage LUs of segments c and d (the coupling scaling of eq. (4.10));
    in the symmetric form C_ss,c^{-1} X C_ss,d^{-T} with the skeleton parts
    of their Cholesky factors."""
    LUc, pivc, nrc = rc.LU, rc.piv, rc.nr
    LUd, nrd = rd.LU, rd.nr
    if rc.chol:
        X = dense.solve_lower(LUc[nrc:, nrc:], X)
        return dense.right_solve_lower_transposed(LUd[nrd:, nrd:], X)
    X = dense.apply_row_pivots(pivc[nrc:] - nrc, X)
    X = dense.solve_lower_unit(LUc[nrc:, nrc:], X)
    X = dense.right_solve_upper(LUd[nrd:, nrd:], X)
    return X


def _segment_factor(M, nr, sym):
    """Two-stage factorization of a segment's diagonal block in [r; s] order:
    pivoted LU with the remainder rows first (Section 4.3), or, in the
    symmetric form, the Cholesky factor of the block (no pivoting, so the
    remainder is eliminated first by construction) with identity pivots."""
    if sym:
        return dense.cholesky(M), np.arange(M.shape[0])
    return dense.lu_window(M, split=nr)


def factor(nd, A, opts=None):
    """spaLU factorization (Algorithm 2) of the grid matrix A (CSR)."""
    opts = Opts() if opts is None else opts
    A = sp.csr_matrix(A)
    A.sort_indices()
    sym = bool(opts.symmetric)
    if sym and (abs(A - A.T)).nnz != 0:
        raise ValueError("the symmetric form needs a symmetric matrix")
    L = nd.L
    N = A.shape[0]
    lvlL = nd.levels[L]

    # level-L blocks from A
    cur = {c: sg.verts.copy() for c, sg in enumerate(lvlL.segs)}
    blocks = {(c, d): _dense(A, cur[c], cur[d]) for (c, d) in lvlL.pairs}

    # 1. leaf elimination
    leaves = []
    interior = np.zeros(N, dtype=bool)
    for (I, bsegs) in nd.leaves:
        interior[I] = True
        Bv = np.concatenate([cur[s] for s in bsegs]) if bsegs else np.zeros(0, np.int64)
        LU, piv = dense.lu_window(_dense(A, I, I))
        if len(Bv):
            X = dense.lu_solve(LU, piv, _dense(A, I, Bv))
            S = _dense(A, Bv, I) @ X
            off = np.concatenate([[0], np.cumsum([len(cur[s]) for s in bsegs])])
            for a, sa in enumerate(bsegs):
                for b, sb in enumerate(bsegs):
                    blocks[(sa, sb)] -= S[off[a]:off[a + 1], off[b]:off[b + 1]]
        leaves.append((I, LU, piv))

    levels = {}
    for lev in range(L, 0, -1):
        lvl = nd.levels[lev]
        nseg = len(lvl.segs)
        pairset = set(lvl.pairs)
        # a. IDs on the level-start matrix
        ids = {}
        if opts.eps > 0:
            for c, sg in enumerate(lvl.segs):
                if sg.regular and (lev, c) not in opts.no_id:
                    r = segment_id(nd, lev, c, blocks, cur, opts, sym)
                    if r is not None:
                        ids[c] = r
        # b./c. transform and two-stage LU of every segment
        recs = []
        for c in range(nseg):
            M = blocks[(c, c)]
            n = len(cur[c])
            if c in ids:
                k, perm, T, h, passes, margin = ids[c]
                nr = n - k
                order = np.concatenate([perm[k:], perm[:k]])
                M1 = M[:, order].copy()
                M1[:, :nr] -= M1[:, nr:] @ T
                M2 = M1[order, :].copy()
                M2[:nr, :] -= T.T @ M2[nr:, :]
                LU, piv = _segment_factor(M2, nr, sym)
                recs.append(SegRec(dofs=cur[c][order], nr=nr, T=T, LU=LU, piv=piv,
                                   sparsified=True, h=h, passes=passes, margin=margin, chol=sym))
            else:
                LU, piv = _segment_factor(M, 0, sym)
                recs.append(SegRec(dofs=cur[c].copy(), nr=0, T=None, LU=LU, piv=piv,
                                   sparsified=False, chol=sym))
        sel = {}
        for c in range(nseg):
            if c in ids:
                k, perm = ids[c][0], ids[c][1]
                sel[c] = perm[:k]
            else:
                sel[c] = np.arange(len(cur[c]))
        scaled = {}
        for (c, d) in lvl.pairs:
            if c == d:
                continue
            X = blocks[(c, d)][sel[c]][:, sel[d]]
            scaled[(c, d)] = _scale_block(X, recs[c], recs[d])
        seps = [c for c, sg in enumerate(lvl.segs) if sg.is_sep]
        sep_coup = {}
        for s in seps:
            sep_coup[s] = [(d, scaled[(d, s)], scaled[(s, d)])
                           for (a, d) in lvl.pairs if a == s and d != s]
        levels[lev] = LevelRec(level=lev, segs=recs, sep_coup=sep_coup,
                               n_before=[len(cur[c]) for c in range(nseg)],
                               k_after=[len(recs[c].skel) for c in range(nseg)])
        if opts.trace is not None:
            opts.trace(lev, dict(blocks=blocks, cur=cur, ids=ids, recs=recs, scaled=scaled))
        if lev == 1:
            break
        # d./e. eliminate the level-l separators while merging into level l-1
        up = nd.levels[lev - 1]
        cons = {C: [] for C in range(len(up.segs))}
        for c, sg in enumerate(lvl.segs):
            if not sg.is_sep:
                cons[sg.parent].append(c)
        off = {}
        cur_next = {}
        for C, lst in cons.items():
            o = 0
            parts = []
            for c in lst:
                off[c] = o
                o += len(recs[c].skel)
                parts.append(recs[c].skel)
            cur_next[C] = np.concatenate(parts) if parts else np.zeros(0, np.int64)
        seps_of = {c: set() for c in range(nseg)}
        for (a, d) in lvl.pairs:
            if a != d and lvl.segs[d].is_sep and not lvl.segs[a].is_sep:
                seps_of[a].add(d)
        uppairs = set(up.pairs)
        for (a, d) in lvl.pairs:
            if not lvl.segs[a].is_sep and not lvl.segs[d].is_sep:
                assert (lvl.segs[a].parent, lvl.segs[d].parent) in uppairs
        for s in seps:
            nb = [d for (a, d) in lvl.pairs if a == s and d != s]
            for a in nb:
                for d in nb:
                    assert (lvl.segs[a].parent, lvl.segs[d].parent) in uppairs
        new_blocks = {}
        for (C, D) in up.pairs:
            out = np.zeros((len(cur_next[C]), len(cur_next[D])))
            for c in cons[C]:
                kc = len(recs[c].skel)
                for d in cons[D]:
                    kd = len(recs[d].skel)
                    sub = out[off[c]:off[c] + kc, off[d]:off[d] + kd]
                    if c == d:
                        sub += np.eye(kc)
                    elif (c, d) in pairset:
                        sub += scaled[(c, d)]
                    for s in sorted(seps_of[c] & seps_of[d]):
                        sub -= scaled[(c, s)] @ scaled[(s, d)]
            new_blocks[(C, D)] = out
        blocks = new_blocks
        cur = cur_next
    return Factor(nd=nd, A=A, opts=opts, symmetric=sym, leaves=leaves, levels=levels,
                  interior_mask=interior)


def apply_inverse(F, B):
    """x = V~ W~ b for every column of B (eqs. (4.12)-(4.13))."""
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    if squeeze:
        B = B[:, None]
    A = F.A
    x = B.copy()
    L = F.nd.L
    # W~: leaf L^{-1}, then per level U_T, blockdiag L^{-1}, Z_l
    w = np.zeros_like(B)
    for (I, LU, piv) in F.leaves:
        w[I] = dense.lu_solve(LU, piv, B[I])
    sepmask = ~F.interior_mask
    x[sepmask] -= (A[sepmask][:, F.interior_mask] @ w[F.interior_mask])
    for lev in range(L, 0, -1):
        rec = F.levels[lev]
        for r in rec.segs:
            v = x[r.dofs]
            if r.sparsified and r.nr > 0:
                v[:r.nr] -= r.T.T @ v[r.nr:]
            if r.chol:
                v = dense.solve_lower(r.LU, v)
            else:
                v = dense.solve_lower_unit(r.LU, dense.apply_row_pivots(r.piv, v))
            x[r.dofs] = v
        for s, lst in rec.sep_coup.items():
            xs = x[rec.segs[s].skel]
            for (d, Ads, _) in lst:
                x[rec.segs[d].skel] -= Ads @ xs
    # V~: per level (root first) Z_u, blockdiag U^{-1}, L_T; then leaf U^{-1}
    for lev in range(1, L + 1):
        rec = F.levels[lev]
        for s, lst in rec.sep_coup.items():
            acc = np.zeros((len(rec.segs[s].skel), x.shape[1]))
            for (d, _, Asd) in lst:
                acc += Asd @ x[rec.segs[d].skel]
            x[rec.segs[s].skel] -= acc
        for r in rec.segs:
            if r.chol:
                v = dense.solve_lower_transposed(r.LU, x[r.dofs])
            else:
                v = dense.solve_upper(r.LU, x[r.dofs])
            if r.sparsified and r.nr > 0:
                v[r.nr:] -= r.T @ v[:r.nr]
            x[r.dofs] = v
    xs = x.copy()
    xs[F.interior_mask] = 0.0
    rhs = B - A @ xs
    for (I, LU, piv) in F.leaves:
        x[I] = dense.lu_solve(LU, piv, rhs[I])
    return x[:, 0] if squeeze else x


def rel_residual(A, x, b):
    """||A x - b||_2 / ||b||_2 per column (the R_es of Section 6)."""
    r = b - A @ x
    nb = np.linalg.norm(b, axis=0)
    return np.linalg.norm(r, axis=0) / np.where(nb == 0, 1.0, nb)


def solve(F, B, tol=None, max_iter=20):
    """Direct solve, then iterative refinement r = b - A x, x += M r (FP64)
    until every column's relative residual is <= tol.  Returns (x, iters,
    residual history)."""
    B = np.asarray(B, dtype=np.float64)
    x = apply_inverse(F, B)
    hist = [rel_residual(F.A, x, B)]
    it = 0
    if tol is not None:
        while hist[-1].max() > tol and it < max_iter:
            x = x + apply_inverse(F, B - F.A @ x)
            hist.append(rel_residual(F.A, x, B))
            it += 1
    return x, it, hist


def compression_stats(F):
    """Per level with sparsified segments: (e_l, e'_l) = (max size before,
    max size after) over the sparsified segments, and q~ = max_l e'_l / e_l
    (the numerical compression factor of Section 6)."""
    out = {}
    q = 0.0
    for lev, rec in F.levels.items():
        sp_ = [i for i, r in enumerate(rec.segs) if r.sparsified]
        if not sp_:
            continue
        e = max(rec.n_before[i] for i in sp_)
        e2 = max(rec.k_after[i] for i in sp_)
        out[lev] = (e, e2)
        if e > 0:
            q = max(q, e2 / e)
    return out, q
