"""Oracle dense kernels: pivoted LU with a pivot window, Cholesky, triangular
solves, and the column-pivoted QR interpolative decomposition.

Plain loops in FP64; each routine is the textbook definition.
"""
from __future__ import annotations

import numpy as np

TIE_REL = 1e-12   # CPQR: column norms within this relative gap of the
                  # maximum count as tied; the smallest original column wins


def lu_window(M, split=None):
    """LU with partial pivoting, P M = L U, done in place on a copy.

    For steps j < split the pivot is searched in rows [j, split), for steps
    j >= split in rows [j, n): the two-stage factorization of a sparsified
    segment (remainder rows first, then skeleton rows, so the remainder is
    eliminated without mixing skeleton rows into it; Section 4.3).  Ties in
    |a| go to the smallest row.  Returns (LU packed, piv) with LAPACK's
    convention: step j swapped rows j and piv[j].
    """
    A = np.array(M, dtype=np.float64, copy=True)
    n = A.shape[0]
    split = n if split is None else split
    piv = np.arange(n)
    for j in range(n):
        hi = split if j < split else n
        col = np.abs(A[j:hi, j])
        p = j + int(np.argmax(col))          # argmax returns the first max
        piv[j] = p
        if p != j:
            A[[j, p], :] = A[[p, j], :]
        if A[j, j] == 0.0:
            raise ZeroDivisionError("singular pivot block")
        A[j + 1:, j] /= A[j, j]
        A[j + 1:, j + 1:] -= np.outer(A[j + 1:, j], A[j, j + 1:])
    return A, piv


def apply_row_pivots(piv, X):
    X = np.array(X, dtype=np.float64, copy=True)
    for j, p in enumerate(piv):
        if p != j:
            X[[j, p]] = X[[p, j]]
    return X


def solve_lower_unit(LU, X):
    """L^{-1} X with L the unit lower triangle of LU."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for j in range(n):
        X[j + 1:] -= np.outer(LU[j + 1:, j], X[j])
    return X


def solve_upper(LU, X):
    """U^{-1} X with U the upper triangle of LU."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for j in range(n - 1, -1, -1):
        X[j] /= LU[j, j]
        X[:j] -= np.outer(LU[:j, j], X[j])
    return X


def right_solve_upper(LU, X):
    """X U^{-1} (solve Z U = X for Z)."""
    return solve_upper_transposed(LU, X.T).T


def solve_upper_transposed(LU, X):
    """U^{-T} X: forward substitution with U^T (lower, non-unit)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = LU.shape[0]
    for j in range(n):
        X[j] /= LU[j, j]
        X[j + 1:] -= np.outer(LU[j, j + 1:], X[j])
    return X


def cholesky(M):
    """Lower-triangular C with M = C C^T, column by column (the textbook
    Cholesky algorithm; only the lower triangle of M is read).  This is the
    LDL^T factorization of a symmetric positive definite block with the
    square root of D split evenly between its two factors, C = L D^{1/2}.
    A pivot <= 0 (M not positive definite) raises ValueError."""
    A = np.array(M, dtype=np.float64, copy=True)
    n = A.shape[0]
    C = np.zeros_like(A)
    for j in range(n):
        d = A[j, j] - np.dot(C[j, :j], C[j, :j])
        if not d > 0.0:
            raise ValueError("non-positive pivot %d: block not positive definite" % j)
        C[j, j] = np.sqrt(d)
        C[j + 1:, j] = (A[j + 1:, j] - C[j + 1:, :j] @ C[j, :j]) / C[j, j]
    return C


def solve_lower(C, X):
    """C^{-1} X with C lower triangular (non-unit diagonal)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = C.shape[0]
    for j in range(n):
        X[j] /= C[j, j]
        X[j + 1:] -= np.outer(C[j + 1:, j], X[j])
    return X


def solve_lower_transposed(C, X):
    """C^{-T} X with C lower triangular (back substitution with C^T)."""
    X = np.array(X, dtype=np.float64, copy=True)
    n = C.shape[0]
    for j in range(n - 1, -1, -1):
        X[j] /= C[j, j]
        X[:j] -= np.outer(C[j, :j], X[j])
    return X


def right_solve_lower_transposed(C, X):
    """X C^{-T} (solve Z C^T = X for Z)."""
    return solve_lower(C, np.asarray(X).T).T


def lu_solve(LU, piv, X):
    """(P^T L U)^{-1} X."""
    return solve_upper(LU, solve_lower_unit(LU, apply_row_pivots(piv, X)))


def cpqr_id(Y, eps, max_rank=None, margins=None):
    """Interpolative decomposition by Householder QR with column pivoting
    (Section 4.1, eqs. (4.1)-(4.3)).

    At each step the pivot is the column with the largest norm of its part
    below the current row, recomputed from scratch (no norm downdating);
    norms within TIE_REL of the maximum are tied and the smallest original
    column index wins.  The rank k is the first step j at which that largest
    norm is <= eps * |R_11|; it is 0 for an all-zero Y.

    Returns (k, perm, T, r11): perm lists original column indices in pivot
    order (first k = skeleton), T = R_11^{-1} R_12 is k x (n-k), and r11 is
    |R_11|.  If ``margins`` is a list, the relative distance of every
    rank decision to the threshold, |norm / (eps |R_11|) - 1|, is appended
    (how close a differently rounded run could come to deciding otherwise).
    """
    Y = np.array(Y, dtype=np.float64, copy=True)
    m, n = Y.shape
    perm = np.arange(n)
    steps = min(m, n) if max_rank is None else min(m, n, max_rank)
    r11 = 0.0
    k = steps
    if steps == 0:
        return 0, perm, np.zeros((0, n)), 0.0
    for j in range(steps):
        norms = np.sqrt(np.sum(Y[j:, j:] ** 2, axis=0))
        mx = norms.max() if norms.size else 0.0
        if j == 0:
            r11 = mx
        if margins is not None and eps > 0 and r11 > 0:
            margins.append(abs(mx / (eps * r11) - 1.0))
        if mx == 0.0 or mx <= eps * r11:
            k = j
            break
        cand = np.nonzero(norms >= mx * (1.0 - TIE_REL))[0]
        q = j + int(cand[np.argmin(perm[j + cand])])
        if q != j:
            Y[:, [j, q]] = Y[:, [q, j]]
            perm[[j, q]] = perm[[q, j]]
        x = Y[j:, j].copy()
        alpha = np.sqrt(np.dot(x, x))
        s = 1.0 if x[0] >= 0.0 else -1.0
        v = x.copy()
        v[0] += s * alpha
        vv = np.dot(v, v)
        Y[j:, j:] -= np.outer(v, (2.0 / vv) * (v @ Y[j:, j:]))
        Y[j + 1:, j] = 0.0
    R11 = np.triu(Y[:k, :k])
    R12 = Y[:k, k:]
    if k > 0:
        T = solve_upper(R11, R12)
    else:
        T = np.zeros((0, n))
    return k, perm, T, r11
