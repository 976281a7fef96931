"""Oracle for block principal pivoting NNLS.  TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the benchmark
may import this module.  The GPU library never calls it and shares no code with it.

Plain, serial, float64.  Follows Cantarella & Piatek, "tsnnls: A solver for large sparse
least squares problems with non-negative variables" (arXiv cs/0408029):

  * problem: min 1/2 ||Ax - b||^2 subject to x >= 0, A m x n of full column rank (Eq. 1);
  * complementarity form: y = A^T A x - A^T b, x >= 0, y >= 0, <x, y> = 0 (Eq. 3);
  * complementary basic solution for a split (F, G): x_F solves the unconstrained least
    squares problem on the columns A_F (Eq. 4) and y_G = A_G^T (A_F x_F - b) (Eq. 5);
  * the pivoting loop of the algorithm box in Sec. 2 (block principal pivoting with the
    paper's change for numerically degenerate problems): exchange all infeasible variables
    while their count falls, allow three non-improving block exchanges, then exchange only
    the infeasible variable of largest index; tested entries of magnitude below 1e-12
    count as zero;
  * Eq. 4 is solved by the normal equations A_F^T A_F x_F = A_F^T b with a Cholesky
    factor (Sec. 2.1), taking A_F^T A_F as the F-principal block of A^T A computed once
    from column dot products (Sec. 3).

Readings where the paper is silent or loose (each also listed in the design notes):
  * zeroing is |v| < tau -> v = 0 with an absolute tau (a literal reading of the box's
    inequality would zero every negative entry; the Sec. 2 text bounds the magnitude);
  * the same classify-and-zero step also runs before the first exchange, on y = -A^T b;
  * y_G is formed from the un-zeroed x_F; zeroing happens at the top of the next pass;
  * negative means strictly below zero after zeroing; the box's count, which shares its
    name with the problem dimension, is k here;
  * indices are 0-based; the largest index is the largest column number;
  * an iteration cap of 5n + 100 (the paper gives none) ends the loop with 'maxiter';
  * a non-positive or non-finite Cholesky pivot ends the loop with 'not_pd' (Sec. 2.1
    expects breakdown once kappa^2 eps >= 1 but prescribes no recovery);
  * the paper assumes finite data: a non-finite entry of A or b, or a tested entry of an
    iterate that is not finite (overflow), ends the loop with 'invalid_value', since no
    sign test can decide it.

Library primitives used as steps: scipy sparse products for A^T A, A^T b and the two
products of Eq. 5; LAPACK dpotrf for the Cholesky factor; triangular solves.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.linalg.lapack as lapack
import scipy.sparse as sp

TAU = 1e-12     # zeroing threshold of Sec. 2
P_MAX = 3       # block-exchange budget p of the Sec. 2 algorithm box

BRANCH_BLOCK_IMPROVED = 0   # k < N: N <- k, p <- 3, exchange all infeasible
BRANCH_BLOCK_BUDGET = 1     # k >= N, p > 0: p <- p - 1, exchange all infeasible
BRANCH_SINGLE = 2           # k >= N, p = 0: exchange the infeasible variable of largest index


@dataclasses.dataclass
class TraceRow:
    k: int            # infeasible count after zeroing
    branch: int       # BRANCH_* taken
    N: int            # best count after the rule
    p: int            # remaining budget after the rule
    n_free: int       # |F| after the exchange
    min_margin: float # smallest |v| over the sign tests that were not zeroed


@dataclasses.dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    free: np.ndarray          # bool[n]: True on F
    iterations: int
    status: str               # 'ok' | 'not_pd' | 'maxiter' | 'invalid_value'
    failed_index: int = -1
    trace: List[TraceRow] = dataclasses.field(default_factory=list)
    last_ninf: int = 0
    final_margin: float = np.inf


def gram(A, b):
    """H = A^T A by column dot products and c = A^T b (Sec. 3; the right-hand side of the
    normal equations, Sec. 2.1).  Sparse A gives a sparse H."""
    if sp.issparse(A):
        A = sp.csc_matrix(A)
        H = (A.T @ A).tocsc()
        c = np.asarray(A.T @ b).ravel()
    else:
        A = np.asarray(A, dtype=np.float64)
        H = A.T @ A
        c = A.T @ b
    return H, c


def principal_block(H, idx: np.ndarray) -> np.ndarray:
    """The F-principal submatrix H[F, F] of the cached Gram matrix (Sec. 3)."""
    if sp.issparse(H):
        return H[idx][:, idx].toarray()
    return H[np.ix_(idx, idx)]


def solve_free(H, c, idx: np.ndarray):
    """x_F from the normal equations H_FF x_F = c_F by Cholesky (Eq. 4 via Sec. 2.1).
    Returns (x_F, failed) where failed is the 0-based position in F of the first
    non-positive pivot, or -1."""
    if idx.size == 0:
        return np.zeros(0), -1
    HFF = principal_block(H, idx)
    L, info = lapack.dpotrf(HFF, lower=1, clean=1)
    if info != 0 or not np.all(np.isfinite(np.diag(L))):
        bad = info - 1 if info > 0 else int(np.argmax(~np.isfinite(np.diag(L))))
        return None, bad
    z = sla.solve_triangular(L, c[idx], lower=True)
    xF = sla.solve_triangular(L, z, lower=True, trans='T')
    return xF, -1


def dual(A, b, idx_free: np.ndarray, xF: np.ndarray, idx_bound: np.ndarray):
    """y_G = A_G^T (A_F x_F - b)  (Eq. 5)."""
    if sp.issparse(A):
        A = sp.csc_matrix(A)
        r = (A[:, idx_free] @ xF if idx_free.size else np.zeros(A.shape[0])) - b
        return np.asarray(A[:, idx_bound].T @ r).ravel()
    A = np.asarray(A)
    r = (A[:, idx_free] @ xF if idx_free.size else np.zeros(A.shape[0])) - b
    return A[:, idx_bound].T @ r


def classify(x, y, free, tau):
    """Zero the tested entries within tau of zero, then flag the negative ones.
    The tested entry of variable i is x_i for i in F and y_i for i in G."""
    v = np.where(free, x, y)
    small = np.abs(v) < tau
    x[free & small] = 0.0
    y[~free & small] = 0.0
    v = np.where(small, 0.0, v)
    infeasible = v < 0.0
    kept = np.abs(v[~small])
    margin = float(kept.min()) if kept.size else np.inf
    return infeasible, margin


def exchange_rule(k: int, N, p: int, p_max: int):
    """The counter logic of the Sec. 2 algorithm box.  Returns (N, p, branch)."""
    if k < N:
        return k, p_max, BRANCH_BLOCK_IMPROVED
    if p > 0:
        return N, p - 1, BRANCH_BLOCK_BUDGET
    return N, p, BRANCH_SINGLE


def bpp_solve(A, b, tau: float = TAU, p_max: int = P_MAX, max_iter: Optional[int] = None) -> Result:
    """Block principal pivoting for min 1/2||Ax - b||^2, x >= 0 (Sec. 2 algorithm box)."""
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    if max_iter is None:
        max_iter = 5 * n + 100
    a_vals = A.data if sp.issparse(A) else np.asarray(A)
    if not (np.all(np.isfinite(a_vals)) and np.all(np.isfinite(b))):
        return Result(x=np.zeros(n), y=np.zeros(n), free=np.zeros(n, dtype=bool), iterations=0,
                      status='invalid_value')
    H, c = gram(A, b)

    # F = empty, G = everything, x = 0, y = -A^T b, p = 3, N = infinity
    free = np.zeros(n, dtype=bool)
    x = np.zeros(n)
    y = -c.copy()
    p = p_max
    N = np.inf
    trace: List[TraceRow] = []
    it = 0
    while True:
        if not np.all(np.isfinite(np.where(free, x, y))):
            return Result(x=x, y=y, free=free, iterations=it, status='invalid_value', trace=trace)
        infeasible, margin = classify(x, y, free, tau)
        k = int(infeasible.sum())
        if k == 0:
            return Result(x=x, y=y, free=free, iterations=it, status='ok', trace=trace,
                          last_ninf=0, final_margin=margin)
        if it >= max_iter:
            return Result(x=x, y=y, free=free, iterations=it, status='maxiter', trace=trace,
                          last_ninf=k, final_margin=margin)
        N, p, branch = exchange_rule(k, N, p, p_max)
        if branch == BRANCH_SINGLE:
            r = int(np.flatnonzero(infeasible).max())
            free[r] = not free[r]
        else:
            free = free ^ infeasible

        idx_f = np.flatnonzero(free)
        idx_g = np.flatnonzero(~free)
        xF, failed = solve_free(H, c, idx_f)
        it += 1
        trace.append(TraceRow(k=k, branch=branch, N=int(N), p=p, n_free=int(idx_f.size),
                              min_margin=margin))
        if xF is None:
            return Result(x=x, y=y, free=free, iterations=it, status='not_pd',
                          failed_index=int(idx_f[failed]), trace=trace, last_ninf=k)
        x = np.zeros(n)
        x[idx_f] = xF
        y = np.zeros(n)
        y[idx_g] = dual(A, b, idx_f, xF, idx_g)


def kkt_residuals(A, b, x, y):
    """Max violations of Eq. 3: (min(x), min(y), |<x,y>|, ||y - (A^T A x - A^T b)||_inf)."""
    if sp.issparse(A):
        g = np.asarray(A.T @ (A @ x - b)).ravel()
    else:
        g = A.T @ (A @ x - b)
    return (float(min(x.min(), 0.0)), float(min(y.min(), 0.0)),
            float(abs(np.dot(x, y))), float(np.max(np.abs(y - g))))


def inverse_onenorm_estimate(H, max_iter: int = 5) -> float:
    """Lower-bound estimate of ||H^-1||_1 for a symmetric positive definite H, from its
    Cholesky factor.  Sec. 3 estimates the condition of A_F^T A_F from the factor it already
    has (LAPACK dpocon); this is the estimator behind such routines: Hager's method
    (1984) with Higham's refinements (1988).  Every value it forms is ||H^-1 v||_1 / ||v||_1
    for some v, so the result never exceeds the true norm.

    1. v = (1/n, ..., 1/n): est = ||H^-1 v||_1, xi = sign(H^-1 v) (+1 for >= 0).
    2. z = H^-1 xi (H is symmetric); j = first index of max |z_j|.
    3. Repeat: v = e_j, est' = ||H^-1 e_j||_1; stop if the signs of H^-1 e_j equal xi or
       est' does not grow; else xi = those signs, z = H^-1 xi, and stop if max |z| sits at
       the previous j again or after max_iter rounds in all; j = the new index.
    4. v_i = (-1)^i (1 + i / (n - 1)): the result is the larger of est and
       ||H^-1 v||_1 / ||v||_1 = 2 ||H^-1 v||_1 / (3 n).
    """
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    fac = sla.cho_factor(H, lower=True)

    def solve(v):
        return sla.cho_solve(fac, v)

    def signs(y):
        return np.where(y >= 0.0, 1.0, -1.0)

    if n == 1:
        return float(abs(solve(np.ones(1))[0]))
    y = solve(np.full(n, 1.0 / n))
    est = float(np.abs(y).sum())
    xi = signs(y)
    z = solve(xi)
    j = int(np.argmax(np.abs(z)))
    rounds = 2
    while True:
        e = np.zeros(n)
        e[j] = 1.0
        y = solve(e)
        new = float(np.abs(y).sum())
        xin = signs(y)
        if np.array_equal(xin, xi) or new <= est:
            est = max(est, new)
            break
        est = new
        xi = xin
        z = solve(xi)
        jlast = j
        j = int(np.argmax(np.abs(z)))
        rounds += 1
        if abs(z[jlast]) == abs(z[j]) or rounds > max_iter:
            break
    v = np.array([(-1.0) ** i * (1.0 + i / (n - 1)) for i in range(n)])
    alt = 2.0 * float(np.abs(solve(v)).sum()) / (3.0 * n)
    return max(est, alt)


def predicted_rel_error(H) -> float:
    """Predicted relative error of a normal-equations solution with the Gram block H
    (Sec. 2.1: about c kappa^2 eps with kappa^2 the condition of A_F^T A_F; Sec. 4 fits
    c = 1/10): 0.1 * ||H||_1 * est(||H^-1||_1) * eps, eps = 2^-52."""
    H = np.asarray(H, dtype=np.float64)
    return 0.1 * float(np.abs(H).sum(axis=0).max()) * inverse_onenorm_estimate(H) * np.finfo(np.float64).eps
