"""Seeded synthetic NNLS instances with a planted, known solution.

This module only draws inputs.  It holds no step of the pivoting solver: it samples a
matrix A, a complementary pair (x*, y*) and builds b so that (x*, y*) is the solution of
the complementarity form y = A^T A x - A^T b, x >= 0, y >= 0, <x, y> = 0 (Eq. 3 of
Cantarella & Piatek, "tsnnls").  Both the CPU oracle and the GPU library are fed from here.

Planted construction (the same for every shape):
  * choose the active set F* by exact count round(f*n), without replacement;
  * x*_i ~ U(lo, 1) on F*, y*_i ~ U(lo, 1) off F*, zero elsewhere;
  * solve A^T A z = y* (dense Cholesky for dense A, conjugate gradients on the operator
    v -> A^T (A v) for sparse A) and set b = A (x* - z).
Then A^T (A x* - b) = A^T A z = y* + delta, where delta is the residual of the z solve,
recorded as ``delta_inf``.  With margin lo >> |delta| the unique NNLS solution keeps the
active set F* and differs from x* by at most ||(H_FF)^-1|| ||delta_F||.

Random numbers: numpy PCG64 through ``numpy.random.default_rng(seed)``; batches draw one
child stream per problem from ``SeedSequence(seed).spawn``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclasses.dataclass
class Instance:
    """One NNLS instance.  ``A`` is a scipy CSC matrix (float64, sorted unique row
    indices per column, int32 indices) or a Fortran-ordered float64 ndarray."""
    A: object
    b: np.ndarray
    x_star: np.ndarray
    y_star: np.ndarray
    active: np.ndarray          # bool[n], True on F*
    delta_inf: float            # ||A^T A z - y*||_inf of the planting solve
    name: str = ""
    seed: int = 0

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def is_sparse(self) -> bool:
        return sp.issparse(self.A)


def _canonical_csc(A) -> sp.csc_matrix:
    A = sp.csc_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def _plant_values(rng, n: int, frac: float, lo: float, zero_pairs: int = 0):
    """Complementary (x*, y*) with exact active count round(frac*n).  ``zero_pairs``
    indices outside the active set get y*_i = 0 too (a degenerate instance)."""
    n_act = int(round(frac * n))
    perm = rng.permutation(n)
    active = np.zeros(n, dtype=bool)
    active[perm[:n_act]] = True
    x_star = np.zeros(n)
    y_star = np.zeros(n)
    x_star[active] = rng.uniform(lo, 1.0, size=n_act)
    y_star[~active] = rng.uniform(lo, 1.0, size=n - n_act)
    if zero_pairs:
        inactive = np.flatnonzero(~active)
        y_star[inactive[:zero_pairs]] = 0.0
    return active, x_star, y_star


def _plant_rhs_dense(A: np.ndarray, x_star, y_star):
    G = A.T @ A
    z = sla.cho_solve(sla.cho_factor(G, lower=True), y_star)
    delta = G @ z - y_star
    return A @ (x_star - z), float(np.max(np.abs(delta), initial=0.0))


def _plant_rhs_sparse(A: sp.csc_matrix, x_star, y_star, rtol: float = 1e-14):
    n = A.shape[1]
    At = A.T.tocsr()
    op = spla.LinearOperator((n, n), matvec=lambda v: At @ (A @ v), dtype=np.float64)
    z, info = spla.cg(op, y_star, rtol=rtol, atol=0.0, maxiter=20 * n)
    if info != 0:
        raise RuntimeError(f"planting solve did not converge (info={info})")
    delta = At @ (A @ z) - y_star
    return A @ (x_star - z), float(np.max(np.abs(delta), initial=0.0))


def _finish(A, rng, frac, lo, name, seed, zero_pairs=0) -> Instance:
    n = A.shape[1]
    active, x_star, y_star = _plant_values(rng, n, frac, lo, zero_pairs)
    if sp.issparse(A):
        b, dinf = _plant_rhs_sparse(A, x_star, y_star)
    else:
        b, dinf = _plant_rhs_dense(A, x_star, y_star)
    return Instance(A=A, b=np.ascontiguousarray(b), x_star=x_star, y_star=y_star,
                    active=active, delta_inf=dinf, name=name, seed=seed)


# ---------------------------------------------------------------- matrix recipes

def bernoulli_diag_csc(rng, m: int, n: int, density: float, diag_scale: Optional[float] = None):
    """Bernoulli(density) pattern, N(0,1) values, plus ``diag_scale`` on A[i,i], i < n.
    Default scale sqrt(density*m), about the norm of a random column."""
    if diag_scale is None:
        diag_scale = math.sqrt(density * m)
    R = sp.random(m, n, density=density, format="csc", random_state=rng,
                  data_rvs=lambda k: rng.standard_normal(k))
    D = sp.csc_matrix((np.full(n, diag_scale), (np.arange(n), np.arange(n))), shape=(m, n))
    return _canonical_csc(R + D)


def rows_per_col_band_csc(rng, m: int, n: int, k: int, band=(5.0, 2.5, 1.25)):
    """``k`` distinct uniform-random rows per column with N(0,1) values, plus a diagonal
    band: entry (j+d, j) += band[d] (rows beyond m dropped); duplicates are summed."""
    rows = np.empty(n * k, dtype=np.int64)
    for j in range(n):
        rows[j * k:(j + 1) * k] = rng.choice(m, size=k, replace=False)
    cols = np.repeat(np.arange(n), k)
    vals = rng.standard_normal(n * k)
    br, bc, bv = [], [], []
    for d, s in enumerate(band):
        j = np.arange(n)
        keep = j + d < m
        br.append(j[keep] + d)
        bc.append(j[keep])
        bv.append(np.full(int(keep.sum()), s))
    rows = np.concatenate([rows] + br)
    cols = np.concatenate([cols] + bc)
    vals = np.concatenate([vals] + bv)
    return _canonical_csc(sp.coo_matrix((vals, (rows, cols)), shape=(m, n)))


def block_band_csc(rng, m: int, n: int, k: int, stride: int = 8, width: int = 64):
    """``k`` random rows per column N(0,1) plus a block band: rows [stride*j, stride*j+width)
    get N(0,1) entries and A[stride*j, j] += sqrt(width + k), which gives a
    lower-triangular full-rank block on rows stride*j."""
    parts_r, parts_c, parts_v = [], [], []
    for j in range(n):
        parts_r.append(rng.choice(m, size=k, replace=False))
        parts_c.append(np.full(k, j))
        parts_v.append(rng.standard_normal(k))
        r0 = stride * j
        band_rows = np.arange(r0, min(r0 + width, m))
        parts_r.append(band_rows)
        parts_c.append(np.full(band_rows.size, j))
        v = rng.standard_normal(band_rows.size)
        if band_rows.size and band_rows[0] == r0:
            v[0] += math.sqrt(width + k)
        parts_v.append(v)
    A = sp.coo_matrix((np.concatenate(parts_v), (np.concatenate(parts_r), np.concatenate(parts_c))),
                      shape=(m, n))
    return _canonical_csc(A)


def gaussian_dense(rng, m: int, n: int):
    """Column-major N(0,1)/sqrt(m) matrix."""
    return np.asfortranarray(rng.standard_normal((m, n)) / math.sqrt(m))


# ---------------------------------------------------------------- named workloads

def sparse_small(seed: int = 1001, m: int = 2000, n: int = 400, density: float = 0.02,
                 frac: float = 0.5, lo: float = 0.1) -> Instance:
    """Single sparse instance: Bernoulli(0.02) N(0,1) pattern plus sqrt(0.02 m) on the
    leading diagonal, half the variables active with x*, y* ~ U(0.1, 1)."""
    rng = np.random.default_rng(seed)
    A = bernoulli_diag_csc(rng, m, n, density)
    return _finish(A, rng, frac, lo, f"sparse_small_m{m}_n{n}", seed)


def sparse_large(seed: int = 1002, m: int = 60000, n: int = 12000, k: int = 25,
                 frac: float = 0.3, lo: float = 1e-3, zero_pairs: int = 0) -> Instance:
    """Single large sparse instance: 25 random N(0,1) rows per column plus a three-wide
    diagonal band (5, 2.5, 1.25); 30% active, margin 1e-3.  ``zero_pairs`` inactive
    variables get y*_i = 0 as well (a degenerate instance: x stays unique, the split not)."""
    rng = np.random.default_rng(seed)
    A = rows_per_col_band_csc(rng, m, n, k)
    return _finish(A, rng, frac, lo, f"sparse_large_m{m}_n{n}", seed, zero_pairs=zero_pairs)


def sparse_blockband(seed: int = 1005, m: int = 400000, n: int = 50000, k: int = 20,
                     frac: float = 0.25, lo: float = 1e-3) -> Instance:
    """Large sparse instance with a block-banded part (width 64, stride 8)."""
    rng = np.random.default_rng(seed)
    A = block_band_csc(rng, m, n, k)
    return _finish(A, rng, frac, lo, f"sparse_blockband_m{m}_n{n}", seed)


def dense_planted(seed: int, m: int, n: int, frac: float = 0.4, lo: float = 0.1,
                  zero_pairs: int = 0) -> Instance:
    rng = np.random.default_rng(seed)
    A = gaussian_dense(rng, m, n)
    return _finish(A, rng, frac, lo, f"dense_m{m}_n{n}", seed, zero_pairs=zero_pairs)


def dense_batch(seed: int = 1003, count: int = 4096, n_lo: int = 16, n_hi: int = 256,
                frac: float = 0.4, lo: float = 0.1) -> List[Instance]:
    """Uneven batch of dense problems: n ~ U{n_lo..n_hi}, m ~ U{2n..4n}."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for i, ss in enumerate(children):
        rng = np.random.default_rng(ss)
        n = int(rng.integers(n_lo, n_hi + 1))
        m = int(rng.integers(2 * n, 4 * n + 1))
        A = gaussian_dense(rng, m, n)
        out.append(_finish(A, rng, frac, lo, f"batch{i}_m{m}_n{n}", seed))
    return out


def _serving_problem(rng, n: int, k: int, name: str, seed: int) -> Instance:
    m = 3 * n
    s = math.sqrt(k)
    A = rows_per_col_band_csc(rng, m, n, k, band=(s, s / 2, s / 4))
    frac = float(rng.uniform(0.3, 0.6))
    return _finish(A, rng, frac, 1e-3, name, seed)


def serving_stream(seed: int = 1004, count: int = 64, rate: float = 2000.0,
                   n_lo: int = 64, n_hi: int = 8192, k: int = 20):
    """Poisson arrival times (exponential gaps, mean 1/rate) and mixed sparse problems:
    n log-uniform in [n_lo, n_hi], m = 3n, k random rows per column plus a band of
    sqrt(k) * (1, 1/2, 1/4), active fraction ~ U[0.3, 0.6], margin 1e-3."""
    children = np.random.SeedSequence(seed).spawn(count + 1)
    trng = np.random.default_rng(children[0])
    arrivals = np.cumsum(trng.exponential(1.0 / rate, size=count))
    probs = []
    for i, ss in enumerate(children[1:]):
        rng = np.random.default_rng(ss)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        probs.append(_serving_problem(rng, n, k, f"serve{i}_m{3 * n}_n{n}", seed))
    return arrivals, probs


def serving_sizes(seed: int, ns, k: int = 20) -> List[Instance]:
    """Problems of the serving recipe at the given sizes n (one child stream each), so that
    a test can span the whole range [64, 8192] of the serving mix with a few requests."""
    children = np.random.SeedSequence(seed).spawn(len(ns))
    return [_serving_problem(np.random.default_rng(ss), int(n), k, f"serve_n{n}", seed)
            for ss, n in zip(children, ns)]


def fig2_matrix(rng, rows: int, density: float):
    """A matrix of the paper's speed experiment (Sec. 4, Fig. 2): rows x (rows - 10) with
    N(0,1) values; dense (column-major ndarray) at density 1.0, else a uniform random
    pattern of that density in CSC (the role MATLAB's sprandn plays in the paper), with a
    right-hand side b ~ N(0,1)."""
    m, n = rows, rows - 10
    if density >= 1.0:
        A = np.asfortranarray(rng.standard_normal((m, n)))
    else:
        A = _canonical_csc(sp.random(m, n, density=density, format="csc", random_state=rng,
                                     data_rvs=rng.standard_normal))
    return A, rng.standard_normal(m)


# the sizes (rows) of Fig. 2: density 1.0 and density 0.01
FIG2_DENSE_ROWS = (120, 200, 300, 499, 699, 938)
FIG2_SPARSE_ROWS = (820, 1000, 1200, 1420)


def svd_conditioned(seed: int, kappa: float, m: int = 80, n: int = 70, rep: int = 4):
    """Dense m x n matrix U diag(s) V^T with prescribed condition number: the distinct
    singular values are geometric from 1 down to 1/kappa and each is repeated ``rep``
    times (a stand-in for the P(m, n, rep, x) test matrices of the paper's Sec. 4).
    Returns (A, x_true, b) with x_true > 0 and b = A x_true, so the NNLS solution is
    x_true with every variable free."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, m)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    n_distinct = -(-n // rep)
    distinct = np.geomspace(1.0, 1.0 / kappa, n_distinct)
    s = np.repeat(distinct, rep)[:n]
    A = np.asfortranarray((U[:, :n] * s) @ V.T)
    x_true = rng.uniform(1.0, 2.0, size=n)
    return A, x_true, A @ x_true


def conditioned_planted(seed: int, m: int, n: int, kappa: float, frac: float = 0.4,
                        lo: float = 0.1) -> Instance:
    """Dense m x n problem whose planted free block is ill conditioned: the active columns
    are U diag(s) V^T with singular values geometric from 1 down to 1/kappa (so the final
    F-block of A^T A has condition kappa^2), the others N(0,1)/sqrt(m); planted
    complementary x*, y* as for every instance.  A float32 factor of that F-block
    contracts slowly under refinement."""
    rng = np.random.default_rng(seed)
    active, x_star, y_star = _plant_values(rng, n, frac, lo)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    k = int(active.sum())
    U, _ = np.linalg.qr(rng.standard_normal((m, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    A[:, active] = (U * np.geomspace(1.0, 1.0 / kappa, k)) @ V.T
    A = np.asfortranarray(A)
    b, dinf = _plant_rhs_dense(A, x_star, y_star)
    return Instance(A=A, b=np.ascontiguousarray(b), x_star=x_star, y_star=y_star, active=active,
                    delta_inf=dinf, name=f"conditioned_m{m}_n{n}_k{kappa:g}", seed=seed)


def csc_arrays(A: sp.csc_matrix):
    """(colptr int32[n+1], rowidx int32[nnz], val float64[nnz]) of a CSC matrix."""
    return (np.ascontiguousarray(A.indptr, dtype=np.int32),
            np.ascontiguousarray(A.indices, dtype=np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


def tiny_dense(seed: int):
    """Small ill-scaled dense problem (n in 3..8, m = n+1..n+3) with a random right-hand
    side and no planted solution.  Column scales span up to three decades and columns are
    mixed, which makes the pivoting take non-improving steps on some seeds (seed 1 takes
    every branch of the exchange rule)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 9))
    m = n + int(rng.integers(1, 4))
    A = rng.standard_normal((m, n)) @ np.diag(np.geomspace(1, 10 ** rng.uniform(0, 3), n))
    A = A @ (np.eye(n) + rng.uniform(0, 0.9) * rng.standard_normal((n, n)))
    b = rng.standard_normal(m)
    return np.asfortranarray(A), b


def random_dense(seed: int, m: int, n: int):
    """N(0,1)/sqrt(m) matrix and an N(0,1) right-hand side, no planted solution."""
    rng = np.random.default_rng(seed)
    return gaussian_dense(rng, m, n), rng.standard_normal(m)
