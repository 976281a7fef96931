"""The symbolic fill count that backs the dense F-block factor (Sec. 3 factors H_FF with a
sparse Cholesky; the solver factors it dense).  The counting functions are pinned on
patterns whose factor has a closed form, against a numeric Cholesky of random matrices with
the same pattern, and against each other; then the F-blocks of scaled-down workloads of
every sparse recipe are checked to fill nearly completely under all three orders."""
import numpy as np
import pytest
import scipy.sparse as sp

from tests import fill_check as FC


def _band(n, b):
    b = min(b, n - 1)
    return FC.symmetric_pattern(sp.diags([np.ones(n - d) for d in range(b + 1)],
                                         [-d for d in range(b + 1)], shape=(n, n), format="csc"))


def _arrow(n, hub):
    M = sp.lil_matrix((n, n))
    M[hub, :] = 1
    M[:, hub] = 1
    return FC.symmetric_pattern(M.tocsc())


def _random_pattern(rng, n, density):
    M = sp.random(n, n, density=density, random_state=rng, format="csc")
    return FC.symmetric_pattern(M)


@pytest.mark.parametrize("n,b", [(1, 0), (5, 1), (100, 0), (100, 3), (130, 70), (40, 60)])
def test_band_fills_nothing(n, b):
    """A band of half-width b factors within the band: column j keeps min(b, n-1-j)."""
    c = FC.column_counts(_band(n, b))
    assert c.tolist() == [min(b, n - 1 - j) for j in range(n)]


@pytest.mark.parametrize("n", [2, 9, 64, 65, 200])
def test_arrowhead_closed_forms(n):
    """Hub first: the factor is full.  Hub last: no fill.  Minimum degree finds the latter."""
    assert FC.column_counts(_arrow(n, 0)).tolist() == [n - 1 - j for j in range(n)]
    assert FC.column_counts(_arrow(n, n - 1)).tolist() == [1] * (n - 1) + [0]
    order, c = FC.min_degree(_arrow(n, 0))
    assert int(c.sum()) == n - 1
    assert FC.cholesky_nnz(_arrow(n, 0)) == n * (n + 1) // 2


def test_counts_match_a_numeric_cholesky():
    """Random patterns with random diagonally dominant values: the exact zeros of the numeric
    factor are the structural ones (no cancellation with probability one), in the natural
    order and in a random one."""
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(1, 48))
        P = _random_pattern(rng, n, float(rng.uniform(0.0, 0.25)))
        V = P.toarray().astype(np.float64) * rng.uniform(0.5, 1.5, size=(n, n))
        V = np.tril(V) + np.tril(V, -1).T
        V[np.diag_indices(n)] = np.abs(V).sum(axis=1) + 1.0
        for order in (None, rng.permutation(n)):
            W = V if order is None else V[np.ix_(order, order)]
            L = np.linalg.cholesky(W)
            numeric = [(np.abs(L[j + 1:, j]) > 0).sum() for j in range(n)]
            assert FC.column_counts(P, order).tolist() == numeric, (trial, n)


def test_min_degree_counts_are_its_orders_factor():
    """The degrees at elimination equal the elimination-tree count in the returned order."""
    rng = np.random.default_rng(6)
    for _ in range(25):
        n = int(rng.integers(1, 120))
        P = _random_pattern(rng, n, float(rng.uniform(0.0, 0.1)))
        order, c = FC.min_degree(P)
        assert sorted(order.tolist()) == list(range(n))
        assert FC.column_counts(P, order).tolist() == c.tolist()


def test_gram_pattern_matches_dense_product():
    rng = np.random.default_rng(7)
    A = sp.random(300, 40, density=0.05, random_state=rng, format="csc")
    cols = np.array([0, 3, 4, 9, 17, 22, 39])
    B = (np.abs(A[:, cols].toarray()) > 0).astype(np.int64)
    want = (B.T @ B > 0) | np.eye(cols.size, dtype=bool)
    assert np.array_equal(FC.gram_pattern(A, cols).toarray() > 0, want)


def test_workload_blocks_fill_nearly_completely():
    """F-blocks of the sparse recipes at a tenth of their sizes (serving at its own sizes):
    the factor keeps at least 75% of the dense triangle and 60% of its work even under
    minimum degree, and at least 85% of the triangle in the natural and reverse
    Cuthill-McKee orders.  A sparse factor would save well under half the work of the dense
    one, which runs on matrix cores."""
    for name, P in FC.workload_blocks(0.1):
        r = FC.fill_report(P)
        assert r["natural"][0] >= 0.85 and r["rcm"][0] >= 0.85, (name, r)
        assert r["min_degree"][0] >= 0.75 and r["min_degree"][1] >= 0.6, (name, r)
