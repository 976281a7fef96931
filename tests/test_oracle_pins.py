"""Pins for the CPU oracle: facts fixed by the paper or by mathematics, not by the oracle.

  * brute force over all 2^n splits (F, G) for n <= 10: Eq. 4 solved by an orthogonal
    least-squares routine, Eq. 5, feasibility test of Sec. 2; exactly one split is feasible
    for a strictly complementary problem and the oracle must land on it;
  * planted instances: the closed-form answer x*, y*, F* of the generator;
  * an independent NNLS routine (Lawson-Hanson active set, scipy.optimize.nnls);
  * the optimality conditions of Eq. 3 (x >= 0, y >= 0, <x, y> = 0, y = A^T A x - A^T b);
  * the error law of the normal-equations path printed in Fig. 1 (Sec. 4);
  * closed forms for orthogonal columns, and edge cases (empty F, breakdown, cap).
"""
import itertools
import os

import numpy as np
import pytest
import scipy.optimize as sopt
import scipy.sparse as sp

import workloads as W
from oracle import (BRANCH_BLOCK_BUDGET, BRANCH_BLOCK_IMPROVED, BRANCH_SINGLE, bpp_solve,
                    kkt_residuals,
                    gram, inverse_onenorm_estimate, predicted_rel_error, principal_block)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def brute_force(A, b, tol=1e-10):
    """All feasible complementary basic solutions (Sec. 2), via lstsq (QR/SVD based)."""
    m, n = A.shape
    feas = []
    for mask in itertools.product([False, True], repeat=n):
        F = np.array(mask)
        x = np.zeros(n)
        if F.any():
            x[F] = np.linalg.lstsq(A[:, F], b, rcond=None)[0]
        y = A.T @ (A @ x - b)
        y[F] = 0.0
        scale = 1.0 + np.abs(x).max() + np.abs(y).max()
        if x[F].min(initial=0) >= -tol * scale and y[~F].min(initial=0) >= -tol * scale:
            feas.append((F, x, y))
    return feas


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("p_max", [3, 0])
def test_bruteforce_random_dense(seed, p_max):
    rng = np.random.default_rng(seed)
    n = 1 + seed % 10
    A, b = W.random_dense(500 + seed, 2 * n + 1, n)
    feas = brute_force(A, b)
    assert len(feas) == 1, "random problem should have a unique feasible split"
    F, x, y = feas[0]
    r = bpp_solve(A, b, p_max=p_max)
    assert r.status == "ok"
    assert np.array_equal(r.free, F)
    assert np.allclose(r.x, x, rtol=1e-12, atol=1e-12)
    assert np.allclose(r.y, y, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", range(1, 41))
@pytest.mark.parametrize("p_max", [3, 0])
def test_bruteforce_ill_scaled(seed, p_max):
    A, b = W.tiny_dense(seed)
    feas = brute_force(A, b, tol=1e-9)
    r = bpp_solve(A, b, p_max=p_max)
    assert r.status == "ok"
    assert any(np.array_equal(r.free, F) for F, _, _ in feas)
    F, x, y = next(f for f in feas if np.array_equal(r.free, f[0]))
    assert np.allclose(r.x, x, rtol=1e-8, atol=1e-10 * np.abs(x).max())


def test_every_branch_reaches_brute_force_answer():
    """Seed 1 of the ill-scaled family takes the improving block exchange, the budgeted
    block exchange and the single exchange; each path must still end at the unique
    feasible split."""
    A, b = W.tiny_dense(1)
    (F, x, y), = brute_force(A, b, tol=1e-9)
    for p_max in (3, 0):
        r = bpp_solve(A, b, p_max=p_max)
        branches = {t.branch for t in r.trace}
        assert BRANCH_SINGLE in branches and BRANCH_BLOCK_IMPROVED in branches
        if p_max == 3:
            assert BRANCH_BLOCK_BUDGET in branches
        assert np.array_equal(r.free, F)
        assert np.allclose(r.x, x, rtol=1e-9, atol=1e-12)


def test_budget_counts_down_from_three():
    """After an improving step the budget is 3 (Sec. 2 box); a run of non-improving steps
    spends it one by one before the single exchange is taken."""
    A, b = W.tiny_dense(1)
    r = bpp_solve(A, b)
    for prev, cur in zip(r.trace, r.trace[1:]):
        if cur.branch == BRANCH_BLOCK_BUDGET:
            assert cur.p == prev.p - 1 and cur.k >= prev.N
        if cur.branch == BRANCH_SINGLE:
            assert prev.p == 0 and cur.k >= prev.N
            assert cur.n_free == prev.n_free + 1 or cur.n_free == prev.n_free - 1
        if cur.branch == BRANCH_BLOCK_IMPROVED:
            assert cur.k < prev.N and cur.p == 3


@pytest.mark.parametrize("seed", range(1001, 1006))
def test_planted_sparse_small(seed):
    inst = W.sparse_small(seed)
    r = bpp_solve(inst.A, inst.b)
    assert r.status == "ok"
    assert np.array_equal(r.free, inst.active)
    assert np.abs(r.x - inst.x_star).max() <= 1e-10
    assert np.abs(r.y - inst.y_star).max() <= 1e-10
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, r.x, r.y)
    assert nx == 0.0 and ny == 0.0 and comp == 0.0 and dres < 1e-10


@pytest.mark.parametrize("m,n,seed", [(40, 16, 1), (300, 100, 2), (700, 256, 3)])
def test_planted_dense(m, n, seed):
    inst = W.dense_planted(seed, m, n)
    r = bpp_solve(inst.A, inst.b)
    assert r.status == "ok"
    assert np.array_equal(r.free, inst.active)
    assert np.abs(r.x - inst.x_star).max() <= 1e-11
    assert np.abs(r.y - inst.y_star).max() <= 1e-11


@pytest.mark.slow
def test_planted_sparse_large_reduced():
    """The large sparse recipe at a quarter of its size in each dimension."""
    inst = W.sparse_large(1002, m=15000, n=3000)
    r = bpp_solve(inst.A, inst.b)
    assert r.status == "ok"
    assert np.array_equal(r.free, inst.active)
    assert np.abs(r.x - inst.x_star).max() <= 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_matches_lawson_hanson(seed):
    m, n = [(60, 40), (120, 80), (30, 29), (200, 10), (90, 45), (64, 64)][seed]
    A, b = W.random_dense(900 + seed, m, n)
    r = bpp_solve(A, b)
    x_lh, _ = sopt.nnls(A, b, maxiter=50 * n)
    assert r.status == "ok"
    assert np.allclose(r.x, x_lh, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("zero_pairs", [1, 5])
def test_degenerate_planted_satisfies_kkt(zero_pairs):
    inst = W.dense_planted(77 + zero_pairs, 120, 60, zero_pairs=zero_pairs)
    r = bpp_solve(inst.A, inst.b)
    assert r.status == "ok"
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, r.x, r.y)
    assert nx == 0.0 and ny == 0.0 and comp == 0.0 and dres < 1e-11
    # x is unique even though the split is not
    assert np.abs(r.x - inst.x_star).max() < 1e-10


def test_error_law_matches_fig1():
    """Normal-equations error vs condition number, against the paper's Fig. 1 data
    (x markers, 109 points): the fitted line through the printed points must predict the
    oracle's error within 0.75 decade for log10(kappa) in [1.5, 6]."""
    d = np.loadtxt(os.path.join(GOLDEN, "fig1_normal_equations_error.txt"))
    lk = 1 + (d[:, 0] - 120) * 7 / 1319
    le = -16 + (d[:, 1] - 82) * 18 / 778
    slope, icpt = np.polyfit(lk, le, 1)
    assert 1.9 < slope < 2.15            # the kappa^2 eps law stated in Sec. 2.1 / Sec. 4
    for lkap in (1.5, 2.5, 3.5, 4.5, 5.5, 6.0):
        errs = []
        for s in range(5):
            A, xt, b = W.svd_conditioned(100 + s, 10 ** lkap)
            r = bpp_solve(A, b)
            assert r.status == "ok"
            errs.append(np.linalg.norm(r.x - xt) / np.linalg.norm(xt))
        got = np.median(np.log10(errs))
        assert abs(got - (slope * lkap + icpt)) < 0.75, (lkap, got)


def test_orthogonal_columns_closed_form():
    """Orthogonal columns make A^T A diagonal, so x_i = max(c_i / h_ii, 0), and the first
    block exchange already lands on it: one iteration with k = #{c_i > 0}."""
    rng = np.random.default_rng(5)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((50, n)))
    d = rng.uniform(0.5, 3.0, n)
    A = Q * d
    b = rng.standard_normal(50)
    c = A.T @ b
    r = bpp_solve(A, b)
    assert r.status == "ok" and r.iterations == 1
    assert r.trace[0].k == int((c > 0).sum())
    assert np.allclose(r.x, np.maximum(c / d ** 2, 0), rtol=1e-12, atol=1e-14)


def test_empty_free_set():
    """A^T b <= 0 makes x = 0 optimal before any exchange; y = -A^T b."""
    A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    b = np.array([-1.0, -2.0, 0.5])
    r = bpp_solve(A, b)
    assert r.status == "ok" and r.iterations == 0
    assert np.array_equal(r.x, np.zeros(2))
    assert np.allclose(r.y, -(A.T @ b))


def test_zeroing_threshold():
    """A component of A^T b within 1e-12 of zero is zeroed and never counted (Sec. 2)."""
    A = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    b = np.array([-5e-13, 2.0, 7.0])
    r = bpp_solve(A, b)
    assert r.status == "ok" and r.iterations == 1
    assert r.y[0] == 0.0 and r.x[0] == 0.0 and r.x[1] == 2.0
    r2 = bpp_solve(A, b, tau=1e-13)
    assert r2.free[0] == False and r2.y[0] == 5e-13


def test_breakdown_reports_column():
    """Two identical unit columns make the F-block singular once both are free: the
    second pivot is exactly zero (Sec. 2.1 breakdown), reported at column 1."""
    A = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    b = np.array([1.0, 1.0, 0.0, 0.0])
    r = bpp_solve(A, b)
    assert r.status == "not_pd" and r.failed_index == 1


def test_iteration_cap():
    A, b = W.tiny_dense(1)
    r = bpp_solve(A, b, max_iter=2)
    assert r.status == "maxiter" and r.iterations == 2 and r.last_ninf > 0


def test_sparse_and_dense_inputs_agree():
    inst = W.sparse_small(1001, m=300, n=60, density=0.1)
    rs = bpp_solve(inst.A, inst.b)
    rd = bpp_solve(inst.A.toarray(), inst.b)
    assert np.array_equal(rs.free, rd.free)
    assert np.allclose(rs.x, rd.x, rtol=1e-13, atol=1e-15)


# ---- condition estimate of the final F-block (Sec. 3: dpocon-style error control) ----

def _exact_inv_onenorm(H):
    return float(np.abs(np.linalg.inv(H)).sum(axis=0).max())


def test_inverse_onenorm_estimate_is_a_tight_lower_bound():
    """Hager/Higham estimate: never above the true ||H^-1||_1, and within a factor 3 of it
    on random SPD matrices with condition numbers up to 1e8."""
    rng = np.random.default_rng(11)
    for _ in range(150):
        n = int(rng.integers(2, 60))
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        H = (Q * np.geomspace(1.0, 10.0 ** rng.uniform(0, 8), n)) @ Q.T
        H = (H + H.T) / 2
        exact, est = _exact_inv_onenorm(H), inverse_onenorm_estimate(H)
        assert est <= exact * (1 + 1e-6)
        assert est >= exact / 3


def test_inverse_onenorm_estimate_closed_forms():
    # diagonal: the method finds the largest 1/d_i exactly
    d = np.array([4.0, 0.5, 2.0, 8.0, 0.25, 1.0])
    assert inverse_onenorm_estimate(np.diag(d)) == pytest.approx(4.0, rel=1e-15)
    # [[2,-1],[-1,2]]^-1 = [[2,1],[1,2]] / 3, whose 1-norm is 1
    assert inverse_onenorm_estimate(np.array([[2.0, -1.0], [-1.0, 2.0]])) == pytest.approx(1.0, rel=1e-14)
    assert inverse_onenorm_estimate(np.array([[4.0]])) == pytest.approx(0.25, rel=1e-15)


def test_predicted_error_bounds_the_fig1_errors():
    """0.1 kappa_1(A_F^T A_F) eps (Sec. 2.1, Sec. 4's constant) against the oracle's actual
    error on the Fig. 1 problems: above it, by less than a factor 30."""
    for lk in (1.5, 2.0, 3.0, 4.0, 5.0, 6.0):
        for seed in range(3):
            A, xt, b = W.svd_conditioned(seed, kappa=10.0 ** lk)
            res = bpp_solve(A, b)
            H, _ = gram(A, b)
            Hff = principal_block(H, np.flatnonzero(res.free))
            Hff = Hff.toarray() if hasattr(Hff, "toarray") else Hff
            err = np.linalg.norm(res.x - xt) / np.linalg.norm(xt)
            pred = predicted_rel_error(Hff)
            assert err <= pred <= 30 * err, (lk, seed, err, pred)


# ---- the single exchange of the Sec. 2 algorithm box, worked by hand ----
#
# A (4 x 3) and b are small integers, so every step can be done exactly by hand:
#   H = A^T A = [[23, -1, -2], [-1, 21, 5], [-2, 5, 2]],   c = A^T b = [-3, 4, 4].
# Start: F = {}, x = 0, y = -c = [3, -4, -4]; the infeasible set is {1, 2}, k = 2 < N = inf:
#   improving block exchange, N = 2, F = {1, 2}.
# F = {1, 2}: [[21, 5], [5, 2]] x_F = [4, 4] gives x_1 = -12/17, x_2 = 64/17, and
#   y_0 = H_01 x_1 + H_02 x_2 - c_0 = 12/17 - 128/17 + 3 = -65/17.
#   Infeasible: {0 (y_0 < 0), 1 (x_1 < 0)}, k = 2, not below N = 2.
#   * p_max = 0: the budget is spent, so only the infeasible variable of LARGEST index, 1,
#     changes side: F = {2}.  (Flipping 0 instead would give F = {0, 1, 2}.)
#     F = {2}: x_2 = 4 / 2 = 2, y_0 = -4 + 3 = -1, y_1 = 10 - 4 = 6; k = 1 < N: F = {0, 2}.
#   * p_max = 3: budgeted block exchange, p = 2, both change side: F = {0, 2}.
# F = {0, 2}: [[23, -2], [-2, 2]] x_F = [-3, 4] gives x_0 = 1/21, x_2 = 43/21, and
#   y_1 = -1/21 + 5 * 43/21 - 4 = 130/21 > 0: feasible, stop.
HAND_A = np.array([[2.0, -2.0, 0.0], [3.0, 2.0, 0.0], [-3.0, 2.0, 1.0], [-1.0, -3.0, -1.0]])
HAND_B = np.array([1.0, -3.0, 0.0, -4.0])
HAND_X = np.array([1.0 / 21.0, 0.0, 43.0 / 21.0])
HAND_Y = np.array([0.0, 130.0 / 21.0, 0.0])
# per iteration: (k, branch, N, p, F after the exchange)
HAND_TRACE = {
    0: [(2, BRANCH_BLOCK_IMPROVED, 2, 0, {1, 2}), (2, BRANCH_SINGLE, 2, 0, {2}),
        (1, BRANCH_BLOCK_IMPROVED, 1, 0, {0, 2})],
    3: [(2, BRANCH_BLOCK_IMPROVED, 2, 3, {1, 2}), (2, BRANCH_BLOCK_BUDGET, 2, 2, {0, 2})],
}


def test_hand_worked_instance_data():
    """The Gram matrix and right-hand side used in the hand computation above."""
    assert np.array_equal(HAND_A.T @ HAND_A, [[23, -1, -2], [-1, 21, 5], [-2, 5, 2]])
    assert np.array_equal(HAND_A.T @ HAND_B, [-3, 4, 4])


@pytest.mark.parametrize("p_max", [0, 3])
def test_single_exchange_takes_the_largest_index(p_max):
    """Sec. 2 algorithm box, worked by hand: with the budget spent, of the two infeasible
    variables {0, 1} only the one of largest index (1) changes side.  The trajectory of
    free sets is fixed by the hand computation; taking any other index changes the second
    free set."""
    r = bpp_solve(HAND_A, HAND_B, p_max=p_max)
    assert r.status == "ok"
    want = HAND_TRACE[p_max]
    assert len(r.trace) == len(want)
    free_sets = []
    free = np.zeros(3, dtype=bool)
    for row, (k, branch, N, p, F) in zip(r.trace, want):
        assert (row.k, row.branch, row.N, row.p, row.n_free) == (k, branch, N, p, len(F))
        free_sets.append(F)
    assert set(np.flatnonzero(r.free)) == want[-1][4]
    assert np.allclose(r.x, HAND_X, rtol=1e-14, atol=1e-15)
    assert np.allclose(r.y, HAND_Y, rtol=1e-14, atol=1e-15)


def test_single_exchange_free_sets_step_by_step():
    """The same hand-worked run, one box iteration at a time through the oracle's own
    steps (classify, exchange rule, solve, dual), checking the free set after each
    exchange against the hand computation."""
    from oracle import classify, dual, exchange_rule, solve_free
    H, c = gram(HAND_A, HAND_B)
    free = np.zeros(3, dtype=bool)
    x, y = np.zeros(3), -c.copy()
    N, p = np.inf, 0
    for k_want, branch_want, _, _, F_want in HAND_TRACE[0]:
        infeasible, _ = classify(x, y, free, 1e-12)
        assert int(infeasible.sum()) == k_want
        N, p, branch = exchange_rule(int(infeasible.sum()), N, p, 0)
        assert branch == branch_want
        if branch == BRANCH_SINGLE:
            assert set(np.flatnonzero(infeasible)) == {0, 1}
            free[int(np.flatnonzero(infeasible).max())] ^= True
        else:
            free ^= infeasible
        assert set(np.flatnonzero(free)) == F_want
        idx_f, idx_g = np.flatnonzero(free), np.flatnonzero(~free)
        xF, failed = solve_free(H, c, idx_f)
        assert failed == -1
        x = np.zeros(3)
        x[idx_f] = xF
        y = np.zeros(3)
        y[idx_g] = dual(HAND_A, HAND_B, idx_f, xF, idx_g)
    infeasible, _ = classify(x, y, free, 1e-12)
    assert not infeasible.any()


# ---- non-finite values (no sign test can decide them) ----

def test_non_finite_input_is_reported():
    A, b = W.random_dense(5, 12, 6)
    b = b.copy()
    b[3] = np.nan
    assert bpp_solve(A, b).status == "invalid_value"
    A2 = A.copy()
    A2[2, 1] = np.inf
    assert bpp_solve(A2, W.random_dense(5, 12, 6)[1]).status == "invalid_value"


NONFINITE_A = np.array([[1e300, 0.0], [0.0, 1.0], [0.0, 1.0]])
NONFINITE_B = np.array([1e10, 1.0, 1.0])


def test_non_finite_iterate_is_reported():
    """Finite A and b whose A^T b overflows (1e300 * 1e10): the first tested entry,
    y_0 = -c_0, is -inf.  No sign test can decide it, so the loop stops with
    invalid_value instead of exchanging on it."""
    with np.errstate(over="ignore", invalid="ignore"):
        r = bpp_solve(NONFINITE_A, NONFINITE_B)
    assert r.status == "invalid_value" and r.iterations == 0
