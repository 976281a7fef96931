"""GPU parity on the paper's own cases and on the method's degenerate and failure cases:

  * the hand-worked single-exchange instance of the Sec. 2 algorithm box (the expected
    trajectory is the hand computation in test_oracle_pins.py, not the oracle's output);
  * the matrices of the paper's speed experiment (Sec. 4, Fig. 2): n x (n - 10) at
    density 1.0 and 0.01, at the paper's sizes, against the oracle;
  * degenerate planted instances (inactive variables with y*_i = 0 as well): x unique,
    checked against the planted x*, the oracle and the optimality conditions of Eq. 3;
  * non-finite iterates, which no sign test can decide;
  * the mixed path's float64 redo of an iteration whose float32 factor fails, on an
    F-block of several tile columns.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import bpp_solve, kkt_residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402
from _gpu_util import DEV, certified, colmajor_dev, oracle_trace, solve_csc, solve_dense, t  # noqa: E402
from test_oracle_pins import HAND_A, HAND_B, HAND_TRACE, HAND_X, HAND_Y, NONFINITE_A, NONFINITE_B  # noqa: E402


@pytest.fixture(scope="module")
def h():
    with N.Handle(0) as hh:
        yield hh


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


# ------------------------------------------------------------------ hand-worked box run
@pytest.mark.parametrize("p_max", [0, 3])
@pytest.mark.parametrize("path", ["dense", "sparse"])
def test_single_exchange_hand_worked(h, p_max, path):
    """Sec. 2 box by hand: with the budget spent, the infeasible variable of largest index
    (1 of {0, 1}) changes side.  Trace (k, branch, N, p, |F|) and x, y as computed by hand."""
    solve = solve_dense if path == "dense" else solve_csc
    A = HAND_A if path == "dense" else sp.csc_matrix(HAND_A)
    st, info, x, y, trace = solve(h, A, HAND_B, p_max=p_max)
    assert st == N.NNLS_OK
    assert trace == [(k, br, Nn, p, len(F)) for k, br, Nn, p, F in HAND_TRACE[p_max]]
    assert np.allclose(x, HAND_X, rtol=1e-13, atol=1e-15)
    assert np.allclose(y, HAND_Y, rtol=1e-13, atol=1e-14)
    assert set(np.flatnonzero(x > 0)) == HAND_TRACE[p_max][-1][4]


def test_single_exchange_hand_worked_batched(h):
    """The same instance in a batched launch (one workgroup runs the whole box)."""
    for p_max in (0, 3):
        A = colmajor_dev(HAND_A)
        b = t(HAND_B)
        x = torch.empty(3, dtype=torch.float64, device=DEV)
        y = torch.empty_like(x)
        st, infos = N.nnls_solve_dense_batched(h, [A], [b], [x], [y], N.default_options(p_max=p_max))
        assert st == N.NNLS_OK and infos[0].iterations == len(HAND_TRACE[p_max])
        assert np.allclose(x.cpu().numpy(), HAND_X, rtol=1e-13, atol=1e-15)


# ------------------------------------------------------------------ Fig. 2 matrices
def _fig2_cases():
    rng = np.random.default_rng(1008)
    cases = []
    for rows in W.FIG2_DENSE_ROWS:
        A, b = W.fig2_matrix(rng, rows, 1.0)
        cases.append(("dense", rows, A, b))
    for rows in W.FIG2_SPARSE_ROWS:
        A, b = W.fig2_matrix(rng, rows, 0.01)
        cases.append(("sparse", rows, A, b))
    return cases


FIG2 = _fig2_cases()


@pytest.mark.parametrize("case", range(len(FIG2)), ids=[f"{c[0]}{c[1]}" for c in FIG2])
def test_fig2_matrices_match_oracle(h, case):
    """The paper's speed workload (Sec. 4, Fig. 2): random rows x (rows - 10) matrices with
    N(0,1) values, dense and at density 0.01, b ~ N(0,1).  Plain float64 path against the
    oracle: same free set, same trajectory where certified, x and y within 1e-10 (widened
    to 100 kappa(H_FF) eps for an ill-conditioned final block)."""
    kind, rows, A, b = FIG2[case]
    res = bpp_solve(A, b)
    st, info, x, y, trace = (solve_dense if kind == "dense" else solve_csc)(h, A, b)
    assert res.status == "ok" and st == N.NNLS_OK, N.status_string(st)
    Ad = A if kind == "dense" else A.toarray()
    Hff = (Ad.T @ Ad)[np.ix_(res.free, res.free)]
    kappa = np.linalg.cond(Hff) if res.free.any() else 1.0
    tol = max(1e-10, 100 * kappa * np.finfo(float).eps)
    scale = np.abs(Ad).max() * np.abs(b).max()
    if certified(res, scale, rel=1e-8):
        assert np.array_equal(x > 0, res.x > 0)
        assert trace == oracle_trace(res)
    assert relerr(x, res.x) <= tol
    assert np.linalg.norm(y - res.y) <= tol * max(np.linalg.norm(res.y), 1.0)
    assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0


# ------------------------------------------------------------------ degenerate instances
@pytest.mark.parametrize("zero_pairs", [1, 5, 40])
def test_degenerate_planted_dense(h, zero_pairs):
    """Inactive variables with y*_i = 0 as well: several splits are optimal, x is unique.
    x against the planted x* and the oracle's x; y >= 0, x >= 0, x^T y = 0 and
    y = A^T A x - A^T b (Eq. 3)."""
    inst = W.dense_planted(77 + zero_pairs, 120, 60, zero_pairs=zero_pairs)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b)
    assert st == N.NNLS_OK and res.status == "ok"
    assert np.abs(x - inst.x_star).max() < 1e-10
    assert relerr(x, res.x) <= 1e-10
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, x, y)
    assert nx == 0 and ny == 0 and comp == 0 and dres < 1e-11


@pytest.mark.parametrize("precision,tol", [(N.NNLS_FP64, 1e-10), (N.NNLS_FP32_IR, 1e-8)])
def test_degenerate_planted_sparse(h, precision, tol):
    """The large sparse recipe at 6000 x 1200 with 60 degenerate pairs, both precisions."""
    inst = W.sparse_large(21, m=6000, n=1200, zero_pairs=60)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=precision)
    assert st == N.NNLS_OK and res.status == "ok"
    assert np.abs(x - inst.x_star).max() < 100 * tol
    assert relerr(x, res.x) <= tol
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, x, y)
    assert nx == 0 and ny == 0 and comp == 0 and dres < 1e-9


# ------------------------------------------------------------------ non-finite iterates
def test_non_finite_iterate_single_problem(h):
    """Finite A and b whose A^T b overflows: the first tested entry is -inf, which the
    control step reports as NNLS_ERR_INVALID_VALUE (the oracle does the same)."""
    with np.errstate(over="ignore", invalid="ignore"):
        assert bpp_solve(NONFINITE_A, NONFINITE_B).status == "invalid_value"
    st, info, *_ = solve_dense(h, NONFINITE_A, NONFINITE_B)
    assert st == N.NNLS_ERR_INVALID_VALUE and info.status == st
    st, info, *_ = solve_csc(h, sp.csc_matrix(NONFINITE_A), NONFINITE_B)
    assert st == N.NNLS_ERR_INVALID_VALUE


def test_non_finite_iterate_batched(h):
    As = [colmajor_dev(NONFINITE_A), colmajor_dev(HAND_A)]
    bs = [t(NONFINITE_B), t(HAND_B)]
    xs = [torch.empty(2, dtype=torch.float64, device=DEV), torch.empty(3, dtype=torch.float64, device=DEV)]
    ys = [torch.empty_like(v) for v in xs]
    st, infos = N.nnls_solve_dense_batched(h, As, bs, xs, ys)
    assert st == N.NNLS_ERR_INVALID_VALUE
    assert infos[0].status == N.NNLS_ERR_INVALID_VALUE and infos[1].status == N.NNLS_OK
    assert np.allclose(xs[1].cpu().numpy(), HAND_X, rtol=1e-13, atol=1e-15)


def test_pivot_step_rejects_nan(h):
    x = t(np.array([0.5, np.nan, 0.0, 0.0]))
    y = t(np.array([0.0, 0.0, -1.0, 2.0]))
    flags = t(np.array([1, 1, 0, 0], dtype=np.uint8))
    state = [-1, 3]
    st, out = N.nnls_pivot_step(h, x, y, flags, 1e-12, 3, state)
    assert st == N.NNLS_ERR_INVALID_VALUE
    assert np.array_equal(flags.cpu().numpy(), [1, 1, 0, 0])   # nothing exchanged


# ------------------------------------------------------------------ mixed-precision redo
def test_mixed_redo_in_float64_on_multi_tile_block(h):
    """kappa(A) = 1e5 (kappa(H) = 1e10): the float32 factor breaks down or its refinement
    stalls, so each iteration is redone with a float64 factor.  The F-blocks have up to 300
    positions (5 tile columns), so the redo's factor waits on its own column counters and
    runs its own backward solve.  Result against the known solution and against the float64
    path with the same float64 refinement (NNLS_FLAG_REFINE_FINAL)."""
    A, xt, b = W.svd_conditioned(7, 1e5, m=360, n=300)
    N.nnls_reset_profile(h)
    st, info, x, y, trace = solve_dense(h, A, b, precision=N.NNLS_FP32_IR, flags=N.NNLS_FLAG_PROFILE)
    prof = N.nnls_get_profile(h)
    assert st == N.NNLS_OK, N.status_string(st)
    assert prof["cholesky"]["launches"] > info.iterations        # at least one float64 redo
    assert info.n_free == 300 and np.all(x > 0)
    assert relerr(x, xt) <= 1e-9
    st2, info2, x2, y2, trace2 = solve_dense(h, A, b, flags=N.NNLS_FLAG_REFINE_FINAL)
    assert st2 == N.NNLS_OK and info2.n_free == 300
    assert relerr(x, x2) <= 1e-9
