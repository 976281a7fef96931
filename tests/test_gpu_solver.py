"""Solver parity: the GPU pivot loop through the C ABI against the CPU oracle on the same
seeded inputs.  The final free set must be identical; x and y must agree to 1e-10
relative (FP64 path); the per-iteration trace (k, branch, N, p, |F|) must be identical
whenever every sign test of the run was certified (no tested value within 1e-8 relative
of the zeroing threshold)."""
import numpy as np
import scipy.linalg as sla
import pytest

import workloads as W
from oracle import bpp_solve, kkt_residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402
from _gpu_util import DEV, certified, colmajor_dev, oracle_trace, solve_csc, solve_dense, t  # noqa: E402

RTOL = 1e-10


@pytest.fixture(scope="module")
def h():
    with N.Handle(0) as hh:
        yield hh


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def check_parity(res, st, info, x, y, trace, rtol=RTOL, scale=1.0):
    assert st == N.NNLS_OK, N.status_string(st)
    assert res.status == "ok"
    assert info.iterations == res.iterations
    assert info.n_free == int(res.free.sum())
    assert np.array_equal(np.flatnonzero(x != 0), np.flatnonzero(res.x != 0))
    assert relerr(x, res.x) <= rtol
    assert np.linalg.norm(y - res.y) <= rtol * max(np.linalg.norm(res.y), 1.0)
    assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0
    if certified(res, scale):
        assert trace == oracle_trace(res)


@pytest.mark.parametrize("seed", range(1001, 1006))
def test_sparse_small_full_size(h, seed):
    """m = 2000, n = 400, 2% Bernoulli N(0,1) plus diagonal, planted, FP64."""
    inst = W.sparse_small(seed)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b)
    check_parity(res, st, info, x, y, trace)
    assert np.array_equal(x > 0, inst.active)


@pytest.mark.parametrize("m,n,seed", [(2400, 480, 7), (6000, 1200, 8), (15000, 3000, 9)])
def test_sparse_large_recipe_reduced(h, m, n, seed):
    inst = W.sparse_large(seed, m=m, n=n)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b)
    check_parity(res, st, info, x, y, trace)


def test_sparse_large_full_size(h):
    """m = 60000, n = 12000, 25 N(0,1) per column + band, 30% active, margin 1e-3 -- the
    benchmark workload, element by element against the oracle and the planted answer."""
    inst = W.sparse_large(1002)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b)
    assert st == N.NNLS_OK
    assert np.array_equal(x > 0, inst.active)
    assert np.abs(x - inst.x_star).max() <= 1e-10
    assert np.abs(y - inst.y_star).max() <= 1e-10
    res = bpp_solve(inst.A, inst.b)
    check_parity(res, st, info, x, y, trace)
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, x, y)
    assert nx == 0 and ny == 0 and comp == 0 and dres < 1e-9


def test_sparse_large_f_block_beyond_one_window(h):
    """m = 200000, n = 44000 of the same recipe: the first F-block has 35163 positions, so
    the F-position lists span two 32768-position windows and the Gram columns two row
    windows.  Checked against the planted answer and the KKT conditions (the oracle is too
    slow at this size)."""
    inst = W.sparse_large(1006, m=200000, n=44000)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b)
    assert st == N.NNLS_OK
    assert trace[0][4] == 35163
    assert np.array_equal(x > 0, inst.active)
    assert np.abs(x - inst.x_star).max() <= 1e-10
    assert np.abs(y - inst.y_star).max() <= 1e-10
    nx, ny, comp, dres = kkt_residuals(inst.A, inst.b, x, y)
    assert nx == 0 and ny == 0 and comp == 0 and dres < 1e-9


@pytest.mark.parametrize("m,n,seed", [(40, 16, 1), (300, 100, 2), (700, 256, 3), (1100, 520, 4)])
def test_dense_planted(h, m, n, seed):
    inst = W.dense_planted(seed, m, n)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b)
    check_parity(res, st, info, x, y, trace)
    assert np.array_equal(x > 0, inst.active)


@pytest.mark.parametrize("seed", range(12))
def test_dense_random_rhs(h, seed):
    n = 1 + seed * 7
    A, b = W.random_dense(500 + seed, 2 * n + 1, n)
    res = bpp_solve(A, b)
    st, info, x, y, trace = solve_dense(h, A, b)
    check_parity(res, st, info, x, y, trace)


@pytest.mark.parametrize("seed", range(1, 41))
def test_ill_scaled_all_branches(h, seed):
    """Small ill-scaled problems that take the budget and single-exchange branches."""
    A, b = W.tiny_dense(seed)
    res = bpp_solve(A, b)
    st, info, x, y, trace = solve_dense(h, A, b)
    assert st == N.NNLS_OK and res.status == "ok"
    Hff = (A.T @ A)[np.ix_(res.free, res.free)]
    kappa = np.linalg.cond(Hff) if res.free.any() else 1.0
    tol = max(RTOL, 100 * kappa * np.finfo(float).eps)
    if certified(res, np.abs(A).max() * np.abs(b).max(), rel=1e-6):
        assert np.array_equal(x != 0, res.x != 0)
        assert trace == oracle_trace(res)
    assert relerr(x, res.x) <= tol


def test_sparse_path_equals_dense_path(h):
    inst = W.sparse_small(1001, m=800, n=200, density=0.05)
    st1, info1, x1, y1, tr1 = solve_csc(h, inst.A, inst.b)
    st2, info2, x2, y2, tr2 = solve_dense(h, inst.A.toarray(), inst.b)
    assert st1 == st2 == N.NNLS_OK and tr1 == tr2
    assert relerr(x1, x2) <= 1e-12


def test_rerun_is_bitwise_identical(h):
    inst = W.sparse_large(1002, m=6000, n=1200)
    a = solve_csc(h, inst.A, inst.b)
    b = solve_csc(h, inst.A, inst.b)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4] == b[4]


@pytest.mark.parametrize("cap,precision", [(1, 0), (7, 0), (64, 0), (7, 1), (64, 2)])
def test_capped_persistent_grid_is_bitwise_identical(h, cap, precision):
    """A capped factor grid (fewer persistent workgroups taking the tile tickets) computes
    every tile with the same operations in the same order as one workgroup per tile.  (The
    bfloat16-update factor's row walkers below a kept block need a cap of at least the new
    tile rows + 9; a cap of 64 leaves them on.)"""
    inst = W.sparse_large(1002, m=6000, n=1200)
    a = solve_csc(h, inst.A, inst.b, precision=precision)
    b = solve_csc(h, inst.A, inst.b, precision=precision, max_workgroups=cap)
    assert a[0] == b[0] == N.NNLS_OK
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4] == b[4]


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-10), (2, 1e-10)])
@pytest.mark.parametrize("m,n,cap", [(6000, 1200, 0), (60000, 12000, 0), (6000, 1200, 7)])
def test_kept_factor_tiles_match_full_refactor(h, m, n, cap, precision, tol):
    """The factor keeps the leading tile columns that no exchange touched (F ordered so
    that they come first); against refactoring the whole F-block every iteration it takes
    the same pivot steps and gives x within rounding, and the later iterations keep tiles.
    With bfloat16 updates (precision 2) the rows below a kept block go through the row
    walkers and the previous factor's coupling tiles."""
    inst = W.sparse_large(1002, m=m, n=n)
    kw = dict(precision=precision, max_workgroups=cap)
    st1, info1, x1, y1, _ = solve_csc(h, inst.A, inst.b, **kw)
    tr1 = N.nnls_get_trace(h, reused=True)
    st2, info2, x2, y2, _ = solve_csc(h, inst.A, inst.b, flags=N.NNLS_FLAG_NO_FACTOR_REUSE, **kw)
    tr2 = N.nnls_get_trace(h, reused=True)
    assert st1 == st2 == N.NNLS_OK
    assert [r[:5] for r in tr1] == [r[:5] for r in tr2]
    assert all(r[5] == 0 for r in tr2)
    kept = [r[5] for r in tr1]
    assert kept[0] == 0 and all(k % 64 == 0 and k < nf for k, nf in zip(kept, [r[4] for r in tr1]))
    assert sum(kept) > 0
    assert np.array_equal(x1 > 0, x2 > 0) and np.array_equal(x1 > 0, inst.active)
    assert relerr(x1, x2) <= tol
    assert np.linalg.norm(y1 - y2) <= tol * max(np.linalg.norm(y2), 1.0)


@pytest.mark.parametrize("m,n,seed", [(300, 100, 2), (1100, 520, 4), (3000, 1000, 5)])
def test_gram_dual_dense_matches_oracle(h, m, n, seed):
    """NNLS_FLAG_GRAM_DUAL on the dense single-problem path (y_G from the cached dense Gram
    matrix, Eq. 3): the oracle's pivot steps, free set, x and y."""
    inst = W.dense_planted(seed, m, n)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b, flags=N.NNLS_FLAG_GRAM_DUAL)
    check_parity(res, st, info, x, y, trace)


def test_gram_dual_is_ignored_on_the_sparse_path(h):
    inst = W.sparse_large(1002, m=6000, n=1200)
    a = solve_csc(h, inst.A, inst.b)
    b = solve_csc(h, inst.A, inst.b, flags=N.NNLS_FLAG_GRAM_DUAL)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3]) and a[4] == b[4]


def test_kept_tiles_when_the_free_set_grows(h):
    """|F| grows from 439 to 515 in the second iteration (7 -> 9 tile rows): on a fresh
    handle the factor buffers are reallocated there, which must end the reuse for that
    iteration only.  Oracle parity, and the same result as refactoring every iteration."""
    rng = np.random.default_rng(3)
    n = int(rng.choice([150, 300, 600]))
    m = n + int(rng.integers(5, n))
    A = rng.standard_normal((m, n))
    xs = np.where(rng.random(n) < 0.7, rng.uniform(0.1, 1, n), 0.0)
    b = A @ xs + 0.5 * rng.standard_normal(m)
    assert (m, n) == (655, 600)
    res = bpp_solve(A, b)
    with N.Handle(0) as fresh:
        st, info, x, y, trace = solve_dense(fresh, A, b)
        tr = N.nnls_get_trace(fresh, reused=True)
    assert [r[4] for r in tr][:2] == [439, 515] and tr[1][5] == 0
    check_parity(res, st, info, x, y, trace, rtol=1e-9)
    st2, info2, x2, y2, trace2 = solve_dense(h, A, b, flags=N.NNLS_FLAG_NO_FACTOR_REUSE)
    assert trace2 == trace and np.array_equal(x > 0, x2 > 0)
    assert relerr(x, x2) <= 1e-11


def test_empty_free_set(h):
    A = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    b = np.array([-1.0, -2.0, 0.5])
    st, info, x, y, trace = solve_dense(h, A, b)
    assert st == N.NNLS_OK and info.iterations == 0 and trace == []
    assert np.array_equal(x, [0.0, 0.0]) and np.allclose(y, -(A.T @ b))


def test_breakdown_reports_column(h):
    A = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    b = np.array([1.0, 1.0, 0.0, 0.0])
    st, info, *_ = solve_dense(h, A, b)
    assert st == N.NNLS_ERR_NOT_PD and info.failed_index == 1
    res = bpp_solve(A, b)
    assert res.status == "not_pd" and res.failed_index == info.failed_index
    import scipy.sparse as sp
    st, info, *_ = solve_csc(h, sp.csc_matrix(A), b)
    assert st == N.NNLS_ERR_NOT_PD and info.failed_index == 1


def test_iteration_cap(h):
    A, b = W.tiny_dense(1)
    st, info, *_ = solve_dense(h, A, b, max_iter=2)
    res = bpp_solve(A, b, max_iter=2)
    assert st == N.NNLS_ERR_MAXITER and res.status == "maxiter"
    assert info.iterations == 2 and info.last_ninf == res.last_ninf


def test_backup_rule_only(h):
    """p_max = 0: every non-improving step is a single exchange."""
    for seed in (1, 3, 5):
        A, b = W.tiny_dense(seed)
        res = bpp_solve(A, b, p_max=0)
        st, info, x, y, trace = solve_dense(h, A, b, p_max=0)
        assert st == N.NNLS_OK
        assert np.array_equal(x != 0, res.x != 0)


def test_invalid_inputs(h):
    import scipy.sparse as sp
    from _gpu_util import DEV, t
    inst = W.sparse_small(3, m=50, n=20, density=0.2)
    A = inst.A
    m, n = A.shape
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)

    def run(colptr, rowidx, val, b, mm=m, nn=n):
        st, _ = N.nnls_solve_csc(h, mm, nn, t(colptr, np.int32), t(rowidx, np.int32), t(val), t(b), x, y)
        return st

    cp, ri, va = A.indptr.copy(), A.indices.copy(), A.data.copy()
    assert run(cp, ri, va, inst.b) == N.NNLS_OK
    bad = cp.copy(); bad[3], bad[4] = bad[4], bad[3]
    assert run(bad, ri, va, inst.b) == N.NNLS_ERR_INVALID_ARG          # colptr not monotone
    bad = ri.copy(); bad[5] = m
    assert run(cp, bad, va, inst.b) == N.NNLS_ERR_INVALID_ARG          # row out of range
    bad = ri.copy(); s = cp[2]; bad[s], bad[s + 1] = bad[s + 1], bad[s]
    assert run(cp, bad, va, inst.b) == N.NNLS_ERR_INVALID_ARG          # rows not ascending
    bad = va.copy(); bad[7] = np.nan
    assert run(cp, ri, bad, inst.b) == N.NNLS_ERR_INVALID_VALUE
    bb = inst.b.copy(); bb[0] = np.inf
    assert run(cp, ri, va, bb) == N.NNLS_ERR_INVALID_VALUE
    assert run(cp[: n + 1], ri, va, inst.b[: n - 1], mm=n - 1) == N.NNLS_ERR_INVALID_ARG  # m < n


# ------------------------------------------------------------------ mixed precision
MIXED_RTOL = 1e-8


def check_mixed(res, st, info, x, y, trace, scale=1.0):
    assert st == N.NNLS_OK, N.status_string(st)
    assert np.array_equal(np.flatnonzero(x != 0), np.flatnonzero(res.x != 0))
    assert info.n_free == int(res.free.sum())
    assert relerr(x, res.x) <= MIXED_RTOL
    assert np.linalg.norm(y - res.y) <= MIXED_RTOL * max(np.linalg.norm(res.y), 1.0)
    assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0
    if certified(res, scale, rel=1e-6):
        assert trace == oracle_trace(res)


@pytest.mark.parametrize("seed", [1001, 1002, 1003])
def test_mixed_sparse_small(h, seed):
    inst = W.sparse_small(seed)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_FP32_IR)
    check_mixed(res, st, info, x, y, trace)
    assert info.ir_steps >= info.iterations   # every factor was refined at least once


def test_mixed_stays_in_float32_when_well_conditioned(h):
    """On a well-conditioned problem every iteration keeps its float32 factor (one factor
    launch per iteration, no float64 redo) and refinement stops within three steps per
    iteration; the result still matches the oracle to the mixed-precision tolerance."""
    inst = W.sparse_large(1002, m=6000, n=1200)
    res = bpp_solve(inst.A, inst.b)
    N.nnls_reset_profile(h)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_FP32_IR, flags=N.NNLS_FLAG_PROFILE)
    check_mixed(res, st, info, x, y, trace)
    prof = N.nnls_get_profile(h)
    assert prof["cholesky"]["launches"] == info.iterations
    assert info.iterations <= info.ir_steps <= 3 * info.iterations


@pytest.mark.parametrize("m,n,seed", [(300, 100, 2), (1100, 520, 4)])
def test_mixed_dense_planted(h, m, n, seed):
    inst = W.dense_planted(seed, m, n)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b, precision=N.NNLS_FP32_IR)
    check_mixed(res, st, info, x, y, trace)


def test_mixed_sparse_large_full_size(h):
    inst = W.sparse_large(1002)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_FP32_IR)
    assert st == N.NNLS_OK
    assert np.array_equal(x > 0, inst.active)
    res = bpp_solve(inst.A, inst.b)
    check_mixed(res, st, info, x, y, trace)


@pytest.fixture(scope="module")
def blockband():
    return W.sparse_blockband(1005)


@pytest.mark.parametrize("precision,tol", [(N.NNLS_FP64, 1e-10), (N.NNLS_FP32_IR, 1e-8), (N.NNLS_BF16_IR, 1e-8)])
def test_large_blockband_full_size(h, blockband, precision, tol):
    """The large sparse instance (m = 400000, n = 50000, block band, 25% active) at full
    size: the free set is the planted one and x is the planted x* (an exact NNLS solution
    by construction, to the z-solve's accuracy) within the path's tolerance."""
    inst = blockband
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=precision)
    assert st == N.NNLS_OK, N.status_string(st)
    assert np.array_equal(x > 0, inst.active)
    assert info.n_free == int(inst.active.sum())
    assert relerr(x, inst.x_star) <= tol
    assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0


@pytest.mark.parametrize("seed", range(1, 21))
def test_mixed_ill_scaled_falls_back(h, seed):
    """Ill-scaled problems where a float32 factor may break down or refinement may stall:
    the iteration is redone in float64 and the result matches the float64 path."""
    A, b = W.tiny_dense(seed)
    st64, info64, x64, y64, tr64 = solve_dense(h, A, b)
    st, info, x, y, tr = solve_dense(h, A, b, precision=N.NNLS_FP32_IR)
    assert st == st64 == N.NNLS_OK
    assert np.array_equal(x != 0, x64 != 0)
    assert relerr(x, x64) <= 1e-6


def _ls_reference(A, b, free, steps=3):
    """x on F of the least-squares problem on the columns A_F: float64 normal equations,
    then refinement whose residual A_F^T (A_F x - b) is formed exactly in rational
    arithmetic (every float is a dyadic rational), so the result is the float64 vector
    nearest the exact solution up to the last correction's rounding."""
    from fractions import Fraction
    AF = np.asarray(A)[:, free]
    cf = sla.cho_factor(AF.T @ AF, lower=True)
    x = sla.cho_solve(cf, AF.T @ b)
    Af = [[Fraction(v) for v in row] for row in AF.tolist()]
    bf = [Fraction(v) for v in np.asarray(b).tolist()]
    m, k = AF.shape
    for _ in range(steps):
        xf = [Fraction(v) for v in x.tolist()]
        r = [sum((a * xv for a, xv in zip(row, xf)), Fraction(0)) - bi for row, bi in zip(Af, bf)]
        g = np.array([float(sum((Af[i][j] * r[i] for i in range(m)), Fraction(0))) for j in range(k)])
        x = x - sla.cho_solve(cf, g)
    return x


@pytest.mark.parametrize("seed", [1, 2])
def test_mixed_certifies_intermediate_signs(h, seed):
    """The planted F-block has condition 1e6, so refinement with the float32 factor gains
    only two to three digits per step.  Intermediate splits stop refining once every tested
    sign is certified (fewer steps than refining each to ir_rtol), the feasible split is
    refined to ir_rtol; free sets and trajectory match the oracle, and x matches a reference
    computed with exact residuals far beyond the float64 normal equations (kappa^2 u ~ 1e-10
    here), within the error bound the solve reports."""
    inst = W.conditioned_planted(seed, 600, 300, 1e3)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b, precision=N.NNLS_FP32_IR)
    steps = [r[5] for r in N.nnls_get_trace(h, ir_steps=True)]
    print(f"seed {seed}: iterations {info.iterations}, refinement steps per iteration {steps}, "
          f"est_rel_err {info.est_rel_err:.2e}", flush=True)
    assert st == N.NNLS_OK and res.status == "ok"
    assert np.array_equal(x > 0, inst.active) and np.array_equal(res.free, inst.active)
    if certified(res, 1.0, rel=1e-6):
        assert trace == oracle_trace(res)
    assert sum(steps) == info.ir_steps and len(steps) == info.iterations >= 3
    # every split refined to ir_rtol: the same trajectory and free set, more steps
    st_a, info_a, x_a, y_a, trace_a = solve_dense(h, inst.A, inst.b, precision=N.NNLS_FP32_IR,
                                                  flags=N.NNLS_FLAG_REFINE_ALL)
    steps_a = [r[5] for r in N.nnls_get_trace(h, ir_steps=True)]
    print(f"  refined to ir_rtol at every split: {steps_a}", flush=True)
    assert st_a == N.NNLS_OK and trace_a == trace and np.array_equal(x_a > 0, x > 0)
    assert sum(steps[:-1]) < sum(steps_a[:-1])
    assert info.ir_steps < info_a.ir_steps
    xr = _ls_reference(inst.A, inst.b, inst.active)
    xf = x[inst.active]
    actual = np.max(np.abs(xf - xr)) / np.max(np.abs(xf))
    assert 0 < info.est_rel_err <= N.default_options().ir_rtol
    assert actual <= info.est_rel_err + 4e-16
    assert actual <= 1e-12
    assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0


def test_mixed_error_bound_sparse(h):
    """The mixed path states a bound on the error of every result: on a sparse problem
    the bound is at most ir_rtol and covers the distance to the oracle's x (whose own
    error is far below it)."""
    inst = W.sparse_small(1002)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_FP32_IR)
    check_mixed(res, st, info, x, y, trace)
    f = res.free
    actual = np.max(np.abs(x[f] - res.x[f])) / np.max(np.abs(x[f]))
    assert 0 < info.est_rel_err <= 1e-12
    assert actual <= info.est_rel_err + 1e-14   # the oracle's own error is below 1e-14 here


# ------------------------------------------------------------------ bfloat16 updates
@pytest.mark.parametrize("seed", [1001, 1002, 1003])
def test_bf16_sparse_small(h, seed):
    inst = W.sparse_small(seed)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_BF16_IR)
    check_mixed(res, st, info, x, y, trace)
    assert 0 < info.est_rel_err <= 1e-12


def test_bf16_sparse_large_full_size(h):
    inst = W.sparse_large(1002)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, precision=N.NNLS_BF16_IR)
    assert np.array_equal(x > 0, inst.active)
    check_mixed(res, st, info, x, y, trace)


@pytest.mark.parametrize("m,n,seed", [(300, 100, 2), (1100, 520, 4)])
def test_bf16_dense_planted(h, m, n, seed):
    inst = W.dense_planted(seed, m, n)
    res = bpp_solve(inst.A, inst.b)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b, precision=N.NNLS_BF16_IR)
    check_mixed(res, st, info, x, y, trace)


def test_bf16_ill_conditioned_climbs_the_ladder(h):
    """kappa(H_FF) = 1e6 is far beyond what bfloat16 updates can refine (kappa 2^-8 >> 1):
    those factors are redone in float32 (then float64 if needed) and the result is still
    the planted free set with x within the reported bound of an exact-residual reference."""
    inst = W.conditioned_planted(1, 600, 300, 1e3)
    st, info, x, y, trace = solve_dense(h, inst.A, inst.b, precision=N.NNLS_BF16_IR)
    assert st == N.NNLS_OK
    assert np.array_equal(x > 0, inst.active)
    xr = _ls_reference(inst.A, inst.b, inst.active)
    xf = x[inst.active]
    actual = np.max(np.abs(xf - xr)) / np.max(np.abs(xf))
    assert 0 < info.est_rel_err <= 1e-12 and actual <= info.est_rel_err + 4e-16


def test_bf16_on_the_batched_path_is_its_float32_tier(h):
    """The batched path has no bfloat16 tier: a NNLS_BF16_IR request runs its float32 tier,
    bit for bit the NNLS_FP32_IR result."""
    A = np.random.default_rng(0).standard_normal((40, 20))
    b = np.ones(40)
    out = {}
    for prec in (N.NNLS_FP32_IR, N.NNLS_BF16_IR):
        x = torch.empty(20, dtype=torch.float64, device=DEV)
        y = torch.empty_like(x)
        st, _ = N.nnls_solve_dense_batched(h, [colmajor_dev(A)], [t(b)], [x], [y],
                                           N.default_options(precision=prec))
        assert st == N.NNLS_OK
        out[prec] = (x.cpu().numpy(), y.cpu().numpy())
    assert np.array_equal(out[N.NNLS_FP32_IR][0], out[N.NNLS_BF16_IR][0])
    assert np.array_equal(out[N.NNLS_FP32_IR][1], out[N.NNLS_BF16_IR][1])
