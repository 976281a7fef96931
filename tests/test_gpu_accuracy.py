"""Accuracy against condition number on the GPU, the analog of the paper's Fig. 1: on
80 x 70 matrices with prescribed condition number and a known all-positive solution, the
normal-equations solution's relative error follows the law fitted to the paper's printed
points (kappa^2 eps, Sec. 2.1 and Sec. 4) on both precisions, and stays within a decade of
the CPU oracle's error on the same problems."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import bpp_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402
from _gpu_util import DEV, colmajor_dev, t  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig1_law():
    d = np.loadtxt(os.path.join(GOLDEN, "fig1_normal_equations_error.txt"))
    lk = 1 + (d[:, 0] - 120) * 7 / 1319
    le = -16 + (d[:, 1] - 82) * 18 / 778
    return np.polyfit(lk, le, 1)


@pytest.fixture(scope="module")
def h():
    with N.Handle(0) as hh:
        yield hh


def batched_errors(h, probs, precision):
    As = [colmajor_dev(A) for A, _, _ in probs]
    bs = [t(b) for _, _, b in probs]
    xs = [torch.empty(A.shape[1], dtype=torch.float64, device=DEV) for A, _, _ in probs]
    ys = [torch.empty(A.shape[1], dtype=torch.float64, device=DEV) for A, _, _ in probs]
    st, infos = N.nnls_solve_dense_batched(h, As, bs, xs, ys, N.default_options(precision=precision))
    assert st == N.NNLS_OK
    return [np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt) for x, (_, xt, _) in zip(xs, probs)]


def oracle_median(probs):
    orc = []
    for A, xt, b in probs:
        r = bpp_solve(A, b)
        orc.append(np.linalg.norm(r.x - xt) / np.linalg.norm(xt))
    return np.median(np.log10(orc))


def test_float64_error_follows_fig1_law(h):
    slope, icpt = fig1_law()
    for lkap in (1.5, 2.5, 3.5, 4.5, 5.5, 6.0):
        probs = [W.svd_conditioned(100 + s, 10 ** lkap) for s in range(5)]
        gpu = np.median(np.log10(batched_errors(h, probs, N.NNLS_FP64)))
        assert abs(gpu - (slope * lkap + icpt)) < 0.75, (lkap, gpu)
        assert abs(gpu - oracle_median(probs)) < 1.0, (lkap, gpu)


def test_mixed_error_no_worse_than_normal_equations(h):
    """The float32 factor refined against the float64 residual from A is never less accurate
    than the float64 normal equations (the law's band), and usually more accurate: the
    refinement's residual does not square the condition number."""
    slope, icpt = fig1_law()
    for lkap in (1.5, 2.5, 3.5, 4.5, 5.5, 6.0):
        probs = [W.svd_conditioned(100 + s, 10 ** lkap) for s in range(5)]
        gpu = np.median(np.log10(batched_errors(h, probs, N.NNLS_FP32_IR)))
        assert gpu < slope * lkap + icpt + 0.75, (lkap, gpu)
        assert gpu < oracle_median(probs) + 1.0, (lkap, gpu)


def test_mixed_single_problem_path_refines_after_fallback(h):
    """Above kappa ~ 1e3.5 the float32 factor no longer contracts and the iteration is
    redone with a float64 factor, which is then refined as well: the mixed single-problem
    path keeps the accuracy of the refined float64 solution."""
    for lkap in (4.0, 5.0, 6.0):
        errs = []
        for s in range(3):
            A, xt, b = W.svd_conditioned(500 + s, 10 ** lkap)
            x = torch.empty(A.shape[1], dtype=torch.float64, device=DEV)
            y = torch.empty_like(x)
            st, info = N.nnls_solve_dense(h, colmajor_dev(A), t(b), x, y,
                                          N.default_options(precision=N.NNLS_FP32_IR))
            assert st == N.NNLS_OK
            errs.append(np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt))
        slope, icpt = fig1_law()
        assert np.median(np.log10(errs)) <= slope * lkap + icpt - 2.0, lkap


def test_single_problem_path_matches_batched_accuracy(h):
    """The dense single-problem path (tiled factor, walker) gives errors of the same size."""
    slope, icpt = fig1_law()
    for lkap in (2.0, 4.0, 6.0):
        errs = []
        for s in range(3):
            A, xt, b = W.svd_conditioned(200 + s, 10 ** lkap)
            x = torch.empty(A.shape[1], dtype=torch.float64, device=DEV)
            y = torch.empty_like(x)
            st, info = N.nnls_solve_dense(h, colmajor_dev(A), t(b), x, y)
            assert st == N.NNLS_OK
            errs.append(np.linalg.norm(x.cpu().numpy() - xt) / np.linalg.norm(xt))
        assert abs(np.median(np.log10(errs)) - (slope * lkap + icpt)) < 0.75, lkap


def test_final_refinement_gains_orders_of_magnitude(h):
    """NNLS_FLAG_REFINE_FINAL (the final recomputation of Sec. 3): float64 refinement of the
    final x_F against the residual from A gains at least two orders of magnitude over the
    normal equations where the paper's final step does (kappa 1e3 .. 1e6), and never loses."""
    slope, icpt = fig1_law()
    for lkap in (1.5, 3.0, 4.0, 5.0, 6.0):
        plain, refd = [], []
        for s in range(3):
            A, xt, b = W.svd_conditioned(400 + s, 10 ** lkap)
            for flags, out in ((0, plain), (N.NNLS_FLAG_REFINE_FINAL, refd)):
                x = torch.empty(A.shape[1], dtype=torch.float64, device=DEV)
                y = torch.empty_like(x)
                st, info = N.nnls_solve_dense(h, colmajor_dev(A), t(b), x, y, N.default_options(flags=flags))
                assert st == N.NNLS_OK
                xh, yh = x.cpu().numpy(), y.cpu().numpy()
                assert np.all(xh >= 0) and np.all(yh >= 0) and np.dot(xh, yh) == 0.0
                out.append(np.linalg.norm(xh - xt) / np.linalg.norm(xt))
        gp, gr = np.median(np.log10(plain)), np.median(np.log10(refd))
        assert gr <= gp + 0.1, (lkap, gp, gr)
        if lkap >= 3.0:
            assert gr <= gp - 2.0, (lkap, gp, gr)


def test_final_refinement_keeps_parity_on_sparse_workload(h):
    inst = W.sparse_large(1002, m=6000, n=1200)
    res = bpp_solve(inst.A, inst.b)
    from _gpu_util import solve_csc
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, flags=N.NNLS_FLAG_REFINE_FINAL)
    assert st == N.NNLS_OK
    assert np.array_equal(x > 0, inst.active) and np.array_equal(x > 0, res.x > 0)
    assert np.linalg.norm(x - res.x) <= 1e-10 * np.linalg.norm(res.x)
    assert np.linalg.norm(x - inst.x_star) <= np.linalg.norm(res.x - inst.x_star) + 1e-14 * np.linalg.norm(inst.x_star)
    assert info.ir_steps >= 1


def _solve_dense_flags(h, A, b, flags):
    x = torch.empty(A.shape[1], dtype=torch.float64, device=DEV)
    y = torch.empty_like(x)
    st, info = N.nnls_solve_dense(h, colmajor_dev(A), t(b), x, y, N.default_options(flags=flags))
    assert st == N.NNLS_OK
    return x.cpu().numpy(), y.cpu().numpy(), info


def test_condition_estimate_matches_oracle_and_brackets_exact(h):
    """NNLS_FLAG_REFINE_AUTO forms 0.1 kappa_1(A_F^T A_F) eps from the split's factor (Sec. 3's
    dpocon test): the same estimate as the oracle's on the same F-block, at most the exact
    value and at least a third of it."""
    from oracle import gram, predicted_rel_error, principal_block
    eps = np.finfo(np.float64).eps
    for lkap in (1.5, 2.5, 3.5, 4.5):
        for s in range(3):
            A, xt, b = W.svd_conditioned(500 + s, 10 ** lkap)
            x, y, info = _solve_dense_flags(h, A, b, N.NNLS_FLAG_REFINE_AUTO)
            H, _ = gram(A, b)
            Hff = principal_block(H, np.flatnonzero(x > 0))
            Hff = Hff.toarray() if hasattr(Hff, "toarray") else Hff
            exact = 0.1 * np.abs(Hff).sum(axis=0).max() * np.abs(np.linalg.inv(Hff)).sum(axis=0).max() * eps
            est = info.est_rel_err
            assert exact / 3 <= est <= exact * (1 + 1e-4), (lkap, s, est, exact)
            assert est == pytest.approx(predicted_rel_error(Hff), rel=1e-4), (lkap, s)


def test_auto_refinement_runs_only_when_the_estimate_misses_the_target(h):
    """Well conditioned: no refinement, the plain float64 result bit for bit.  kappa(A) = 1e4
    (predicted error ~1e-8 > ir_rtol): refined, the REFINE_FINAL result bit for bit."""
    A, xt, b = W.svd_conditioned(601, 10 ** 1.5)
    x0, _, _ = _solve_dense_flags(h, A, b, 0)
    xa, _, ia = _solve_dense_flags(h, A, b, N.NNLS_FLAG_REFINE_AUTO)
    assert 0 < ia.est_rel_err <= 1e-12 and ia.ir_steps == 0
    assert np.array_equal(x0, xa)
    A, xt, b = W.svd_conditioned(602, 1e4)
    xf, _, i_f = _solve_dense_flags(h, A, b, N.NNLS_FLAG_REFINE_FINAL)
    xa, ya, ia = _solve_dense_flags(h, A, b, N.NNLS_FLAG_REFINE_AUTO)
    assert ia.est_rel_err > 1e-12 and ia.ir_steps == i_f.ir_steps >= 1
    assert i_f.est_rel_err == -1.0
    assert np.array_equal(xf, xa)
    assert np.linalg.norm(xa - xt) / np.linalg.norm(xt) < 1e-11


def test_auto_refinement_on_the_sparse_workload(h):
    """Sparse source (whole Gram columns restricted to F): the estimate brackets the exact
    value; this well-conditioned workload needs no refinement."""
    from _gpu_util import solve_csc
    from oracle import gram, principal_block
    inst = W.sparse_large(1002, m=6000, n=1200)
    st, info, x, y, trace = solve_csc(h, inst.A, inst.b, flags=N.NNLS_FLAG_REFINE_AUTO)
    assert st == N.NNLS_OK and np.array_equal(x > 0, inst.active)
    H, _ = gram(inst.A, inst.b)
    Hff = principal_block(H, np.flatnonzero(x > 0))
    Hff = Hff.toarray() if hasattr(Hff, "toarray") else np.asarray(Hff)
    eps = np.finfo(np.float64).eps
    exact = 0.1 * np.abs(Hff).sum(axis=0).max() * np.abs(np.linalg.inv(Hff)).sum(axis=0).max() * eps
    assert exact / 3 <= info.est_rel_err <= exact * (1 + 1e-4)
    assert info.ir_steps == 0
