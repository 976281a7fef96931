"""Batched dense path (one launch, one workgroup per problem) against the oracle: identical
free sets, x within 1e-10 (float64 factor) or 1e-8 (float32 factor + float64 refinement),
and bitwise identical results alone and inside any batch."""
import numpy as np
import pytest

import workloads as W
from oracle import bpp_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402
from _gpu_util import DEV, colmajor_dev, t  # noqa: E402


@pytest.fixture(scope="module")
def h():
    with N.Handle(0) as hh:
        yield hh


def run_batch(h, problems, **opt):
    As = [colmajor_dev(A) for A, _ in problems]
    bs = [t(b) for _, b in problems]
    xs = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    ys = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    st, infos = N.nnls_solve_dense_batched(h, As, bs, xs, ys, N.default_options(**opt))
    return st, infos, [x.cpu().numpy() for x in xs], [y.cpu().numpy() for y in ys]


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


@pytest.fixture(scope="module")
def batch24():
    insts = W.dense_batch(1003, count=24)
    return [(i.A, i.b) for i in insts], insts


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
def test_batch_matches_oracle(h, batch24, precision, tol):
    problems, insts = batch24
    st, infos, xs, ys = run_batch(h, problems, precision=precision)
    assert st == N.NNLS_OK
    for inst, info, x, y in zip(insts, infos, xs, ys):
        res = bpp_solve(inst.A, inst.b)
        assert info.status == N.NNLS_OK and res.status == "ok"
        assert info.iterations == res.iterations
        assert info.n_free == int(res.free.sum())
        assert np.array_equal(x > 0, inst.active)
        assert relerr(x, res.x) <= tol
        assert np.linalg.norm(y - res.y) <= tol * max(np.linalg.norm(res.y), 1.0)
        assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0
        if precision == 1:
            assert info.ir_steps >= 1


@pytest.mark.parametrize("precision", [0, 1])
def test_alone_equals_in_batch(h, batch24, precision):
    problems, _ = batch24
    st, infos, xs, ys = run_batch(h, problems, precision=precision)
    for k in (0, 7, 23):
        st1, inf1, x1, y1 = run_batch(h, [problems[k]], precision=precision)
        assert np.array_equal(x1[0], xs[k]) and np.array_equal(y1[0], ys[k])
        assert inf1[0].iterations == infos[k].iterations
    # reversed order, and a batch mixed with other problems
    st2, inf2, x2, y2 = run_batch(h, problems[::-1], precision=precision)
    for k in range(len(problems)):
        assert np.array_equal(x2[len(problems) - 1 - k], xs[k])


def test_multi_tile_and_ragged_sizes(h):
    sizes = [(40, 16, 1), (300, 100, 2), (700, 256, 3), (1100, 520, 4), (200, 65, 5), (130, 64, 6)]
    insts = [W.dense_planted(s, m, n) for m, n, s in sizes]
    st, infos, xs, ys = run_batch(h, [(i.A, i.b) for i in insts])
    assert st == N.NNLS_OK
    for inst, info, x in zip(insts, infos, xs):
        res = bpp_solve(inst.A, inst.b)
        assert np.array_equal(x > 0, inst.active)
        assert relerr(x, res.x) <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_all_branches_in_batch(h, precision):
    problems = [W.tiny_dense(s) for s in range(1, 21)]
    st, infos, xs, ys = run_batch(h, problems, precision=precision)
    assert st == N.NNLS_OK
    for (A, b), info, x in zip(problems, infos, xs):
        res = bpp_solve(A, b)
        assert np.array_equal(x != 0, res.x != 0)
        Hff = (A.T @ A)[np.ix_(res.free, res.free)]
        kappa = np.linalg.cond(Hff) if res.free.any() else 1.0
        assert relerr(x, res.x) <= max(1e-9, 100 * kappa * np.finfo(float).eps)


def test_failures_stay_in_their_problem(h):
    good = W.dense_planted(11, 120, 50)
    bad_nan = good.A.copy()
    bad_nan[3, 4] = np.nan
    dup = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    problems = [(good.A, good.b), (bad_nan, good.b), (dup, np.array([1.0, 1.0, 0.0, 0.0])),
                (good.A, good.b)]
    st, infos, xs, ys = run_batch(h, problems)
    assert st == N.NNLS_ERR_INVALID_VALUE
    assert [i.status for i in infos] == [N.NNLS_OK, N.NNLS_ERR_INVALID_VALUE, N.NNLS_ERR_NOT_PD, N.NNLS_OK]
    assert infos[2].failed_index == 1
    assert np.array_equal(xs[0], xs[3])
    res = bpp_solve(good.A, good.b)
    assert relerr(xs[0], res.x) <= 1e-10


@pytest.mark.parametrize("precision", [0, 1])
def test_gram_column_groups_and_edges(h, precision):
    """Sizes on both sides of each 32-column group of the streamed Gram matrix, m not a
    multiple of its 16-row steps, and n past its limit (the in-kernel tiled Gram)."""
    ns = [1, 2, 31, 32, 33, 63, 64, 65, 96, 97, 128, 129, 160, 193, 224, 225, 255, 256, 257, 300]
    insts = [W.dense_planted(500 + k, max(n + 1, 2 * n + 7 * k % 13), n) for k, n in enumerate(ns)]
    st, infos, xs, ys = run_batch(h, [(i.A, i.b) for i in insts], precision=precision)
    assert st == N.NNLS_OK
    for inst, info, x in zip(insts, infos, xs):
        res = bpp_solve(inst.A, inst.b)
        assert info.iterations == res.iterations
        assert np.array_equal(x > 0, res.x > 0)
        assert relerr(x, res.x) <= 1e-10, (inst.m, inst.n)


@pytest.mark.parametrize("n", [40, 300])
def test_non_finite_entries_rejected(h, n):
    """A NaN or an infinity anywhere in A (first and last row and column) or b is reported
    for its own problem only, on both sides of the streamed Gram matrix's size limit."""
    good = W.dense_planted(21, 2 * n + 5, n)
    m = good.A.shape[0]
    cases = []
    for (i, j, v) in [(0, 0, np.nan), (m - 1, n - 1, np.inf), (m - 1, 0, -np.inf), (0, n - 1, np.nan)]:
        A = good.A.copy()
        A[i, j] = v
        cases.append((A, good.b))
    for i in (0, m - 1):
        b = good.b.copy()
        b[i] = np.nan
        cases.append((good.A, b))
    problems = [(good.A, good.b)] + cases + [(good.A, good.b)]
    for precision in (0, 1):
        st, infos, xs, ys = run_batch(h, problems, precision=precision)
        assert st == N.NNLS_ERR_INVALID_VALUE
        assert [i.status for i in infos] == [N.NNLS_OK] + [N.NNLS_ERR_INVALID_VALUE] * len(cases) + [N.NNLS_OK]
        assert all(i.failed_index == -1 and i.iterations == 0 for i in infos[1:-1])
        assert np.array_equal(xs[0], xs[-1])


def test_empty_and_invalid(h):
    st, infos, xs, ys = run_batch(h, [])
    assert st == N.NNLS_OK and infos == []
    A = np.ones((3, 5))
    st, infos, xs, ys = run_batch(h, [(A, np.ones(3))])   # m < n
    assert st == N.NNLS_ERR_INVALID_ARG


def test_packed_descriptors_reused(h, batch24):
    problems, insts = batch24
    As = [colmajor_dev(A) for A, _ in problems]
    bs = [t(b) for _, b in problems]
    xs = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    ys = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    packed = N.BatchedArgs(As, bs, xs, ys)
    st1, _ = N.nnls_solve_dense_batched(h, packed=packed)
    first = [x.cpu().numpy().copy() for x in xs]
    for x in xs:
        x.fill_(np.nan)
    st2, infos = N.nnls_solve_dense_batched(h, packed=packed)
    assert st1 == st2 == N.NNLS_OK
    for a, x, inst in zip(first, xs, insts):
        assert np.array_equal(a, x.cpu().numpy())
        assert np.array_equal(a > 0, inst.active)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
def test_gram_dual_matches_oracle(h, batch24, precision, tol):
    """NNLS_FLAG_GRAM_DUAL (y_G = H_GF x_F - c_G, Eq. 3, from the workspace Gram matrix): the
    oracle's free sets and x, and y within the same tolerance; the same pivot steps as the
    residual form (Eq. 5)."""
    problems, insts = batch24
    st, infos, xs, ys = run_batch(h, problems, precision=precision, flags=N.NNLS_FLAG_GRAM_DUAL)
    st0, infos0, xs0, ys0 = run_batch(h, problems, precision=precision)
    assert st == st0 == N.NNLS_OK
    for inst, info, info0, x, y, x0 in zip(insts, infos, infos0, xs, ys, xs0):
        res = bpp_solve(inst.A, inst.b)
        assert info.status == N.NNLS_OK and info.iterations == info0.iterations
        assert np.array_equal(x > 0, res.x > 0) and np.array_equal(x > 0, x0 > 0)
        assert relerr(x, res.x) <= tol
        assert np.linalg.norm(y - res.y) <= tol * max(np.linalg.norm(res.y), 1.0)
        assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0


@pytest.mark.parametrize("precision", [0, 1])
def test_plan_replays_match_eager(h, batch24, precision):
    """A prepared batch replayed from its captured graph: each replay, with the program's own
    work on the stream and host synchronisations between replays and new values in b, gives
    bitwise the result of nnls_solve_dense_batched on the same inputs."""
    problems, insts = batch24
    opts = N.default_options(precision=precision)
    As = [colmajor_dev(A) for A, _ in problems]
    bs = [t(b) for _, b in problems]
    nan = lambda k: torch.full((k,), np.nan, dtype=torch.float64, device=DEV)
    xs = [nan(A.shape[1]) for A, _ in problems]
    ys = [nan(A.shape[1]) for A, _ in problems]
    xe = [nan(A.shape[1]) for A, _ in problems]
    ye = [nan(A.shape[1]) for A, _ in problems]
    plan = N.BatchPlan(h, As, bs, xs, ys, opts)
    shapes = plan.tile_shapes()   # the autotuner's choice per 32-column bucket
    assert set(shapes) == {(A.shape[1] + 31) // 32 for A, _ in problems}
    assert all(v in ((2, 3, 4) if precision == 0 else (4, 6, 8)) for v in shapes.values())
    for k, scale in enumerate([1.0, 0.5, 2.0, 1.0, -1.0]):
        for b, (_, b0) in zip(bs, problems):          # eager work between the replays
            b.copy_(torch.from_numpy(b0 * scale).to(DEV))
        for x in xs:
            x.fill_(np.nan)
        if k % 2:
            assert plan.execute(wait=False) == N.NNLS_OK
            st, infos = plan.info()
        else:
            st, infos = plan.execute()
        ste, infe = N.nnls_solve_dense_batched(h, As, bs, xe, ye, opts)
        torch.cuda.synchronize()
        assert st == ste == N.NNLS_OK
        for i in range(len(problems)):
            assert torch.equal(xs[i], xe[i]) and torch.equal(ys[i], ye[i]), (k, i)
            assert infos[i].iterations == infe[i].iterations and infos[i].ir_steps == infe[i].ir_steps
        if scale == 1.0:
            for x, inst in zip(xs, insts):
                assert np.array_equal(x.cpu().numpy() > 0, inst.active)
    plan.close()


def test_plan_rejects_bad_batches(h):
    with pytest.raises(RuntimeError):
        N.BatchPlan(h, [], [], [], [])
    A = torch.zeros((3, 5), dtype=torch.float64, device=DEV).t().contiguous().t()   # m < n
    with pytest.raises(RuntimeError):
        N.BatchPlan(h, [A], [torch.zeros(3, dtype=torch.float64, device=DEV)],
                    [torch.zeros(5, dtype=torch.float64, device=DEV)], [torch.zeros(5, dtype=torch.float64, device=DEV)])


def test_bf16_request_runs_the_float32_tier(h, batch24):
    """NNLS_BF16_IR on the batched path runs its float32 tier: the same statuses, iteration
    counts and bitwise the same x and y as NNLS_FP32_IR."""
    problems, insts = batch24
    st32, inf32, x32, y32 = run_batch(h, problems, precision=N.NNLS_FP32_IR)
    st16, inf16, x16, y16 = run_batch(h, problems, precision=N.NNLS_BF16_IR)
    assert st32 == st16 == N.NNLS_OK
    for a, b, xa, xb, ya, yb in zip(inf32, inf16, x32, x16, y32, y16):
        assert a.status == b.status and a.iterations == b.iterations and a.ir_steps == b.ir_steps
        assert np.array_equal(xa, xb) and np.array_equal(ya, yb)
