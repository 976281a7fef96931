"""Parity of each step of the pivot iteration, called through the C ABI on the GPU,
against the CPU oracle's step functions and textbook bounds."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import classify, dual, exchange_rule, gram

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402
from _gpu_util import DEV, colmajor_dev, csc_dev, t  # noqa: E402

EPS = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def h():
    with N.Handle(0) as hh:
        yield hh


@pytest.mark.parametrize("m,n,density,seed", [(300, 70, 0.1, 1), (2000, 400, 0.02, 2),
                                              (5000, 2500, 0.003, 3), (64, 64, 0.5, 4)])
def test_gram_and_rhs(h, m, n, density, seed):
    inst = W.sparse_small(seed, m=m, n=n, density=density)
    A = inst.A
    colptr, rowidx, val = csc_dev(A)
    H = colmajor_dev(np.full((n, n), np.nan))
    c = torch.empty(n, dtype=torch.float64, device=DEV)
    assert N.nnls_gram_csc(h, m, n, colptr, rowidx, val, t(inst.b), H, c) == N.NNLS_OK
    H_or, c_or = gram(A, inst.b)
    H_or = H_or.toarray()
    absA = abs(A)
    bound = (absA.T @ absA).toarray() * (m * EPS) + 1e-300
    Hg = H.cpu().numpy()
    assert np.all(np.abs(Hg - H_or) <= bound)
    assert np.array_equal(Hg, Hg.T)
    assert np.allclose(c.cpu().numpy(), c_or, rtol=1e-13, atol=1e-13 * np.abs(c_or).max())


@pytest.mark.parametrize("m,n,seed", [(1, 1, 1), (17, 3, 2), (70, 65, 3), (300, 129, 4), (1000, 257, 5),
                                      (64, 64, 6), (5003, 100, 7), (130, 130, 8)])
def test_gram_dense_mfma(h, m, n, seed):
    """Dense H = A^T A on MFMA (64 x 64 tiles of its lower half, ragged edges, 16-row steps)
    and c = A^T b, against the oracle's Gram step, within the float64 dot-product bound
    m eps (|A|^T |A|)_ij; H exactly symmetric."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    H = colmajor_dev(np.full((n, n), np.nan))
    c = torch.empty(n, dtype=torch.float64, device=DEV)
    assert N.nnls_gram_dense(h, colmajor_dev(A), t(b), H, c) == N.NNLS_OK
    H_or, c_or = gram(A, b)
    H_or = np.asarray(H_or.toarray() if hasattr(H_or, "toarray") else H_or)
    bound = (np.abs(A).T @ np.abs(A)) * (m * EPS) + 1e-300
    Hg = H.cpu().numpy()
    assert np.all(np.abs(Hg - H_or) <= bound)
    assert np.array_equal(Hg, Hg.T)
    cb = (np.abs(A).T @ np.abs(b)) * (m * EPS) + 1e-300
    assert np.all(np.abs(c.cpu().numpy() - c_or) <= cb)


def test_gram_windows_sweeps_and_long_rows(h):
    """The Gram kernel's rarer paths: more than one 32768-row window (n = 33000, with one
    row of A meeting columns on both sides of the window edge), columns of H with more than
    1024 rows (several accumulator sweeps), and rows of A longer than 16 entries.  Sampled
    columns of the dense H are compared with the oracle's sparse product, and with the
    matching rows for symmetry."""
    m, n = 300, 33000
    rng = np.random.default_rng(33000)
    rows = [rng.integers(0, m, size=2 * n)]
    cols = [np.repeat(np.arange(n), 2)]
    dense_cols = np.unique(np.concatenate([np.arange(0, 40), rng.choice(n, 2500, replace=False),
                                           np.arange(n - 40, n)]))
    rows.append(np.zeros(dense_cols.size, dtype=np.int64))            # one long row of A
    cols.append(dense_cols)
    mid = np.arange(32700, 32840)                                      # across the window edge
    rows.append(np.ones(mid.size, dtype=np.int64))
    cols.append(mid)
    A = sp.csc_matrix((rng.standard_normal(sum(r.size for r in rows)),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
    A.sum_duplicates()
    A.sort_indices()
    b = rng.standard_normal(m)
    colptr, rowidx, val = csc_dev(A)
    H = torch.full((n, n), float("nan"), dtype=torch.float64, device=DEV).t()
    c = torch.empty(n, dtype=torch.float64, device=DEV)
    assert N.nnls_gram_csc(h, m, n, colptr, rowidx, val, t(b), H, c) == N.NNLS_OK
    H_or, c_or = gram(A, b)
    H_or = sp.csc_matrix(H_or)
    absA = abs(A)
    bound_all = sp.csc_matrix(absA.T @ absA)
    sample = np.unique(np.concatenate([[0, 1, 39, 32700, 32767, 32768, 32839, n - 1],
                                       dense_cols[:: max(1, dense_cols.size // 12)]]))
    assert (H_or[:, [0]] != 0).sum() > 1024                            # several sweeps
    for j in sample:
        col = H[:, j].cpu().numpy()
        row = H[j, :].cpu().numpy()
        ref = H_or[:, [j]].toarray().ravel()
        bound = bound_all[:, [j]].toarray().ravel() * (m * EPS) + 1e-300
        assert np.all(np.abs(col - ref) <= bound), j
        assert np.array_equal(col, row), j
    assert np.allclose(c.cpu().numpy(), c_or, rtol=1e-13, atol=1e-13 * np.abs(c_or).max())
    del H
    torch.cuda.empty_cache()


def spd(n, seed, cond=100.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, 1.0 / cond, n)
    return (Q * ev) @ Q.T


@pytest.mark.parametrize("n", [1, 2, 15, 17, 63, 64, 65, 127, 128, 129, 200, 255, 300, 700])
def test_cholesky_fp64(h, n):
    S = spd(n, n)
    Sd = colmajor_dev(S)
    L = colmajor_dev(np.full((n, n), np.nan))
    st, failed = N.nnls_cholesky(h, Sd, L, N.NNLS_FP64)
    assert st == N.NNLS_OK and failed == -1
    Lg = L.cpu().numpy()
    assert np.all(np.triu(Lg, 1) == 0)
    assert np.linalg.norm(Lg @ Lg.T - S) <= 4 * n * EPS * np.linalg.norm(S)
    assert np.allclose(Lg, np.linalg.cholesky(S), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 33, 64, 100, 257])
def test_cholesky_fp32(h, n):
    S = spd(n, 10 + n)
    Sd = colmajor_dev(S)
    L = colmajor_dev(np.zeros((n, n)))
    st, failed = N.nnls_cholesky(h, Sd, L, N.NNLS_FP32_IR)
    assert st == N.NNLS_OK
    Lg = L.cpu().numpy()
    e32 = np.finfo(np.float32).eps
    assert np.linalg.norm(Lg @ Lg.T - S) <= 4 * n * e32 * np.linalg.norm(S)


@pytest.mark.parametrize("n", [130, 257, 513, 700])
def test_cholesky_bf16_updates(h, n):
    """NNLS_BF16_IR: the left-looking updates take bfloat16 copies of the finished tiles
    (u = 2^-8) with float32 accumulation, so every entry of L L^T - S is within
    2u sqrt(S_ii S_jj) (each product of two rounded entries is within 2u, and the products
    of a row pair sum to at most sqrt(S_ii S_jj) in magnitude), well above what float32
    updates leave: the bfloat16 path is the one that ran.  (It runs from three tile
    columns on: the walker applies each diagonal tile's last term in float32.)"""
    S = spd(n, 20 + n)
    L = colmajor_dev(np.zeros((n, n)))
    st, failed = N.nnls_cholesky(h, colmajor_dev(S), L, N.NNLS_BF16_IR)
    assert st == N.NNLS_OK and failed == -1
    Lg = L.cpu().numpy()
    assert np.all(np.triu(Lg, 1) == 0)
    d = np.sqrt(np.diag(S))
    rel = np.abs(Lg @ Lg.T - S) / np.outer(d, d)
    u = 2.0 ** -8
    assert rel.max() <= 2 * u * 1.05
    assert rel.max() > 1e-5


@pytest.mark.parametrize("n,k", [(10, 3), (100, 70), (130, 128), (64, 0)])
def test_cholesky_breakdown_position(h, n, k):
    """A negative pivot at position k: the factor reports k, as LAPACK's info does."""
    rng = np.random.default_rng(k)
    S = np.eye(n) * 4.0 + 0.01 * rng.standard_normal((n, n))
    S = (S + S.T) / 2
    S[k, k] = -1.0
    st, failed = N.nnls_cholesky(h, colmajor_dev(S), colmajor_dev(np.zeros((n, n))), N.NNLS_FP64)
    assert st == N.NNLS_ERR_NOT_PD and failed == k


@pytest.mark.parametrize("n", [1, 5, 64, 65, 190, 513])
def test_spd_solve(h, n):
    S = spd(n, 100 + n, cond=1e3)
    rhs = np.random.default_rng(n).standard_normal(n)
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    st, failed = N.nnls_spd_solve(h, colmajor_dev(S), t(rhs), x)
    assert st == N.NNLS_OK
    xr = np.linalg.solve(S, rhs)
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e3 * 50 * n * EPS * np.linalg.norm(xr)


def test_spd_solve_after_failed_call(h):
    """A call that ends in an error leaves the triangular solves' hand-over slots to be
    emptied again before the next call; solves after it (same size, then a larger one that
    reallocates the slots) must be exact."""
    n = 300
    rng = np.random.default_rng(11)
    bad = spd(n, 7, cond=1e2)
    bad[10, 10] = -1.0
    x = torch.empty(n, dtype=torch.float64, device=DEV)
    st, failed = N.nnls_spd_solve(h, colmajor_dev(bad), t(rng.standard_normal(n)), x)
    assert st == N.NNLS_ERR_NOT_PD and failed == 10
    for nn in (n, 3 * n + 17, n):
        S = spd(nn, 8 + nn, cond=1e3)
        rhs = rng.standard_normal(nn)
        xx = torch.empty(nn, dtype=torch.float64, device=DEV)
        st, failed = N.nnls_spd_solve(h, colmajor_dev(S), t(rhs), xx)
        assert st == N.NNLS_OK and failed == -1
        xr = np.linalg.solve(S, rhs)
        assert np.linalg.norm(xx.cpu().numpy() - xr) <= 1e3 * 50 * nn * EPS * np.linalg.norm(xr)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dual_step(h, seed):
    inst = W.sparse_small(seed, m=1500, n=500, density=0.03)
    rng = np.random.default_rng(seed)
    free = rng.random(inst.n) < 0.4
    x = np.where(free, rng.standard_normal(inst.n), 0.0)
    colptr, rowidx, val = csc_dev(inst.A)
    yd = torch.full((inst.n,), np.nan, dtype=torch.float64, device=DEV)
    rd = torch.empty(inst.m, dtype=torch.float64, device=DEV)
    st = N.nnls_dual_csc(h, inst.m, inst.n, colptr, rowidx, val, t(inst.b), t(free, np.uint8),
                         t(x), rd, yd)
    assert st == N.NNLS_OK
    idx_f, idx_g = np.flatnonzero(free), np.flatnonzero(~free)
    y_or = np.zeros(inst.n)
    y_or[idx_g] = dual(inst.A, inst.b, idx_f, x[idx_f], idx_g)
    yg = yd.cpu().numpy()
    assert np.all(yg[free] == 0.0)
    absA = abs(inst.A)
    r = inst.A @ x - inst.b
    bound = (absA.T @ (absA @ np.abs(x) + np.abs(inst.b))) * 4 * inst.m * EPS
    assert np.all(np.abs(yg - y_or) <= bound + 1e-300)


@pytest.mark.parametrize("m,n,density", [(3000, 400, 0.0015), (3000, 400, 0.004), (3000, 400, 0.008),
                                           (3000, 400, 0.016), (3000, 400, 0.04), (900, 600, 0.08)])
def test_residual_every_lane_width(h, m, n, density):
    """The row-major residual uses 1..16 lanes per row by average row length; every width
    must give r = A x - b and y = A^T r within the rounding bound."""
    inst = W.sparse_small(7, m=m, n=n, density=density)
    rng = np.random.default_rng(3)
    free = np.zeros(inst.n, dtype=bool)
    x = rng.standard_normal(inst.n)
    colptr, rowidx, val = csc_dev(inst.A)
    yd = torch.full((inst.n,), np.nan, dtype=torch.float64, device=DEV)
    rd = torch.empty(inst.m, dtype=torch.float64, device=DEV)
    st = N.nnls_dual_csc(h, inst.m, inst.n, colptr, rowidx, val, t(inst.b), t(free, np.uint8), t(x), rd, yd)
    assert st == N.NNLS_OK
    absA = abs(inst.A)
    r_ref = inst.A @ x - inst.b
    rbound = (absA @ np.abs(x) + np.abs(inst.b)) * 4 * inst.n * EPS
    assert np.all(np.abs(rd.cpu().numpy() - r_ref) <= rbound + 1e-300)
    y_ref = inst.A.T @ r_ref
    ybound = (absA.T @ (absA @ np.abs(x) + np.abs(inst.b))) * 8 * inst.m * EPS
    assert np.all(np.abs(yd.cpu().numpy() - y_ref) <= ybound + 1e-300)


def _random_rows_csc(rng, m, n, k):
    """k random rows per column (duplicates summed), N(0,1) values, sorted CSC."""
    rows = rng.integers(0, m, size=n * k)
    cols = np.repeat(np.arange(n), k)
    A = sp.csc_matrix((rng.standard_normal(n * k), (rows, cols)), shape=(m, n))
    A.sum_duplicates()
    A.sort_indices()
    return A


@pytest.mark.parametrize("m,n,k", [(1_300_000, 600_000, 3), ((1 << 19) + 1, 70_000, 5),
                                   (200_000, (1 << 19) + 3, 2), (1 << 19, 1 << 19, 2),
                                   (600_000, 1_000, 700)])
def test_dual_step_sliced(h, m, n, k):
    """Vectors longer than 2^19 doubles are gathered in slices of 2 MB (x for the residual when
    n is that long, r for the dual when m is): r = A x - b and y_G = A_G^T r still within the
    rounding bound, y_F exactly 0, and y_G against the oracle's Eq. 5.  Covers both, one of
    each, a last slice of a single row or column, the sizes just below the threshold, and
    long columns (a wave's range of one slice spans several staging windows)."""
    rng = np.random.default_rng(m + n)
    A = _random_rows_csc(rng, m, n, k)
    b = rng.standard_normal(m)
    free = rng.random(n) < 0.4
    x = np.where(free, rng.standard_normal(n), 0.0)
    colptr, rowidx, val = csc_dev(A)
    yd = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    rd = torch.empty(m, dtype=torch.float64, device=DEV)
    print(f"sliced dual m={m} n={n} nnz={A.nnz}", flush=True)
    st = N.nnls_dual_csc(h, m, n, colptr, rowidx, val, t(b), t(free, np.uint8), t(x), rd, yd)
    assert st == N.NNLS_OK
    absA = abs(A)
    lr = int(np.diff(A.tocsr().indptr).max()) + 1   # longest row, plus b
    r_ref = A @ x - b
    rbound = (absA @ np.abs(x) + np.abs(b)) * 4 * lr * EPS
    assert np.all(np.abs(rd.cpu().numpy() - r_ref) <= rbound + 1e-300)
    yg = yd.cpu().numpy()
    assert np.all(yg[free] == 0.0)
    idx_f, idx_g = np.flatnonzero(free), np.flatnonzero(~free)
    y_or = np.zeros(n)
    y_or[idx_g] = dual(A, b, idx_f, x[idx_f], idx_g)
    ybound = (absA.T @ (absA @ np.abs(x) + np.abs(b))) * 8 * (lr + k + 1) * EPS
    assert np.all(np.abs(yg - y_or) <= ybound + 1e-300)


@pytest.mark.parametrize("m,n", [(40, 30), (300, 70), (5000, 40), (20000, 700), (1000, 1000)])
def test_dual_dense_step(h, m, n):
    """Dense Eq. 5 step (the residual splits over column chunks when the grid is short)."""
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    free = rng.random(n) < 0.4
    x = np.where(free, rng.standard_normal(n), 0.0)
    yd = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    rd = torch.empty(m, dtype=torch.float64, device=DEV)
    st = N.nnls_dual_dense(h, colmajor_dev(A), t(b), t(free, np.uint8), t(x), rd, yd)
    assert st == N.NNLS_OK
    r_ref = A @ x - b
    rbound = (np.abs(A) @ np.abs(x) + np.abs(b)) * 4 * n * EPS
    assert np.all(np.abs(rd.cpu().numpy() - r_ref) <= rbound + 1e-300)
    idx_f, idx_g = np.flatnonzero(free), np.flatnonzero(~free)
    y_or = np.zeros(n)
    y_or[idx_g] = dual(sp.csc_matrix(A), b, idx_f, x[idx_f], idx_g)
    yg = yd.cpu().numpy()
    assert np.all(yg[free] == 0.0)
    bound = (np.abs(A).T @ (np.abs(A) @ np.abs(x) + np.abs(b))) * 8 * m * EPS
    assert np.all(np.abs(yg - y_or) <= bound + 1e-300)


@pytest.mark.parametrize("seed", range(6))
def test_pivot_step_matches_rule(h, seed):
    """Classify, count, counter rule and exchange: bit-exact against the oracle's steps."""
    rng = np.random.default_rng(seed)
    n = [7, 64, 1000, 1023, 1025, 5000][seed]
    free = rng.random(n) < 0.5
    x = np.where(free, rng.standard_normal(n), 0.0)
    y = np.where(~free, rng.standard_normal(n), 0.0)
    # some entries inside the zeroing band, some exactly on its edge
    for arr in (x, y):
        k = rng.choice(n, size=max(1, n // 10), replace=False)
        arr[k] = rng.uniform(-1e-12, 1e-12, size=k.size)
    x[free & (rng.random(n) < 0.02)] = 1e-12
    for N_in, p_in in [(-1, 3), (n, 0), (0, 2), (0, 0)]:
        xo, yo, fo = x.copy(), y.copy(), free.copy()
        infeasible, _ = classify(xo, yo, fo, 1e-12)
        k = int(infeasible.sum())
        xd, yd, fd = t(x), t(y), t(free, np.uint8)
        state = [N_in, p_in]
        st, out = N.nnls_pivot_step(h, xd, yd, fd, 1e-12, 3, state)
        assert st == N.NNLS_OK
        assert out[0] == k
        Nprev = np.inf if N_in < 0 else N_in
        if k == 0:
            assert out[1] == -1
            continue
        N_new, p_new, branch = exchange_rule(k, Nprev, p_in, 3)
        assert out[1] == branch and state == [N_new, p_new]
        assert out[2] == int(np.flatnonzero(infeasible).max())
        if branch == 2:
            fo[out[2]] = not fo[out[2]]
        else:
            fo = fo ^ infeasible
        assert np.array_equal(fd.cpu().numpy().astype(bool), fo)
        assert out[3] == int(fo.sum())
        xg, yg = xd.cpu().numpy(), yd.cpu().numpy()
        # zeroed on the tested side, and x_G = 0, y_F = 0 on the new split
        assert np.array_equal(xg[fo], xo[fo]) and np.all(xg[~fo] == 0)
        assert np.array_equal(yg[~fo], yo[~fo]) and np.all(yg[fo] == 0)
