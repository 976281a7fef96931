"""nnls_solve_dense_batched_noalloc (every device buffer from the library's fixed per-GPU
scratch array) against nnls_solve_dense_batched on the same problems: bitwise identical x,
y and per-problem results, on two calls in a row where the second batch is smaller (the
scratch array then still holds the first call's contents), and a batch larger than the
array rejected before anything runs."""
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


def _buffers(problems):
    As = [colmajor_dev(A) for A, _ in problems]
    bs = [t(b) for _, b in problems]
    xs = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    ys = [torch.full((A.shape[1],), np.nan, dtype=torch.float64, device=DEV) for A, _ in problems]
    return As, bs, xs, ys


def _both(h, problems, **opt):
    o = N.default_options(**opt)
    As, bs, xs, ys = _buffers(problems)
    st_a, info_a = N.nnls_solve_dense_batched_noalloc(h, As, bs, xs, ys, o)
    xa = [x.cpu().numpy() for x in xs]
    ya = [y.cpu().numpy() for y in ys]
    for v in xs + ys:
        v.fill_(np.nan)
    st_r, info_r = N.nnls_solve_dense_batched(h, As, bs, xs, ys, o)
    xr = [x.cpu().numpy() for x in xs]
    yr = [y.cpu().numpy() for y in ys]
    return (st_a, info_a, xa, ya), (st_r, info_r, xr, yr)


def _assert_same(a, r):
    st_a, info_a, xa, ya = a
    st_r, info_r, xr, yr = r
    assert st_a == st_r == N.NNLS_OK
    for ia, ir, x1, x2, y1, y2 in zip(info_a, info_r, xa, xr, ya, yr):
        assert (ia.status, ia.iterations, ia.n_free, ia.last_ninf, ia.ir_steps, ia.failed_index) == \
               (ir.status, ir.iterations, ir.n_free, ir.last_ninf, ir.ir_steps, ir.failed_index)
        assert np.array_equal(x1, x2) and np.array_equal(y1, y2)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_batched_twice_smaller_second(h, precision):
    first = [(i.A, i.b) for i in W.dense_batch(1003, count=40)]
    insts2 = [i for i in W.dense_batch(2003, count=40) if i.n <= 128][:12]
    second = [(i.A, i.b) for i in insts2]
    assert len(second) == 12
    print(f"noalloc: precision={precision} first batch 40 (n max {max(A.shape[1] for A, _ in first)}), "
          f"second batch 12 (n max {max(A.shape[1] for A, _ in second)})", flush=True)
    a, r = _both(h, first, precision=precision)
    _assert_same(a, r)
    a, r = _both(h, second, precision=precision)
    _assert_same(a, r)
    # the second call's results are right on their own as well (planted free sets, oracle x)
    tol = 1e-10 if precision == 0 else 1e-8
    for inst, x in zip(insts2, a[2]):
        assert np.array_equal(x > 0, inst.active)
        ref = bpp_solve(inst.A, inst.b)
        assert np.linalg.norm(x - ref.x) <= tol * np.linalg.norm(ref.x)


def test_noalloc_rejects_batch_beyond_scratch(h):
    m, n = 1024, 256
    rng = np.random.default_rng(7)
    A = colmajor_dev(rng.standard_normal((m, n)) / np.sqrt(m))
    b = t(rng.standard_normal(m))
    count = 80   # about 1 MB of workspace each: beyond the 64 MiB array
    x = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    y = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    st, _ = N.nnls_solve_dense_batched_noalloc(h, [A] * count, [b] * count, [x] * count, [y] * count)
    assert st == N.NNLS_ERR_TOO_LARGE
    assert N.status_string(st) == "NNLS_ERR_TOO_LARGE"
    assert torch.isnan(x).all() and torch.isnan(y).all()   # nothing ran
