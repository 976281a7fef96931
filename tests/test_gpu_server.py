"""Serving engine (continuous batching) against the oracle: every request of a mixed stream,
on both lanes (batched launches for small n, concurrent sparse solves for large n), gives
the oracle's free set and x within 1e-10 (float64) or 1e-8 (float32 factor + float64
refinement); each result is bitwise the same alone and in the mix; admission respects the
device-memory budget; bad requests fail alone."""
import threading

import numpy as np
import pytest

import workloads as W
from oracle import bpp_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_cs_0408029_amd as N  # noqa: E402


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def submit(srv, inst):
    m, n = inst.A.shape
    cp, ri, va = W.csc_arrays(inst.A)
    st, ticket = N.nnls_server_submit_csc(srv, m, n, cp, ri, va, inst.b)
    assert st == N.NNLS_OK, N.status_string(st)
    return ticket


def run_all(srv, insts):
    tickets = [submit(srv, p) for p in insts]
    out = []
    for tk, p in zip(tickets, insts):
        st, x, y, info = N.nnls_server_wait(srv, tk, p.A.shape[1], timeout_ms=60000)
        assert st != N.NNLS_ERR_TIMEOUT
        out.append((st, x, y, info))
    return out


@pytest.fixture(scope="module")
def stream_small():
    # n log-uniform in [24, 600]: both lanes at batch_max_n = 160
    _, probs = W.serving_stream(1004, count=20, n_lo=24, n_hi=600)
    return probs


@pytest.fixture(scope="module")
def oracle_small(stream_small):
    return [bpp_solve(p.A.toarray(), p.b) for p in stream_small]


def check_against_oracle(insts, results, refs, tol):
    for p, (st, x, y, info), res in zip(insts, results, refs):
        assert res.status == "ok"
        assert st == N.NNLS_OK and info.status == N.NNLS_OK, (p.name, N.status_string(st))
        assert info.n_free == int(res.free.sum()), p.name
        assert np.array_equal(x > 0, res.x > 0), p.name
        assert np.array_equal(x > 0, p.active), p.name
        assert relerr(x, res.x) <= tol, p.name
        assert np.linalg.norm(y - res.y) <= tol * max(np.linalg.norm(res.y), 1.0), p.name
        assert np.all(x >= 0) and np.all(y >= 0) and np.dot(x, y) == 0.0


def test_default_config_matches_oracle(stream_small, oracle_small):
    """The engine's defaults (16 sparse workers, each factor capped at 96 workgroups, 2
    batched lanes for n <= 256): every request of the mixed stream gives the oracle's split
    and x within 1e-10."""
    with N.Server(0) as srv:
        res = run_all(srv, stream_small)
    check_against_oracle(stream_small, res, oracle_small, 1e-10)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8), (2, 1e-8)])
def test_mixed_stream_matches_oracle(stream_small, oracle_small, precision, tol):
    """precision 2 (NNLS_BF16_IR): bfloat16-update factors on the sparse lane, the float32
    tier on the batched lanes."""
    with N.Server(0, opts=N.default_options(precision=precision), workers=4, batch_lanes=2,
                  batch_max_n=160) as srv:
        results = run_all(srv, stream_small)
        stats = N.nnls_server_stats(srv)
    check_against_oracle(stream_small, results, oracle_small, tol)
    ns = [p.A.shape[1] for p in stream_small]
    assert min(ns) <= 160 < max(ns)          # both lanes were used
    assert stats["completed"] == len(stream_small) and stats["pending"] == 0
    assert stats["batches"] >= 1
    assert 0 < stats["p50_ms"] <= stats["p99_ms"] <= stats["max_ms"]


@pytest.fixture(scope="module")
def stream_full():
    """The serving recipe across the whole size range of the serving mix, n in [64, 8192]
    (m = 3n): two requests for the batched lane, five for the concurrent sparse lane."""
    return W.serving_sizes(1014, [64, 200, 600, 1500, 3000, 5500, 8192])


@pytest.fixture(scope="module")
def oracle_full(stream_full):
    return [bpp_solve(p.A, p.b) for p in stream_full]


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
def test_full_size_range_matches_oracle(stream_full, oracle_full, precision, tol):
    """Every request of the full size range against the sparse oracle, with several large
    requests factored at once on their capped persistent grids (128 workgroups each)."""
    with N.Server(0, opts=N.default_options(precision=precision), workers=4, batch_lanes=1,
                  batch_max_n=256) as srv:
        results = run_all(srv, stream_full)
        stats = N.nnls_server_stats(srv)
    check_against_oracle(stream_full, results, oracle_full, tol)
    assert stats["completed"] == len(stream_full)
    assert stats["max_running"] > 1


def test_alone_equals_mix_bitwise(stream_small):
    with N.Server(0, workers=4, batch_lanes=2, batch_max_n=160) as srv:
        alone = []
        for p in stream_small:      # one request in the server at a time
            alone.append(run_all(srv, [p])[0])
        mixed = run_all(srv, stream_small)
        stats = N.nnls_server_stats(srv)
    assert stats["max_running"] > 1           # the mix really overlapped
    for p, a, b in zip(stream_small, alone, mixed):
        assert a[0] == b[0] == N.NNLS_OK
        assert np.array_equal(a[1], b[1]), p.name
        assert np.array_equal(a[2], b[2]), p.name
        assert a[3].iterations == b[3].iterations


def test_concurrent_submitters(stream_small, oracle_small):
    """Several host threads submit and wait at once (the calls are thread-safe)."""
    results = [None] * len(stream_small)
    with N.Server(0, workers=3, batch_lanes=1, batch_max_n=160) as srv:
        def client(idx):
            for i in idx:
                results[i] = run_all(srv, [stream_small[i]])[0]
        threads = [threading.Thread(target=client, args=(list(range(k, len(stream_small), 4)),))
                   for k in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
    check_against_oracle(stream_small, results, oracle_small, 1e-10)


def test_budget_limits_admission(stream_small, oracle_small):
    # a budget below any request's footprint admits one request at a time
    with N.Server(0, workers=4, batch_lanes=2, batch_max_n=160, hbm_budget=1) as srv:
        results = run_all(srv, stream_small)
        stats = N.nnls_server_stats(srv)
    assert stats["max_running"] == 1
    check_against_oracle(stream_small, results, oracle_small, 1e-10)


def test_sparse_lane_only_matches_batched_lane(stream_small):
    """The same requests through either lane: same free sets, x within 1e-10."""
    sub = stream_small[:8]
    with N.Server(0, workers=2, batch_max_n=-1) as srv:
        sparse = run_all(srv, sub)
    with N.Server(0, workers=1, batch_lanes=1, batch_max_n=100000) as srv:
        batched = run_all(srv, sub)
    for p, a, b in zip(sub, sparse, batched):
        assert a[0] == b[0] == N.NNLS_OK
        assert np.array_equal(a[1] > 0, b[1] > 0), p.name
        assert relerr(a[1], b[1]) <= 1e-10, p.name


@pytest.mark.parametrize("precision", [0, 1])
def test_iteration_level_steps_equal_whole_solves(stream_small, precision):
    """The batched lane advances live requests a few pivot iterations per step and admits
    and retires requests between steps; the pivot state carried from step to step gives
    bitwise the same result as a whole solve in one launch, for every step size."""
    sub = [p for p in stream_small if p.A.shape[1] <= 160]
    opts = N.default_options(precision=precision)
    runs = {}
    for iters in (-1, 1, 2):
        with N.Server(0, opts=opts, workers=1, batch_lanes=1, batch_max_n=160, batch_step_iters=iters) as srv:
            runs[iters] = run_all(srv, sub)
            stats = N.nnls_server_stats(srv)
        if iters == 1:   # a request takes several steps, so there were more steps than requests
            assert stats["batches"] > 1
    for k, p in enumerate(sub):
        ref = runs[-1][k]
        assert ref[0] == N.NNLS_OK, p.name
        for iters in (1, 2):
            got = runs[iters][k]
            assert got[0] == N.NNLS_OK
            assert np.array_equal(got[1], ref[1]), (p.name, iters)
            assert np.array_equal(got[2], ref[2]), (p.name, iters)
            assert got[3].iterations == ref[3].iterations
            assert got[3].ir_steps == ref[3].ir_steps


def test_bad_requests_fail_alone(stream_small):
    good = stream_small[:6]
    with N.Server(0, workers=2, batch_lanes=1, batch_max_n=160) as srv:
        m, n = good[0].A.shape
        cp, ri, va = W.csc_arrays(good[0].A)
        # host-side structure checks: nothing is queued
        bad_ri = ri.copy()
        bad_ri[0] = m
        assert N.nnls_server_submit_csc(srv, m, n, cp, bad_ri, va, good[0].b)[0] == N.NNLS_ERR_INVALID_ARG
        if cp[1] - cp[0] >= 2:
            swp = ri.copy()
            swp[0], swp[1] = swp[1], swp[0]
            assert N.nnls_server_submit_csc(srv, m, n, cp, swp, va, good[0].b)[0] == N.NNLS_ERR_INVALID_ARG
        assert N.nnls_server_submit_csc(srv, n - 1, n, cp, ri, va, good[0].b[:n - 1])[0] == N.NNLS_ERR_INVALID_ARG
        # non-finite values are found on the device, per request, on both lanes
        tickets = []
        for i, p in enumerate(good):
            mm, nn = p.A.shape
            c2, r2, v2 = W.csc_arrays(p.A)
            b2 = p.b.copy()
            if i in (1, 4):
                b2[3] = np.nan
            st, tk = N.nnls_server_submit_csc(srv, mm, nn, c2, r2, v2, b2)
            assert st == N.NNLS_OK
            tickets.append((tk, nn, i))
        for tk, nn, i in tickets:
            st, x, y, info = N.nnls_server_wait(srv, tk, nn, timeout_ms=60000)
            if i in (1, 4):
                assert st == N.NNLS_ERR_INVALID_VALUE and info.status == st
            else:
                assert st == N.NNLS_OK and np.array_equal(x > 0, good[i].active)
        # unknown / already claimed tickets
        assert N.nnls_server_wait(srv, tickets[0][0], 5, timeout_ms=0)[0] == N.NNLS_ERR_INVALID_ARG
        st, done, *_ = N.nnls_server_poll(srv, 123456789, 5)
        assert st == N.NNLS_ERR_INVALID_ARG


def test_poll_reports_progress_and_reset_stats(stream_small):
    p = stream_small[0]
    with N.Server(0, workers=1, batch_max_n=-1) as srv:
        tk = submit(srv, p)
        n = p.A.shape[1]
        seen_done = False
        for _ in range(200000):
            st, done, x, y, info = N.nnls_server_poll(srv, tk, n)
            if done:
                seen_done = True
                break
        if not seen_done:
            st, x, y, info = N.nnls_server_wait(srv, tk, n, timeout_ms=60000)
        assert st == N.NNLS_OK and np.array_equal(x > 0, p.active)
        assert info.solve_ms >= info.setup_ms >= 0
        s1 = N.nnls_server_stats(srv)
        assert s1["completed"] == 1 and s1["submitted"] == 1
        N.nnls_server_reset_stats(srv)
        s2 = N.nnls_server_stats(srv)
        assert s2["completed"] == 0 and s2["submitted"] == 0


def test_destroy_with_queued_requests(stream_small):
    srv = N.Server(0, workers=1, batch_lanes=1, batch_max_n=160)
    for p in stream_small:
        submit(srv, p)
    srv.close()          # running requests finish, queued ones are dropped
