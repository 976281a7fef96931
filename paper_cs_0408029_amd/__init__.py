"""MI355X (gfx950) block principal pivoting NNLS.

Thin Python layer over the C ABI of lib/libnnls.so (include/nnls.h).  The functions below
carry the C names and only marshal arguments: they take torch device tensors, check
dtype / device / layout, and pass raw device pointers and the handle's HIP stream.
PyTorch supplies device memory and streams; every step of the method runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Tuple

from ._lib import (LIB_PATH, NNLS_ERR_DEVICE, NNLS_ERR_INVALID_ARG, NNLS_ERR_INVALID_VALUE,  # noqa: F401
                   NNLS_ERR_MAXITER, NNLS_ERR_NO_MEMORY, NNLS_ERR_NOT_PD, NNLS_ERR_REFINE,
                   NNLS_ERR_TIMEOUT, NNLS_ERR_TOO_LARGE, NNLS_NOALLOC_SCRATCH_BYTES, NNLS_FLAG_GRAM_DUAL, NNLS_FLAG_NO_FACTOR_REUSE, NNLS_FLAG_PROFILE, NNLS_FLAG_REFINE_ALL, NNLS_FLAG_REFINE_AUTO, NNLS_FLAG_REFINE_FINAL, NNLS_BF16_IR, NNLS_FP32_IR, NNLS_FP64, NNLS_OK,
                   NNLS_PROFILE_CLASSES, PROFILE_CLASS_NAMES, default_options, load, nnls_info,
                   nnls_options, nnls_server_config, nnls_serving_stats, nnls_trace_row,
                   status_string)


def _torch():
    import torch
    return torch


def _ptr(t, dtype, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs at least {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


class Handle:
    """Owns an nnls_handle bound to a device and a HIP stream (torch's current stream of
    that device unless one is given)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = C.c_void_p()
        st = self.lib.nnls_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != NNLS_OK:
            raise RuntimeError(f"nnls_create failed: {status_string(st)}")
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        if self._h:
            self.lib.nnls_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nnls_solve_csc(h: Handle, m: int, n: int, colptr, rowidx, val, b, x, y,
                   opts: Optional[nnls_options] = None) -> Tuple[int, nnls_info]:
    torch = _torch()
    nnz = int(rowidx.numel())
    info = nnls_info()
    st = h.lib.nnls_solve_csc(h.ptr, m, n, nnz, _ptr(colptr, torch.int32, "colptr", n + 1),
                              _ptr(rowidx, torch.int32, "rowidx"), _ptr(val, torch.float64, "val", nnz),
                              _ptr(b, torch.float64, "b", m), _ptr(x, torch.float64, "x", n),
                              _ptr(y, torch.float64, "y", n), C.byref(opts) if opts else None,
                              C.byref(info))
    return st, info


def nnls_solve_dense(h: Handle, A, b, x, y, opts: Optional[nnls_options] = None) -> Tuple[int, nnls_info]:
    """A: float64 device tensor of shape (m, n) in column-major layout (A.stride(0) == 1),
    e.g. the transpose of a contiguous (n, m) tensor."""
    torch = _torch()
    m, n = A.shape
    if A.dtype != torch.float64 or not A.is_cuda or A.stride(0) != 1:
        raise ValueError("A: expected a column-major float64 device tensor")
    lda = A.stride(1) if n > 1 else m
    info = nnls_info()
    st = h.lib.nnls_solve_dense(h.ptr, m, n, C.c_void_p(A.data_ptr()), lda, _ptr(b, torch.float64, "b", m),
                                _ptr(x, torch.float64, "x", n), _ptr(y, torch.float64, "y", n),
                                C.byref(opts) if opts else None, C.byref(info))
    return st, info


class BatchedArgs:
    """Host descriptor arrays of a batch (sizes, leading dimensions, device pointers),
    marshalled once so that repeated nnls_solve_dense_batched calls on the same tensors
    pass them without rebuilding them."""

    def __init__(self, As, bs, xs, ys):
        torch = _torch()
        batch = len(As)
        if not (len(bs) == len(xs) == len(ys) == batch):
            raise ValueError("As, bs, xs, ys must have the same length")
        cap = max(batch, 1)
        self.batch = batch
        self.m = (C.c_int32 * cap)()
        self.n = (C.c_int32 * cap)()
        self.lda = (C.c_int32 * cap)()
        self.pa = (C.c_void_p * cap)()
        self.pb = (C.c_void_p * cap)()
        self.px = (C.c_void_p * cap)()
        self.py = (C.c_void_p * cap)()
        for i, (A, b, x, y) in enumerate(zip(As, bs, xs, ys)):
            mi, ni = A.shape
            if A.dtype != torch.float64 or not A.is_cuda or A.stride(0) != 1:
                raise ValueError("A: expected a column-major float64 device tensor")
            self.m[i], self.n[i] = mi, ni
            self.lda[i] = A.stride(1) if ni > 1 else mi
            self.pa[i] = A.data_ptr()
            self.pb[i] = _ptr(b, torch.float64, "b", mi).value
            self.px[i] = _ptr(x, torch.float64, "x", ni).value
            self.py[i] = _ptr(y, torch.float64, "y", ni).value
        self.infos = (nnls_info * cap)()
        # keep the tensors alive as long as the descriptors point at them
        self._keep = (As, bs, xs, ys)


def nnls_solve_dense_batched(h: Handle, As=None, bs=None, xs=None, ys=None,
                             opts: Optional[nnls_options] = None, packed: Optional[BatchedArgs] = None):
    """As: list of column-major float64 device matrices (m_i, n_i); bs, xs, ys: lists of
    float64 device vectors (or `packed`, a BatchedArgs built from them once).  Returns
    (status, [nnls_info per problem])."""
    p = packed if packed is not None else BatchedArgs(As, bs, xs, ys)
    vp = lambda arr: C.cast(arr, C.c_void_p)
    st = h.lib.nnls_solve_dense_batched(h.ptr, p.batch, vp(p.m), vp(p.n), vp(p.pa), vp(p.lda), vp(p.pb),
                                        vp(p.px), vp(p.py), C.byref(opts) if opts else None, vp(p.infos))
    return st, list(p.infos[:p.batch])


def nnls_solve_dense_batched_noalloc(h: Handle, As=None, bs=None, xs=None, ys=None,
                                     opts: Optional[nnls_options] = None,
                                     packed: Optional[BatchedArgs] = None):
    """nnls_solve_dense_batched with every device buffer taken from the library's fixed
    per-GPU scratch array (no allocation).  Same arguments and result."""
    p = packed if packed is not None else BatchedArgs(As, bs, xs, ys)
    vp = lambda arr: C.cast(arr, C.c_void_p)
    st = h.lib.nnls_solve_dense_batched_noalloc(h.ptr, p.batch, vp(p.m), vp(p.n), vp(p.pa), vp(p.lda),
                                                vp(p.pb), vp(p.px), vp(p.py), C.byref(opts) if opts else None,
                                                vp(p.infos))
    return st, list(p.infos[:p.batch])


class BatchPlan:
    """A prepared batched solve (nnls_batch_plan): the batch's descriptors and workspace are
    set up once and one solve is captured in a HIP graph; execute() replays it on the
    handle's stream with whatever values A and b hold.  The tensors must stay alive and in
    place while the plan exists (the plan keeps references to them)."""

    def __init__(self, h: Handle, As, bs, xs, ys, opts: Optional[nnls_options] = None):
        self.h = h
        self.args = BatchedArgs(As, bs, xs, ys)
        p = self.args
        vp = lambda arr: C.cast(arr, C.c_void_p)
        plan = C.c_void_p()
        st = h.lib.nnls_batch_plan_create(h.ptr, p.batch, vp(p.m), vp(p.n), vp(p.pa), vp(p.lda), vp(p.pb),
                                          vp(p.px), vp(p.py), C.byref(opts) if opts else None, C.byref(plan))
        if st != NNLS_OK:
            raise RuntimeError(f"nnls_batch_plan_create failed: {status_string(st)}")
        self._p = plan

    def execute(self, wait: bool = True):
        """Replay once.  wait=True: returns (status, [nnls_info]); wait=False: returns the
        status of queueing it (read the results with info())."""
        if not wait:
            return self.h.lib.nnls_batch_plan_execute(self._p, None)
        st = self.h.lib.nnls_batch_plan_execute(self._p, C.cast(self.args.infos, C.c_void_p))
        return st, list(self.args.infos[:self.args.batch])

    def info(self):
        st = self.h.lib.nnls_batch_plan_info(self._p, C.cast(self.args.infos, C.c_void_p))
        return st, list(self.args.infos[:self.args.batch])

    def tile_shapes(self) -> dict:
        """{ceil(n/32): rectangles per wave per pass} as chosen by the autotuner."""
        out = (C.c_int32 * 9)()
        self.h.lib.nnls_batch_plan_tile_shapes(self._p, C.cast(out, C.c_void_p))
        return {k: out[k] for k in range(1, 9) if out[k]}

    def close(self):
        if self._p:
            self.h.lib.nnls_batch_plan_destroy(self._p)
            self._p = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nnls_get_trace(h: Handle, reused: bool = False, ir_steps: bool = False) -> List[Tuple[int, ...]]:
    """Per-iteration (k, branch, N, p, |F|); with reused=True also the count of leading F
    positions whose factor tiles were kept from the previous iteration; with ir_steps=True
    (instead) the refinement steps of each iteration's solve."""
    cnt = h.lib.nnls_get_trace(h.ptr, None, 0)
    rows = (nnls_trace_row * max(cnt, 1))()
    h.lib.nnls_get_trace(h.ptr, rows, cnt)
    if ir_steps:
        return [(r.k, r.branch, r.N, r.p, r.n_free, r.ir_steps) for r in rows[:cnt]]
    if reused:
        return [(r.k, r.branch, r.N, r.p, r.n_free, r.n_reused) for r in rows[:cnt]]
    return [(r.k, r.branch, r.N, r.p, r.n_free) for r in rows[:cnt]]


def nnls_get_profile(h: Handle) -> dict:
    la = (C.c_int64 * NNLS_PROFILE_CLASSES)()
    ms = (C.c_double * NNLS_PROFILE_CLASSES)()
    wk = (C.c_double * NNLS_PROFILE_CLASSES)()
    h.lib.nnls_get_profile(h.ptr, la, ms, wk)
    return {PROFILE_CLASS_NAMES[c]: {"launches": la[c], "ms": ms[c], "work": wk[c]}
            for c in range(NNLS_PROFILE_CLASSES)}


def nnls_reset_profile(h: Handle) -> int:
    return h.lib.nnls_reset_profile(h.ptr)


def nnls_set_profiling(h: Handle, on: bool) -> int:
    return h.lib.nnls_set_profiling(h.ptr, 1 if on else 0)


def nnls_gram_csc(h: Handle, m: int, n: int, colptr, rowidx, val, b, H, c) -> int:
    torch = _torch()
    nnz = int(rowidx.numel())
    if H.dtype != torch.float64 or not H.is_cuda or H.stride(0) != 1 or H.shape != (n, n):
        raise ValueError("H: expected an (n, n) column-major float64 device tensor")
    return h.lib.nnls_gram_csc(h.ptr, m, n, nnz, _ptr(colptr, torch.int32, "colptr", n + 1),
                               _ptr(rowidx, torch.int32, "rowidx"), _ptr(val, torch.float64, "val", nnz),
                               _ptr(b, torch.float64, "b", m), C.c_void_p(H.data_ptr()),
                               H.stride(1) if n > 1 else n, _ptr(c, torch.float64, "c", n))


def nnls_gram_dense(h: Handle, A, b, H, c) -> int:
    """A: column-major float64 device matrix (m, n); H: (n, n) column-major; c: (n,)."""
    torch = _torch()
    m, n = A.shape
    if A.dtype != torch.float64 or not A.is_cuda or A.stride(0) != 1:
        raise ValueError("A: expected a column-major float64 device matrix")
    if H.dtype != torch.float64 or not H.is_cuda or H.stride(0) != 1 or H.shape != (n, n):
        raise ValueError("H: expected an (n, n) column-major float64 device tensor")
    return h.lib.nnls_gram_dense(h.ptr, m, n, C.c_void_p(A.data_ptr()), A.stride(1) if n > 1 else m,
                                 _ptr(b, torch.float64, "b", m), C.c_void_p(H.data_ptr()),
                                 H.stride(1) if n > 1 else n, _ptr(c, torch.float64, "c", n))


def _colmajor(M, name):
    torch = _torch()
    if M.dtype != torch.float64 or not M.is_cuda or M.stride(0) != 1 or M.dim() != 2:
        raise ValueError(f"{name}: expected a column-major float64 device matrix")
    return C.c_void_p(M.data_ptr()), (M.stride(1) if M.shape[1] > 1 else M.shape[0])


def nnls_cholesky(h: Handle, S, L, precision: int = NNLS_FP64) -> Tuple[int, int]:
    n = S.shape[0]
    sp, lds = _colmajor(S, "S")
    lp, ldl = _colmajor(L, "L")
    failed = C.c_int32(-1)
    st = h.lib.nnls_cholesky(h.ptr, n, sp, lds, lp, ldl, precision, C.byref(failed))
    return st, failed.value


def nnls_spd_solve(h: Handle, S, rhs, x) -> Tuple[int, int]:
    torch = _torch()
    n = S.shape[0]
    sp, lds = _colmajor(S, "S")
    failed = C.c_int32(-1)
    st = h.lib.nnls_spd_solve(h.ptr, n, sp, lds, _ptr(rhs, torch.float64, "rhs", n),
                              _ptr(x, torch.float64, "x", n), C.byref(failed))
    return st, failed.value


def nnls_dual_csc(h: Handle, m: int, n: int, colptr, rowidx, val, b, free_flags, x, r, y) -> int:
    torch = _torch()
    nnz = int(rowidx.numel())
    return h.lib.nnls_dual_csc(h.ptr, m, n, nnz, _ptr(colptr, torch.int32, "colptr", n + 1),
                               _ptr(rowidx, torch.int32, "rowidx"), _ptr(val, torch.float64, "val", nnz),
                               _ptr(b, torch.float64, "b", m), _ptr(free_flags, torch.uint8, "free", n),
                               _ptr(x, torch.float64, "x", n),
                               _ptr(r, torch.float64, "r", m) if r is not None else None,
                               _ptr(y, torch.float64, "y", n))


def nnls_dual_dense(h: Handle, A, b, free_flags, x, r, y) -> int:
    """A: column-major float64 device matrix (m, n)."""
    torch = _torch()
    m, n = A.shape
    ap, lda = _colmajor(A, "A")
    return h.lib.nnls_dual_dense(h.ptr, m, n, ap, lda, _ptr(b, torch.float64, "b", m),
                                 _ptr(free_flags, torch.uint8, "free", n), _ptr(x, torch.float64, "x", n),
                                 _ptr(r, torch.float64, "r", m) if r is not None else None,
                                 _ptr(y, torch.float64, "y", n))


def nnls_pivot_step(h: Handle, x, y, free_flags, tau: float, p_max: int, state: List[int]):
    """state: [N, p] (N < 0 = infinity), updated in place.  Returns (status, [k, branch,
    largest infeasible index, new |F| or -1])."""
    torch = _torch()
    n = x.numel()
    st_arr = (C.c_int32 * 3)(state[0], state[1], 0)
    out = (C.c_int32 * 4)()
    st = h.lib.nnls_pivot_step(h.ptr, n, _ptr(x, torch.float64, "x", n), _ptr(y, torch.float64, "y", n),
                               _ptr(free_flags, torch.uint8, "free", n), tau, p_max, st_arr, out)
    state[0], state[1] = st_arr[0], st_arr[1]
    return st, list(out)


# ------------------------------------------------------------------------------------------
# Serving engine (host arrays in, host arrays out)
# ------------------------------------------------------------------------------------------

class Server:
    """Owns an nnls_server (continuous batching of independent requests on one device)."""

    def __init__(self, device: int = 0, config: Optional[nnls_server_config] = None,
                 opts: Optional[nnls_options] = None, **config_fields):
        self.lib = load()
        if config is None:
            config = nnls_server_config()
        for k, v in config_fields.items():
            setattr(config, k, v)
        s = C.c_void_p()
        st = self.lib.nnls_server_create(C.byref(s), device, C.byref(config),
                                         C.byref(opts) if opts else None)
        if st != NNLS_OK:
            raise RuntimeError(f"nnls_server_create failed: {status_string(st)}")
        self._s = s

    @property
    def ptr(self):
        return self._s

    def close(self):
        if self._s:
            self.lib.nnls_server_destroy(self._s)
            self._s = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host(a, dtype, name):
    import numpy as np
    arr = np.ascontiguousarray(a, dtype=dtype)
    if arr.ndim != 1:
        raise ValueError(f"{name}: expected a 1-D array")
    return arr


def nnls_server_create(device: int = 0, config: Optional[nnls_server_config] = None,
                       opts: Optional[nnls_options] = None, **config_fields) -> Server:
    return Server(device, config, opts, **config_fields)


def nnls_server_submit_csc(srv: Server, m: int, n: int, colptr, rowidx, val, b) -> Tuple[int, int]:
    """Host CSC arrays (numpy-convertible).  Returns (status, ticket)."""
    import numpy as np
    cp = _host(colptr, np.int32, "colptr")
    ri = _host(rowidx, np.int32, "rowidx")
    va = _host(val, np.float64, "val")
    bb = _host(b, np.float64, "b")
    if cp.size < n + 1 or bb.size < m or va.size < ri.size:
        raise ValueError("array sizes do not match m, n, nnz")
    ticket = C.c_uint64(0)
    st = srv.lib.nnls_server_submit_csc(srv.ptr, m, n, int(ri.size), cp.ctypes.data, ri.ctypes.data,
                                        va.ctypes.data, bb.ctypes.data, C.byref(ticket))
    return st, ticket.value


def _result_buffers(n):
    import numpy as np
    return np.empty(n, dtype=np.float64), np.empty(n, dtype=np.float64)


def nnls_server_poll(srv: Server, ticket: int, n: int):
    """Returns (status, done, x, y, info); x, y, info are None until done."""
    x, y = _result_buffers(n)
    info = nnls_info()
    done = C.c_int32(0)
    st = srv.lib.nnls_server_poll(srv.ptr, ticket, C.byref(done), x.ctypes.data, y.ctypes.data,
                                  C.byref(info))
    if not done.value:
        return st, False, None, None, None
    return st, True, x, y, info


def nnls_server_wait(srv: Server, ticket: int, n: int, timeout_ms: float = -1.0):
    """Returns (status, x, y, info); x, y, info are None on NNLS_ERR_TIMEOUT."""
    x, y = _result_buffers(n)
    info = nnls_info()
    st = srv.lib.nnls_server_wait(srv.ptr, ticket, timeout_ms, x.ctypes.data, y.ctypes.data,
                                  C.byref(info))
    if st in (NNLS_ERR_TIMEOUT, NNLS_ERR_INVALID_ARG):
        return st, None, None, None
    return st, x, y, info


def nnls_server_stats(srv: Server) -> dict:
    out = nnls_serving_stats()
    st = srv.lib.nnls_server_stats(srv.ptr, C.byref(out))
    if st != NNLS_OK:
        raise RuntimeError(f"nnls_server_stats failed: {status_string(st)}")
    return {name: getattr(out, name) for name, _ in nnls_serving_stats._fields_}


def nnls_server_reset_stats(srv: Server) -> int:
    return srv.lib.nnls_server_reset_stats(srv.ptr)


def nnls_server_destroy(srv: Server) -> int:
    srv.close()
    return NNLS_OK
