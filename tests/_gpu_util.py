"""Helpers for the GPU tests: move seeded instances to the device and call the C ABI."""
import numpy as np
import scipy.sparse as sp
import torch

import paper_cs_0408029_amd as N

DEV = torch.device("cuda:0")


def t(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV) if dtype is None else \
        torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).to(DEV)


def csc_dev(A):
    A = sp.csc_matrix(A)
    return (t(A.indptr, np.int32), t(A.indices, np.int32), t(A.data, np.float64))


def colmajor_dev(M):
    """(rows, cols) float64 device tensor in column-major layout."""
    return t(np.asarray(M, dtype=np.float64).T.copy()).t()


def solve_csc(h, A, b, **opt):
    A = sp.csc_matrix(A)
    m, n = A.shape
    colptr, rowidx, val = csc_dev(A)
    x = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    y = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    o = N.default_options(**opt)
    st, info = N.nnls_solve_csc(h, m, n, colptr, rowidx, val, t(b, np.float64), x, y, o)
    return st, info, x.cpu().numpy(), y.cpu().numpy(), N.nnls_get_trace(h)


def solve_dense(h, A, b, **opt):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Ad = colmajor_dev(A)
    x = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    y = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    o = N.default_options(**opt)
    st, info = N.nnls_solve_dense(h, Ad, t(b, np.float64), x, y, o)
    return st, info, x.cpu().numpy(), y.cpu().numpy(), N.nnls_get_trace(h)


def oracle_trace(res):
    return [(r.k, r.branch, r.N, r.p, r.n_free) for r in res.trace]


def certified(res, scale, rel=1e-8):
    """True when every sign test of the oracle run was at least rel*scale away from the
    zeroing threshold, so that rounding differences cannot flip a pivot decision."""
    margins = [r.min_margin for r in res.trace] + [res.final_margin]
    return min(margins) > rel * scale
