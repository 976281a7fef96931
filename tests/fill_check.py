"""Symbolic Cholesky fill of the F-block H_FF = A_F^T A_F of the sparse workloads.

The paper factors H_FF with a sparse supernodal Cholesky (Sec. 3).  The solver here
factors it as a dense tiled matrix, which is only sound when the sparse factor of H_FF
would be nearly dense anyway.  This module measures that from the nonzero pattern alone
(no values, so no numerical cancellation is counted), for three orders of F:

* the natural order of the columns;
* reverse Cuthill-McKee (scipy), a bandwidth-reducing order;
* greedy minimum degree on the elimination graph, the classic fill-reducing heuristic.

``python -m tests.fill_check`` prints the table of the full-size workloads; the tests in
``test_fill_cpu.py`` pin the counting functions on patterns whose fill has a closed form
and check the fill of scaled-down workloads of the same recipes.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

_ONE = np.uint64(1)


def _bits(idx: np.ndarray, nw: int) -> np.ndarray:
    w = np.zeros(nw, dtype=np.uint64)
    if idx.size:
        np.bitwise_or.at(w, idx >> 6, np.left_shift(_ONE, (idx & 63).astype(np.uint64)))
    return w


def _first_bit(w: np.ndarray) -> int:
    nz = np.flatnonzero(w)
    if nz.size == 0:
        return -1
    q = int(nz[0])
    v = int(w[q])
    return 64 * q + ((v & -v).bit_length() - 1)


def symmetric_pattern(H) -> sp.csc_matrix:
    """The structurally symmetric pattern of H (both triangles), as a 0/1 CSC matrix with
    sorted indices and the diagonal included."""
    P = sp.csc_matrix(H, copy=True)
    P.data = np.ones_like(P.data, dtype=np.int8)
    P = (P + P.T + sp.identity(P.shape[0], dtype=np.int8, format="csc")).tocsc()
    P.data[:] = 1
    P.sort_indices()
    return P


def gram_pattern(A, cols=None) -> sp.csc_matrix:
    """Pattern of A_F^T A_F for the columns ``cols`` of A (all columns if None)."""
    B = sp.csc_matrix(A if cols is None else A[:, cols], copy=True)
    B.data = np.ones_like(B.data, dtype=np.int32)
    H = (B.T @ B).tocsc()
    return symmetric_pattern(H)


def column_counts(P: sp.csc_matrix, order=None) -> np.ndarray:
    """Below-diagonal nonzeros of each column of the Cholesky factor of a symmetric pattern
    P taken in the given order (a permutation of range(n); natural order if None).

    Column j of L holds the rows i > j of P's column j and the rows of every column c whose
    elimination-tree parent is j (the first row below c in c's column), except j itself.
    Column patterns are bitsets; a finished column is merged into its parent's pending set
    at once, so only the not-yet-reached parents hold storage."""
    n = P.shape[0]
    if order is not None:
        order = np.asarray(order)
        P = P[order][:, order].tocsc()
        P.sort_indices()
    nw = (n + 63) // 64
    pending: dict[int, np.ndarray] = {}
    counts = np.zeros(n, dtype=np.int64)
    indptr, indices = P.indptr, P.indices
    for j in range(n):
        rows = indices[indptr[j]:indptr[j + 1]]
        w = _bits(rows[rows > j], nw)
        acc = pending.pop(j, None)
        if acc is not None:
            np.bitwise_or(w, acc, out=w)
            w[j >> 6] &= ~np.left_shift(_ONE, np.uint64(j & 63))
        counts[j] = int(np.bitwise_count(w).sum())
        p = _first_bit(w)
        if p >= 0:
            q = pending.get(p)
            if q is None:
                pending[p] = w
            else:
                np.bitwise_or(q, w, out=q)
    return counts


def cholesky_nnz(P: sp.csc_matrix, order=None) -> int:
    """nnz(L), diagonal included (see column_counts)."""
    return P.shape[0] + int(column_counts(P, order).sum())


def flop_ratio(counts: np.ndarray) -> float:
    """Work of a sparse factor with these column counts against the dense factor of the
    same size: the column-by-column update work is the sum of the squared counts."""
    n = counts.size
    dense = np.arange(n - 1, -1, -1, dtype=np.float64)
    d = float((dense * dense).sum())
    return float((counts.astype(np.float64) ** 2).sum()) / d if d > 0 else 1.0


def min_degree(P: sp.csc_matrix):
    """Greedy minimum-degree elimination of a symmetric pattern: at each step the vertex of
    least current degree (lowest index on ties) is eliminated and its neighbours become a
    clique.  Returns (order, counts): the degree of each step's vertex at its elimination,
    which is the below-diagonal count of that column of the factor in that order."""
    n = P.shape[0]
    nw = (n + 63) // 64
    adj = np.zeros((n, nw), dtype=np.uint64)
    indptr, indices = P.indptr, P.indices
    for j in range(n):
        rows = indices[indptr[j]:indptr[j + 1]]
        rows = rows[rows != j]
        if rows.size:
            np.bitwise_or.at(adj[j], rows >> 6, np.left_shift(_ONE, (rows & 63).astype(np.uint64)))
    alive = np.ones(n, dtype=bool)
    deg = np.bitwise_count(adj).sum(axis=1).astype(np.int64)
    order = np.empty(n, dtype=np.int64)
    counts = np.zeros(n, dtype=np.int64)
    big = np.iinfo(np.int64).max
    for step in range(n):
        v = int(np.argmin(np.where(alive, deg, big)))
        order[step] = v
        alive[v] = False
        row = adj[v].copy()
        nb_idx = np.flatnonzero(np.unpackbits(row.view(np.uint8), bitorder="little")[:n])
        counts[step] = nb_idx.size
        if nb_idx.size:
            vbit = np.left_shift(_ONE, np.uint64(v & 63))
            sub = adj[nb_idx]
            sub |= row                                   # neighbours become a clique
            sub[:, v >> 6] &= ~vbit                      # v leaves the graph
            sub[np.arange(nb_idx.size), nb_idx >> 6] &= ~np.left_shift(
                _ONE, (nb_idx & 63).astype(np.uint64))   # no self loops
            adj[nb_idx] = sub
            deg[nb_idx] = np.bitwise_count(sub).sum(axis=1)
        adj[v] = 0
    return order, counts


def fill_report(P: sp.csc_matrix, with_min_degree: bool = True) -> dict:
    """Density of H_FF and, per order, the factor's density (nnz(L) / (n (n + 1) / 2)) and
    its work against the dense factor's (flop_ratio)."""
    n = P.shape[0]
    full = n * (n + 1) // 2
    lower = (P.nnz - n) // 2 + n
    out = {"n": n, "H_density": lower / full}
    orders = {"natural": None, "rcm": reverse_cuthill_mckee(P, symmetric_mode=True)}
    for name, order in orders.items():
        c = column_counts(P, order)
        out[name] = ((n + int(c.sum())) / full, flop_ratio(c))
    if with_min_degree:
        _, c = min_degree(P)
        out["min_degree"] = ((n + int(c.sum())) / full, flop_ratio(c))
    return out


def _active_subset(n: int, frac: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=int(round(frac * n)), replace=False))


def workload_blocks(scale: float = 1.0):
    """(name, H_FF pattern) for F-blocks of the sparse recipes: the planted active fraction
    and, for the block-band instance, the first iteration's 60% as well.  ``scale`` < 1
    shrinks m and n together (same nonzeros per column and rows per column)."""
    sys.path.insert(0, __file__.rsplit("/tests/", 1)[0])
    import workloads as W
    out = []
    m, n = int(60000 * scale), int(12000 * scale)
    A = W.rows_per_col_band_csc(np.random.default_rng(1002), m, n, 25)
    out.append((f"sparse {m}x{n}, 25/col + band, |F| = 30%", gram_pattern(A, _active_subset(n, 0.30, 7))))
    m, n = int(400000 * scale), int(50000 * scale)
    A = W.block_band_csc(np.random.default_rng(1005), m, n, 20)
    out.append((f"sparse {m}x{n}, 20/col + block band, |F| = 25%", gram_pattern(A, _active_subset(n, 0.25, 7))))
    out.append((f"sparse {m}x{n}, 20/col + block band, |F| = 60%", gram_pattern(A, _active_subset(n, 0.60, 8))))
    for nn in (1024, 8192):
        A = W.rows_per_col_band_csc(np.random.default_rng(1004), 3 * nn, nn, 20,
                                    band=(20 ** 0.5, 20 ** 0.5 / 2, 20 ** 0.5 / 4))
        out.append((f"serving {3 * nn}x{nn}, 20/col + band, |F| = 45%", gram_pattern(A, _active_subset(nn, 0.45, 9))))
    return out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--md-max", type=int, default=8000,
                    help="run minimum degree only on F-blocks up to this size")
    args = ap.parse_args()
    print("Factor density nnz(L) / (n (n+1)/2), and work against the dense factor, per order of F")
    print()
    print("| F-block | n | H_FF density | natural | reverse Cuthill-McKee | minimum degree | s |")
    print("|---|---|---|---|---|---|---|")
    for name, P in workload_blocks(args.scale):
        t0 = time.perf_counter()
        r = fill_report(P, with_min_degree=P.shape[0] <= args.md_max)
        cell = lambda k: f"{r[k][0]:.3f} / {r[k][1]:.3f}" if k in r else "-"
        print(f"| {name} | {r['n']} | {r['H_density']:.4f} | {cell('natural')} | {cell('rcm')} | "
              f"{cell('min_degree')} | {time.perf_counter() - t0:.1f} |", flush=True)


if __name__ == "__main__":
    main()
