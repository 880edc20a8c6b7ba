"""The oracle's outer iteration (oracle.slk.assign with a given pass count) evaluated over row
blocks on a thread pool, for the full-size lock-step tests.

TEST INFRASTRUCTURE ONLY.  It calls the oracle's own functions in assign's order; each of them
works row by row (distances, the Gaussian kernel, the CSR product, the softmax, the per-row bound
terms, the log-odds), so splitting the rows changes no operation, and the global sums are taken
with math.fsum over all rows, which is exactly rounded and so independent of any split.  Results
equal oracle.slk.assign bit for bit (checked on the CPU in test_oracle.py)."""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import slk as orc


def _blocks(n, parts):
    step = max(1, -(-n // parts))
    return [(s, min(n, s + step)) for s in range(0, n, step)]


class RowPool:
    def __init__(self, threads=None):
        self.threads = threads or min(16, os.cpu_count() or 1)
        self.ex = ThreadPoolExecutor(self.threads)

    def map_rows(self, n, fn, parts=None):
        """fn(s, e) for row blocks [s, e); returns the results in row order."""
        return list(self.ex.map(lambda b: fn(*b), _blocks(n, parts or 4 * self.threads)))

    def close(self):
        self.ex.shutdown()


def assign(pool, X, row_ptr, col_idx, modes, sigma2, lam, n_inner, *, delta=0.0, scale=1.0, W=None, XT=None):
    """oracle.slk.assign(X, row_ptr, col_idx, modes, sigma2, lam, n_inner=n_inner, delta=..., scale=...)."""
    X64 = np.asarray(X, dtype=np.float64)
    N = X64.shape[0]
    W = orc.csr_matrix(row_ptr, col_idx, N) if W is None else W
    XT = np.ascontiguousarray(X64.T) if XT is None else XT
    M = X64[np.asarray(modes, dtype=np.int64)]
    A = np.concatenate(pool.map_rows(N, lambda s, e: orc.gaussian(orc.sqdist_block(XT[:, s:e], M).T, sigma2)))
    Z = np.concatenate(pool.map_rows(N, lambda s, e: orc.softmax_rows(A[s:e])))
    R_trace = []
    S = None
    Z_in = Z
    for _ in range(n_inner):
        B = np.concatenate(pool.map_rows(N, lambda s, e: orc.pairwise(W[s:e], Z, 0.0)))
        if delta:
            B = B + delta * Z
        S = A + scale * lam * B
        R_trace.append(math.fsum(np.concatenate(pool.map_rows(
            N, lambda s, e: orc.bound_rows(Z[s:e], A[s:e], B[s:e], lam, scale))).tolist()))
        Z_in = Z
        Z = np.concatenate(pool.map_rows(N, lambda s, e: orc.softmax_rows(S[s:e])))
    labels = orc.hard_labels(S)
    V = np.concatenate(pool.map_rows(N, lambda s, e: orc.log_odds(S[s:e])))
    new_modes, ties, V = orc.byproduct_modes(S, V)
    E, cut = orc.energy(A, labels, row_ptr, col_idx, lam)
    return dict(Z=Z, Z_in=Z_in, S=S, A=A, labels=labels, modes_next=new_modes, ties=ties, V=V, E=E, cut=cut,
                R_trace=R_trace, n_pass=len(R_trace), bound=R_trace[-1])
