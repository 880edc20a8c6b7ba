"""FP64 oracle of the extensions around SLK-BO (the rows after the hot path).

TEST INFRASTRUCTURE ONLY: nothing on the product path may import or call this module.

  predict      out-of-sample assignment.  Section 1 remarks that explicit assignment variables
               give a direct out-of-sample extension; the reading taken here applies the
               z-update of Eq. (8) once to each query with the fit held fixed: unary term to
               the fitted modes (Eq. (6a)), pairwise term over the query's k nearest fitted
               points with binary weights (Eq. (6b), the kNN affinity of Section 4.2).
"""
from __future__ import annotations

import numpy as np

from .slk import F64, gaussian, softmax_rows, sqdist_block


def knn_query(X, Y, K: int, block: int = 64):
    """For each row of Y, the K nearest rows of X under the Euclidean distance, ordered by
    (squared distance, index); nothing is excluded (the queries are not points of X).
    Distances are the fixed-order FP64 sums of sqdist_block."""
    X64 = np.asarray(X, dtype=F64)
    Y64 = np.asarray(Y, dtype=F64)
    N = X64.shape[0]
    if not (1 <= K <= N):
        raise ValueError("need 1 <= K <= N")
    XT = np.ascontiguousarray(X64.T)
    M = Y64.shape[0]
    out_i = np.empty((M, K), dtype=np.int64)
    out_d = np.empty((M, K), dtype=F64)
    qidx = np.arange(N)
    for s in range(0, M, block):
        d = sqdist_block(XT, Y64[s: s + block])
        for b in range(d.shape[0]):
            dp = d[b]
            kth = np.partition(dp, K - 1)[K - 1]
            cand = np.nonzero(dp <= kth)[0]
            order = np.lexsort((qidx[cand], dp[cand]))[:K]
            out_i[s + b] = cand[order]
            out_d[s + b] = dp[cand[order]]
    return out_i, out_d


def predict(X, Z, modes, Y, K: int, sigma2: float, lam: float):
    """Out-of-sample assignment of the queries Y against a fit (X, Z, modes).

    Returns dict(Z=softmax rows, S=logits, labels=argmax of S (ties to the smaller l),
    idx=the queries' neighbours, A=unary term, B=pairwise sums)."""
    X64 = np.asarray(X, dtype=F64)
    Y64 = np.asarray(Y, dtype=F64)
    Z64 = np.asarray(Z, dtype=F64)
    idx, _ = knn_query(X64, Y64, K)
    M64 = X64[np.asarray(modes, dtype=np.int64)]
    A = gaussian(sqdist_block(np.ascontiguousarray(M64.T), Y64), sigma2)      # Eq. (6a)
    B = Z64[idx].sum(axis=1)                                                  # Eq. (6b)
    S = A + lam * B
    return dict(Z=softmax_rows(S), S=S, labels=np.argmax(S, axis=1), idx=idx, A=A, B=B)
