"""FP64 oracle of the extensions around SLK-BO (the rows after the hot path).

TEST INFRASTRUCTURE ONLY: nothing on the product path may import or call this module.

  predict      out-of-sample assignment.  Section 1 remarks that explicit assignment variables
               give a direct out-of-sample extension; the reading taken here applies the
               z-update of Eq. (8) once to each query with the fit held fixed: unary term to
               the fitted modes (Eq. (6a)), pairwise term over the query's k nearest fitted
               points with binary weights (Eq. (6b), the kNN affinity of Section 4.2).
  mean_shift   SLK-MS mode update: Eq. (9) iterated (readings MS1-MS3 below).
  fit_ms       Algorithm 1 with the SLK-MS branch.
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


# ----------------------------------------------------------------------------------
# SLK-MS: modes by mean-shift (Eq. (9), Algorithm 1's SLK-MS branch)
# ----------------------------------------------------------------------------------
# Readings where the paper is silent:
#   MS1  Eq. (9) takes the relaxed assignment of the last z-update (soft Z), the modes are
#        free vectors (no longer points of X), and the unary term of the next outer
#        iteration is k(x_p, m_l) at those vectors.
#   MS2  "until converges": the mean-shift loop stops when no mode moves by more than
#        tol * sigma in one step (or after max_iter steps); the outer loop stops when no
#        mode moves by more than tol * sigma over a whole mode update (or after max_outer).
#   MS3  a cluster with sum_p z_pl k(x_p, m_l) = 0 keeps its mode.

def unary_at(X, M, sigma2: float) -> np.ndarray:
    """A[p, l] = k(x_p, m_l) for mode vectors M (L x D)  (Eq. (6a))."""
    M64 = np.asarray(M, dtype=F64)
    return gaussian(sqdist_block(np.ascontiguousarray(M64.T), np.asarray(X, dtype=F64)), sigma2)


def mean_shift_step(X, Z, M, sigma2: float):
    """One step of Eq. (9) for every cluster: m_l <- sum_p w_pl x_p / sum_p w_pl with
    w_pl = z_pl k(x_p, m_l)."""
    X64 = np.asarray(X, dtype=F64)
    W = np.asarray(Z, dtype=F64) * unary_at(X64, M, sigma2)
    den = W.sum(axis=0)
    num = W.T @ X64
    Mn = np.array(M, dtype=F64, copy=True)
    ok = den > 0
    Mn[ok] = num[ok] / den[ok, None]
    return Mn


def mean_shift(X, Z, M, sigma2: float, tol: float = 1e-6, max_iter: int = 100):
    """Eq. (9) iterated until no mode moves by more than tol * sigma (MS2)."""
    M = np.asarray(M, dtype=F64)
    it = 0
    for it in range(1, max_iter + 1):
        Mn = mean_shift_step(X, Z, M, sigma2)
        shift = float(np.sqrt(((Mn - M) ** 2).sum(axis=1)).max())
        M = Mn
        if shift <= tol * np.sqrt(sigma2):
            break
    return M, it


def fit_ms(X, row_ptr, col_idx, M0, sigma2: float, lam: float, *, tol: float = 1e-8, max_inner: int = 1000,
           max_outer: int = 20, ms_tol: float = 1e-6, ms_max: int = 100, schedule=None):
    """Algorithm 1 with the SLK-MS mode update: per outer iteration the z-update block of SLK-BO
    for the unary term at the current mode vectors, then Eq. (9) iterated with the new Z."""
    from .slk import assign, csr_matrix
    X64 = np.asarray(X, dtype=F64)
    W = csr_matrix(row_ptr, col_idx, X64.shape[0])
    M = np.asarray(M0, dtype=F64)
    hist = []
    converged = False
    out = None
    for t in range(max_outer):
        n_inner = None if schedule is None else schedule[t]
        out = assign(X64, row_ptr, col_idx, None, sigma2, lam, tol=tol, max_inner=max_inner, n_inner=n_inner,
                     A=unary_at(X64, M, sigma2), W=W)
        Mn, its = mean_shift(X64, out["Z"], M, sigma2, ms_tol, ms_max)
        move = float(np.sqrt(((Mn - M) ** 2).sum(axis=1)).max())
        hist.append(dict(M=M, M_next=Mn, n_pass=out["n_pass"], ms_iters=its, E=out["E"], cut=out["cut"],
                         labels=out["labels"].copy(), move=move))
        if move <= ms_tol * np.sqrt(sigma2):
            converged = True
            M = Mn
            break
        M = Mn
    return dict(Z=out["Z"], S=out["S"], labels=out["labels"], modes=M, modes_used=hist[-1]["M"], E=out["E"],
                cut=out["cut"], history=hist, converged=converged, outer_iters=len(hist),
                inner_total=sum(h["n_pass"] for h in hist), last=out)
