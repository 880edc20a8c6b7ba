"""FP64 oracle of SLK-BO, written step by step from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product path
may import or call this module.

Every input array is widened to float64; every function computes in float64 with
plain NumPy/SciPy operations and no blocking or reordering beyond what the stated
definition allows.  Readings of the paper where it is silent or garbled:

  R1  factor 2: the z-update is the printed softmax(a + lambda*b) of Eq. (8); the
      relaxed bound it decreases is  sum z log z - sum z.a - (lambda/2) sum z.(K z)
      (the factor multiplying lambda/2 is `scale`, 1 by default; scale = 2 gives
      Eq. (2) as printed together with the update softmax(a + 2 lambda b)).
  R2  Z restarts from softmax(a) in every outer iteration (Algorithm 1).
  R3  two kernels: the Gaussian kernel in the unary term and the mode definition,
      the binary kNN affinity in the pairwise term (Section 4.2).
  R4  the kNN affinity is OR-symmetrised, binary, without self-loops.
  R5  optional diagonal shift K + delta*I (footnote to Proposition 1); delta = 0
      by default.
  R6  sigma^2 = mean squared distance over the N*k_n directed kNN pairs (Section 4.2).
  R7  kNN ties are broken by the smaller index; distances are the fixed-order
      FP64 sum of squared differences (no fused multiply-add).
  R8  byproduct modes (Eq. (11)) are ranked by the log-odds
      v_ql = s_ql - log sum_{j != l} exp(s_qj), which is increasing in z_ql;
      ties go to the smaller index; candidates within eps of the best form a tie set.
  R9  hard labels are the arg-max of the logits s_p (ties to the smaller l).
  R10 the inner loop stops when the relative change of the relaxed bound between
      consecutive iterates is <= tol, or after max_inner passes; the outer loop
      stops when the modes do not change (Section 3) or after max_outer.
  R11 the discrete energy is evaluated at the hard labels of the last z-update and
      the modes that produced its unary term.
"""
from __future__ import annotations

import math
import numpy as np
import scipy.sparse as sp
from scipy.special import logsumexp, xlogy

F64 = np.float64


# ----------------------------------------------------------------------------------
# Distances and the kNN affinity (Section 4.2, "Implementation details")
# ----------------------------------------------------------------------------------

def sqdist_block(XT: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances from each row of Q (B x D) to every point.

    XT is the D x N transpose of the float64 points.  The sum runs over the
    coordinates j = 0..D-1 in order; each step rounds (x - y), its square and the
    running sum separately (NumPy never fuses them)."""
    D, N = XT.shape
    d = np.zeros((Q.shape[0], N), dtype=F64)
    for j in range(D):
        t = XT[j][None, :] - Q[:, j][:, None]
        d += t * t
    return d


def knn(X, K: int, rows=None, block: int = 16):
    """Exact K nearest neighbours of each query row under the Euclidean distance,
    the point itself excluded, ordered by (distance, index).

    Returns (idx int64 [R, K], d2 float64 [R, K]) for the requested rows (all by
    default)."""
    X64 = np.asarray(X, dtype=F64)
    N = X64.shape[0]
    if not (1 <= K < N):
        raise ValueError("need 1 <= K < N")
    XT = np.ascontiguousarray(X64.T)
    rows = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    out_i = np.empty((len(rows), K), dtype=np.int64)
    out_d = np.empty((len(rows), K), dtype=F64)
    qidx = np.arange(N)
    for s in range(0, len(rows), block):
        r = rows[s: s + block]
        d = sqdist_block(XT, X64[r])
        for b, p in enumerate(r):
            dp = d[b]
            dp[p] = np.inf                      # a point is not its own neighbour
            kth = np.partition(dp, K - 1)[K - 1]
            cand = np.nonzero(dp <= kth)[0]
            order = np.lexsort((qidx[cand], dp[cand]))[:K]
            out_i[s + b] = cand[order]
            out_d[s + b] = dp[cand[order]]
    return out_i, out_d


def symmetrize(knn_idx: np.ndarray, N: int):
    """Binary affinity W with w_pq = 1 iff q is a kNN of p or p is a kNN of q,
    zero diagonal; returned as CSR (row_ptr int64, col_idx int64, sorted columns)."""
    K = knn_idx.shape[1]
    p = np.repeat(np.arange(N, dtype=np.int64), K)
    q = np.asarray(knn_idx, dtype=np.int64).ravel()
    keys = np.concatenate([p * N + q, q * N + p])
    keys = keys[(keys // N) != (keys % N)]
    keys = np.unique(keys)
    rows = keys // N
    cols = keys % N
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=N), out=row_ptr[1:])
    return row_ptr, cols


def csr_matrix(row_ptr, col_idx, N: int, vals=None):
    v = np.ones(len(col_idx), dtype=F64) if vals is None else np.asarray(vals, dtype=F64)
    return sp.csr_matrix((v, np.asarray(col_idx), np.asarray(row_ptr)), shape=(N, N))


def sigma2_from_knn(knn_d2: np.ndarray) -> float:
    """sigma^2 = (1 / (N k_n)) * sum over points and their k_n neighbours of the
    squared distance (Section 4.2)."""
    vals = np.asarray(knn_d2, dtype=F64).ravel()
    return math.fsum(vals.tolist()) / vals.size


# ----------------------------------------------------------------------------------
# Unary term a_p (Eq. (6a)) with the Gaussian kernel (Section 4.2)
# ----------------------------------------------------------------------------------

def gaussian(d2, sigma2: float):
    """k(x, y) = exp(-||x - y||^2 / (2 sigma^2))."""
    return np.exp(-np.asarray(d2, dtype=F64) / (2.0 * sigma2))


def unary(X, modes, sigma2: float) -> np.ndarray:
    """A[p, l] = k(x_p, m_l) with m_l = X[modes[l]]  (Eq. (6a))."""
    X64 = np.asarray(X, dtype=F64)
    XT = np.ascontiguousarray(X64.T)
    M = X64[np.asarray(modes, dtype=np.int64)]
    return gaussian(sqdist_block(XT, M).T, sigma2)


# ----------------------------------------------------------------------------------
# The z-update (Eqs. (6b), (7), (8)) and the bound (Eqs. (2), (4), (5))
# ----------------------------------------------------------------------------------

def softmax_rows(S: np.ndarray) -> np.ndarray:
    """Closed-form KKT solution of min_{z in simplex} z.(log z - s): z = exp(s)/1'exp(s)."""
    m = S.max(axis=1, keepdims=True)
    e = np.exp(S - m)
    return e / e.sum(axis=1, keepdims=True)


def pairwise(W, Z: np.ndarray, delta: float = 0.0) -> np.ndarray:
    """b_p = sum_q k(x_p, x_q) z_q with the affinity K + delta*I  (Eq. (6b))."""
    B = W @ Z
    if delta:
        B = B + delta * Z
    return B


def bound_rows(Z, A, B, lam: float, scale: float = 1.0) -> np.ndarray:
    """Per-point terms of the relaxed objective
    r_p = z_p.log z_p - z_p.a_p - (scale*lambda/2) z_p.b_p  with b = (K + delta I) Z."""
    return xlogy(Z, Z).sum(axis=1) - (Z * A).sum(axis=1) - 0.5 * scale * lam * (Z * B).sum(axis=1)


def relaxed_bound(Z, A, B, lam: float, scale: float = 1.0) -> float:
    return math.fsum(bound_rows(Z, A, B, lam, scale).tolist())


def aux_at_minimiser(S, Z_cur, B_cur, lam: float, scale: float = 1.0) -> float:
    """A_i(Z^{i+1}) with the additive constant that makes A_i(Z^i) = R(Z^i):
    sum_p -LSE(s_p) + (scale*lambda/2) sum_p z^i_p . b^i_p  (Eq. (5) at its minimiser)."""
    lse = logsumexp(S, axis=1)
    return math.fsum((-lse).tolist()) + 0.5 * scale * lam * math.fsum((Z_cur * B_cur).sum(axis=1).tolist())


def aux_value(Z, S, Z_cur, B_cur, lam: float, scale: float = 1.0) -> float:
    """A_i(Z) = sum_p z_p.(log z_p - s_p) + (scale*lambda/2) sum_p z^i_p.b^i_p for any Z."""
    t = (xlogy(Z, Z) - Z * S).sum(axis=1)
    return math.fsum(t.tolist()) + 0.5 * scale * lam * math.fsum((Z_cur * B_cur).sum(axis=1).tolist())


# ----------------------------------------------------------------------------------
# Labels, byproduct modes (Eq. (11)) and the discrete energy (Eq. (1), Eq. (3))
# ----------------------------------------------------------------------------------

def hard_labels(S: np.ndarray) -> np.ndarray:
    """l_p = argmax_l s_pl, ties to the smaller l (np.argmax returns the first)."""
    return np.argmax(S, axis=1).astype(np.int64)


def log_odds(S: np.ndarray) -> np.ndarray:
    """v_ql = s_ql - log sum_{j != l} exp(s_qj) = log(z_ql / (1 - z_ql)), computed
    without forming z; +inf when L = 1 (the sum is empty)."""
    N, L = S.shape
    V = np.empty_like(S)
    for l in range(L):
        if L == 1:
            V[:, l] = np.inf
            continue
        rest = np.delete(S, l, axis=1)
        V[:, l] = S[:, l] - logsumexp(rest, axis=1)
    return V


def ulp32(x: float) -> float:
    x = abs(float(x))
    if not math.isfinite(x):
        return 0.0
    return float(np.spacing(np.float32(x)))


def tie_eps(vmax: float) -> float:
    """Width of the tie set around the best log-odds: 64 FP32 ulps + 1e-6."""
    return 64.0 * ulp32(vmax) + 1e-6


def byproduct_modes(S: np.ndarray, V=None):
    """m_l = x_q with q = argmax_q z_ql  (Eq. (11)), ranked by log-odds, ties to the
    smaller index.  Also returns, per cluster, the tie set of candidates whose
    log-odds lie within tie_eps of the best.  V = log_odds(S) may be passed in when it
    is already at hand."""
    V = log_odds(S) if V is None else V
    modes = np.argmax(V, axis=0).astype(np.int64)
    ties = []
    for l in range(S.shape[1]):
        vmax = V[modes[l], l]
        if math.isinf(vmax):
            ties.append(np.nonzero(np.isinf(V[:, l]))[0])
        else:
            ties.append(np.nonzero(V[:, l] >= vmax - tie_eps(vmax))[0])
    return modes, ties, V


def cut_count(row_ptr, col_idx, labels) -> int:
    """Number of ordered pairs (p, q) with w_pq = 1 and l_p != l_q (exact integer)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(len(row_ptr) - 1), np.diff(row_ptr))
    lab = np.asarray(labels)
    return int(np.count_nonzero(lab[rows] != lab[np.asarray(col_idx)]))


def energy(A, labels, row_ptr, col_idx, lam: float):
    """E = -sum_p k(x_p, m_{l_p}) + (lambda/2) sum_{p,q} w_pq ||z_p - z_q||^2 for one-hot
    Z; the pairwise part equals lambda * (ordered cut) by Eq. (3).  Returns (E, cut)."""
    lab = np.asarray(labels, dtype=np.int64)
    un = math.fsum(np.asarray(A, dtype=F64)[np.arange(len(lab)), lab].tolist())
    cut = cut_count(row_ptr, col_idx, lab)
    return -un + lam * cut, cut


# ----------------------------------------------------------------------------------
# Algorithm 1 (SLK-BO)
# ----------------------------------------------------------------------------------

def inner_settled(r_prev: float, r_cur: float, tol: float) -> bool:
    """R10, the inner "until convergence" of Algorithm 1: the loop has settled once the relaxed
    bound of the newest input iterate differs from the bound of the one before it by at most
    tol times the magnitude of the earlier bound."""
    return abs(r_cur - r_prev) <= tol * abs(r_prev)


def assign(X, row_ptr, col_idx, modes, sigma2: float, lam: float, *, delta: float = 0.0,
           scale: float = 1.0, tol: float = 1e-8, max_inner: int = 1000,
           n_inner: int | None = None, A=None, W=None):
    """One outer iteration of Algorithm 1 for fixed modes: unary term, Z^0 = softmax(a),
    inner z-updates until the bound settles (R10) or for exactly n_inner passes
    (lock-step), then labels, byproduct modes and the energy."""
    X64 = np.asarray(X, dtype=F64)
    N = X64.shape[0]
    if W is None:
        W = csr_matrix(row_ptr, col_idx, N)
    if A is None:
        A = unary(X64, modes, sigma2)
    Z = softmax_rows(A)
    R_trace, Aux_trace = [], []
    passes = n_inner if n_inner is not None else max_inner
    S = None
    Z_in = Z
    for i in range(passes):
        B = pairwise(W, Z, delta)
        S = A + scale * lam * B
        R_trace.append(relaxed_bound(Z, A, B, lam, scale))
        Aux_trace.append(aux_at_minimiser(S, Z, B, lam, scale))
        Z_in = Z
        Z = softmax_rows(S)
        if n_inner is None and i >= 1 and inner_settled(R_trace[-2], R_trace[-1], tol):
            break
    labels = hard_labels(S)
    new_modes, ties, V = byproduct_modes(S)
    E, cut = energy(A, labels, row_ptr, col_idx, lam)
    return dict(Z=Z, Z_in=Z_in, S=S, A=A, labels=labels, modes_next=new_modes, ties=ties,
                V=V, E=E, cut=cut, R_trace=R_trace, Aux_trace=Aux_trace,
                n_pass=len(R_trace), bound=R_trace[-1])


def fit(X, row_ptr, col_idx, init_modes, sigma2: float, lam: float, *, delta: float = 0.0,
        scale: float = 1.0, tol: float = 1e-8, max_inner: int = 1000, max_outer: int = 20,
        schedule=None, choose_modes=None):
    """Algorithm 1 (SLK-BO): alternate z-updates with the modes fixed and byproduct
    mode updates until the modes do not change.

    schedule    -- optional list of inner pass counts per outer iteration (lock-step).
    choose_modes -- optional callable(t, oracle_modes, ties) -> modes used for the next
                    outer iteration (lets a test follow another implementation's pick
                    inside the oracle's tie sets)."""
    X64 = np.asarray(X, dtype=F64)
    N = X64.shape[0]
    W = csr_matrix(row_ptr, col_idx, N)
    modes = np.asarray(init_modes, dtype=np.int64).copy()
    history = []
    converged = False
    out = None
    for t in range(max_outer):
        n_inner = None if schedule is None else schedule[t]
        out = assign(X64, row_ptr, col_idx, modes, sigma2, lam, delta=delta, scale=scale,
                     tol=tol, max_inner=max_inner, n_inner=n_inner, W=W)
        nxt = out["modes_next"]
        if choose_modes is not None:
            nxt = np.asarray(choose_modes(t, nxt, out["ties"]), dtype=np.int64)
        history.append(dict(modes=modes.copy(), modes_next=nxt.copy(), n_pass=out["n_pass"],
                            E=out["E"], cut=out["cut"], bound=out["bound"], ties=out["ties"],
                            labels=out["labels"].copy()))
        if np.array_equal(nxt, modes):
            converged = True
            break
        modes = nxt
    return dict(Z=out["Z"], S=out["S"], labels=out["labels"], modes=history[-1]["modes_next"],
                modes_used=history[-1]["modes"], E=out["E"], cut=out["cut"], bound=out["bound"],
                history=history, converged=converged, outer_iters=len(history),
                inner_total=sum(h["n_pass"] for h in history), last=out)


def energy_of(X, row_ptr, col_idx, labels, modes, sigma2: float, lam: float):
    """E(l, M) computed from the points: unary term from the FP64 Gaussian kernel."""
    A = unary(X, modes, sigma2)
    return energy(A, labels, row_ptr, col_idx, lam)
