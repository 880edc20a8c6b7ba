"""FP64 oracle of the initialisation protocol of Section 4.2 and of the exact modes.

TEST INFRASTRUCTURE ONLY: nothing on the product path may import or call this module.

  kmeanspp          K-means++ seeding (Section 4.2 names it for the initial centres; the
                    method is that of Arthur and Vassilvitskii, 2007: the first centre
                    uniform, every next one drawn with probability proportional to the
                    squared distance to the nearest centre chosen so far).
  nearest_labels    the initial assignment of every point to its nearest seed.
  dense_modes       modes by the definition in Eq. (1), m_l = argmax_{y in X} sum_p z_pl k(x_p, y),
                    and, with the previous modes given, the proximal hard-max of Eq. (10),
                    argmax_{y in X} [k(y, m_l) + sum_p z_pl k(x_p, y)].

Readings where the paper is silent:
  KP1  the random numbers are inputs: u_0 .. u_{L-1} in [0, 1).  The first centre is the point
       floor(u_0 N); centre r >= 1 is the smallest p whose prefix sum of D^2 (in point order)
       exceeds u_r * sum D^2, D^2(p) the squared distance to the nearest chosen centre.  When
       sum D^2 = 0 (every point sits on a chosen centre) centre r is floor(u_r N).
  KP2  distances are the fixed-order FP64 sums of sqdist_block (as for the kNN graph); the
       prefix sums run in point order.  Section 4.2's choice of the best of several seedings
       by validation accuracy is label-based tuning and is not part of the method here.
  IN1  the initial assignment puts every point in the cluster of its nearest seed (ties to
       the smaller l), one-hot.
  DM1  the kernel in Eqs. (1) and (10) is the Gaussian kernel of the unary term (Section 4.2);
       candidates y run over all points of X; ties go to the smaller index.
  DM2  a cluster with no weight (sum_p z_pl = 0) keeps its previous mode (its seed).
"""
from __future__ import annotations

import numpy as np

from .slk import F64, gaussian, sqdist_block


def kmeanspp(X, L: int, u):
    """K-means++ centres (point indices) for the uniforms u (length L), reading KP1.
    Returns (centres int64 [L], D2 float64 [N] after the last centre)."""
    X64 = np.asarray(X, dtype=F64)
    N = X64.shape[0]
    u = np.asarray(u, dtype=F64)
    if not (1 <= L <= N) or u.shape != (L,) or np.any(u < 0) or np.any(u >= 1):
        raise ValueError("need 1 <= L <= N and L uniforms in [0, 1)")
    XT = np.ascontiguousarray(X64.T)
    centres = [min(int(np.floor(u[0] * N)), N - 1)]
    D2 = np.full(N, np.inf)
    for r in range(1, L + 1):
        D2 = np.minimum(D2, sqdist_block(XT, X64[centres[-1]][None, :])[0])
        if r == L:
            break
        cum = np.cumsum(D2)
        total = cum[-1]
        if total > 0:
            p = int(np.searchsorted(cum, u[r] * total, side="right"))
        else:
            p = min(int(np.floor(u[r] * N)), N - 1)
        centres.append(p)
    return np.asarray(centres, dtype=np.int64), D2


def kmeanspp_margin(X, centres, u) -> np.ndarray:
    """For every draw r >= 1 the distance of the target u_r * sum D^2 from the nearest prefix
    sum, relative to sum D^2: where it is far above 2^-40 the choice does not depend on the
    order in which the prefix sums are formed."""
    X64 = np.asarray(X, dtype=F64)
    XT = np.ascontiguousarray(X64.T)
    D2 = np.full(X64.shape[0], np.inf)
    out = []
    for r in range(1, len(centres)):
        D2 = np.minimum(D2, sqdist_block(XT, X64[centres[r - 1]][None, :])[0])
        cum = np.cumsum(D2)
        total = cum[-1]
        if total <= 0:
            out.append(np.inf)
            continue
        t = u[r] * total
        out.append(float(np.min(np.abs(cum - t))) / total)
    return np.asarray(out)


def nearest_labels(X, centres) -> np.ndarray:
    """Reading IN1: label of every point = index of its nearest centre (ties to the smaller)."""
    X64 = np.asarray(X, dtype=F64)
    d = sqdist_block(np.ascontiguousarray(X64.T), X64[np.asarray(centres, dtype=np.int64)])   # L x N
    return np.argmin(d, axis=0)


def densities(X, Z, sigma2: float, prev=None, block: int = 256) -> np.ndarray:
    """P[y, l] = sum_p z_pl k(x_p, x_y) for every point y (the density term of Eqs. (1) and
    (10)); with prev (L point indices) the proximity term k(x_y, x_{prev_l}) is added."""
    X64 = np.asarray(X, dtype=F64)
    Z64 = np.asarray(Z, dtype=F64)
    XT = np.ascontiguousarray(X64.T)
    N = X64.shape[0]
    P = np.empty((N, Z64.shape[1]), dtype=F64)
    for s in range(0, N, block):
        K = gaussian(sqdist_block(XT, X64[s: s + block]), sigma2)        # candidates x points
        P[s: s + block] = K @ Z64
    if prev is not None:
        prev = np.asarray(prev, dtype=np.int64)
        P += gaussian(sqdist_block(np.ascontiguousarray(X64[prev].T), X64), sigma2)    # N x L
    return P


def dense_modes(X, Z, sigma2: float, prev=None, keep=None):
    """Modes by Eq. (1) (prev None) or Eq. (10) (prev = the previous modes): per cluster the
    candidate of largest P[y, l], ties to the smaller y.  A cluster with no weight keeps
    keep[l] (DM2; keep defaults to prev).  Returns (modes int64 [L], P)."""
    Z64 = np.asarray(Z, dtype=F64)
    P = densities(X, Z64, sigma2, prev)
    modes = np.argmax(P, axis=0).astype(np.int64)
    keep = prev if keep is None else keep
    empty = Z64.sum(axis=0) == 0
    if empty.any():
        if keep is None:
            raise ValueError("a cluster has no weight and there is no mode to keep")
        modes[empty] = np.asarray(keep, dtype=np.int64)[empty]
    return modes, P


def initial_modes(X, L: int, u, sigma2: float):
    """The initialisation of Section 4.2: K-means++ seeds, the nearest-seed assignment, and the
    start modes by the definition in Eq. (1).  Returns dict(seeds, labels, modes, P)."""
    seeds, _ = kmeanspp(X, L, u)
    lab = nearest_labels(X, seeds)
    Z = np.eye(L)[lab]
    modes, P = dense_modes(X, Z, sigma2, keep=seeds)
    return dict(seeds=seeds, labels=lab, modes=modes, P=P)
