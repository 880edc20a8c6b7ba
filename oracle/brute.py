"""Brute-force minimisation of the discrete Laplacian K-modes objective (Eq. (1)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For tiny problems (N <= 8, L <= 4) every labeling l in [L]^N is enumerated.  The
modes are taken by their definition in Eq. (1): m_l = argmax_{y in X} sum_{p: l_p = l}
k(x_p, y) with the Gaussian kernel (ties to the smaller index; an empty cluster has no
mode and contributes nothing), and

    E_def(l) = -sum_p k(x_p, m_{l_p}) + lambda * #{ordered (p, q): w_pq = 1, l_p != l_q}.
"""
from __future__ import annotations

import itertools
import math
import numpy as np

from . import slk


def gram(X, sigma2: float) -> np.ndarray:
    """G[p, q] = k(x_p, x_q), Gaussian kernel on the FP64 fixed-order distances."""
    X64 = np.asarray(X, dtype=np.float64)
    XT = np.ascontiguousarray(X64.T)
    return slk.gaussian(slk.sqdist_block(XT, X64), sigma2)


def modes_by_definition(G: np.ndarray, labels, L: int):
    """Mode of each cluster as the data point maximising the cluster's kernel density
    (Eq. (1), second line); -1 for an empty cluster."""
    lab = np.asarray(labels)
    modes = np.full(L, -1, dtype=np.int64)
    for l in range(L):
        members = np.nonzero(lab == l)[0]
        if len(members) == 0:
            continue
        dens = G[members].sum(axis=0)          # density of cluster l at every y in X
        modes[l] = int(np.argmax(dens))        # first maximiser: smaller index wins
    return modes


def energy_def(G: np.ndarray, row_ptr, col_idx, labels, L: int, lam: float):
    lab = np.asarray(labels, dtype=np.int64)
    modes = modes_by_definition(G, lab, L)
    un = math.fsum(G[p, modes[lab[p]]] for p in range(len(lab)))
    cut = slk.cut_count(row_ptr, col_idx, lab)
    return -un + lam * cut, modes


def minimise(X, row_ptr, col_idx, L: int, sigma2: float, lam: float):
    """Exhaustive minimum of E_def over all L^N labelings.  Returns (E_min, labels, modes)."""
    N = np.asarray(X).shape[0]
    if N > 8 or L > 4:
        raise ValueError("brute force is limited to N <= 8 and L <= 4")
    G = gram(X, sigma2)
    best = (math.inf, None, None)
    for lab in itertools.product(range(L), repeat=N):
        E, modes = energy_def(G, row_ptr, col_idx, lab, L, lam)
        if E < best[0] - 1e-12:
            best = (E, np.asarray(lab), modes)
    return best


def canonical(labels) -> tuple:
    """Labels renamed in order of first appearance (compares partitions up to relabelling)."""
    seen = {}
    return tuple(seen.setdefault(int(v), len(seen)) for v in labels)
