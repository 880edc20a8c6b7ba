"""Pins of the oracle's extensions (oracle/extend.py) against library routines, closed forms
and invariants; `test_planted_*` plant mistakes and check that a pin catches each."""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

import gen
from oracle import extend, slk


@pytest.fixture(scope="module")
def fitted():
    inst = gen.gaussian_mixture(n=600, d=6, L=4, K=8, seed=41)
    rng = np.random.default_rng(42)
    Y = (inst.X[rng.choice(inst.N, 50, replace=False)] + rng.normal(0, 0.3, (50, inst.D))).astype(np.float32)
    Z = rng.dirichlet(np.ones(inst.L), size=inst.N)
    idx, d2 = slk.knn(inst.X, inst.K, block=256)
    return dict(inst=inst, Y=Y, Z=Z, s2=slk.sigma2_from_knn(d2))


def test_knn_query_matches_kdtree(fitted):
    inst, Y = fitted["inst"], fitted["Y"]
    idx, d2 = extend.knn_query(inst.X, Y, 7)
    dd, ii = cKDTree(inst.X.astype(np.float64)).query(Y.astype(np.float64), k=7)
    np.testing.assert_allclose(d2, dd ** 2, rtol=1e-12, atol=1e-12)
    assert np.mean(idx == ii) > 0.99          # equal up to exact ties


def test_knn_query_of_a_copied_point_is_itself_then_its_neighbours(fitted):
    inst = fitted["inst"]
    rows = np.array([3, 77, 512])
    idx, d2 = extend.knn_query(inst.X, inst.X[rows], 6)
    own, own_d = slk.knn(inst.X, 5, rows=rows)
    assert np.array_equal(idx[:, 0], rows) and np.all(d2[:, 0] == 0.0)
    assert np.array_equal(idx[:, 1:], own) and np.array_equal(d2[:, 1:], own_d)


def test_lambda_zero_is_nearest_mode(fitted):
    inst, Y = fitted["inst"], fitted["Y"]
    out = extend.predict(inst.X, fitted["Z"], inst.init_modes, Y, 5, fitted["s2"], 0.0)
    near = np.argmin(cdist(Y.astype(np.float64), inst.X[inst.init_modes].astype(np.float64), "sqeuclidean"), axis=1)
    assert np.array_equal(out["labels"], near)
    np.testing.assert_allclose(out["Z"].sum(axis=1), 1.0, atol=1e-12)
    assert np.all(out["Z"] >= 0)


def test_large_lambda_is_neighbour_vote(fitted):
    """With one-hot Z and a very large lambda the query takes the most frequent label among its
    k neighbours (a kNN classifier); where the vote ties, the label is one of the tied ones."""
    inst, Y = fitted["inst"], fitted["Y"]
    lab = np.random.default_rng(5).integers(0, inst.L, inst.N)
    Z = np.eye(inst.L)[lab]
    out = extend.predict(inst.X, Z, inst.init_modes, Y, 7, fitted["s2"], 1e6)
    _, nn = cKDTree(inst.X.astype(np.float64)).query(Y.astype(np.float64), k=7)
    votes = np.array([np.bincount(lab[r], minlength=inst.L) for r in nn])
    top = votes.max(axis=1)
    unique = (votes == top[:, None]).sum(axis=1) == 1
    assert unique.sum() > 30
    assert np.array_equal(out["labels"][unique], np.argmax(votes, axis=1)[unique])
    assert np.all(votes[np.arange(len(Y)), out["labels"]] == top)


def test_query_order_equivariance(fitted):
    inst, Y = fitted["inst"], fitted["Y"]
    perm = np.random.default_rng(9).permutation(len(Y))
    a = extend.predict(inst.X, fitted["Z"], inst.init_modes, Y, 5, fitted["s2"], 0.7)
    b = extend.predict(inst.X, fitted["Z"], inst.init_modes, Y[perm], 5, fitted["s2"], 0.7)
    np.testing.assert_array_equal(a["Z"][perm], b["Z"])


def test_planted_predict_mistakes_are_caught(fitted, monkeypatch):
    inst, Y = fitted["inst"], fitted["Y"]
    good = extend.predict

    def wrong_sign(X, Z, modes, Y, K, s2, lam):
        out = good(X, Z, modes, Y, K, s2, lam)
        S = out["A"] - lam * out["B"]
        return dict(out, S=S, Z=slk.softmax_rows(S), labels=np.argmax(S, axis=1))

    monkeypatch.setattr(extend, "predict", wrong_sign)
    with pytest.raises(AssertionError):
        test_large_lambda_is_neighbour_vote(fitted)
    monkeypatch.setattr(extend, "predict", good)

    def self_excluded(X, Y, K, block=64):
        # a plausible slip: excluding the nearest point as if the query were in X
        i, d = extend_knn(X, Y, K + 1)
        return i[:, 1:], d[:, 1:]

    extend_knn = extend.knn_query
    monkeypatch.setattr(extend, "knn_query", self_excluded)
    with pytest.raises(AssertionError):
        test_knn_query_of_a_copied_point_is_itself_then_its_neighbours(fitted)
