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


# ------------------------------------------------------------------- SLK-MS (Eq. (9))

def symmetric_cloud(seed=0, n=200, d=5):
    """Points in pairs c + u, c - u: symmetric about c."""
    rng = np.random.default_rng(seed)
    u = rng.normal(0, 1.0, (n // 2, d))
    c = rng.normal(0, 3.0, d)
    return np.vstack([c + u, c - u]), c


def test_mean_shift_symmetric_cloud_converges_to_centre():
    X, c = symmetric_cloud()
    Z = np.ones((len(X), 1))
    # the centre is a fixed point of one step (the weights of x and its mirror are equal)
    np.testing.assert_allclose(extend.mean_shift_step(X, Z, c[None, :], 2.0)[0], c, rtol=0, atol=1e-12)
    M, it = extend.mean_shift(X, Z, (c + 0.3)[None, :], 2.0, tol=1e-12, max_iter=2000)
    np.testing.assert_allclose(M[0], c, atol=1e-8)


def test_mean_shift_climbs_to_the_nearer_group():
    """Two symmetric groups 10 apart, one cluster, a narrow kernel: started near the first group
    the mode goes to that group's centre (the far group's weight is below e^-18), not to the
    midpoint a plain average would give."""
    A, ca = symmetric_cloud(seed=1, n=100, d=2)
    A = ca + 0.2 * (A - ca)
    B = A + 10.0
    X = np.vstack([A, B])
    M, _ = extend.mean_shift(X, np.ones((len(X), 1)), (ca + 0.1)[None, :], 1.0, tol=1e-12, max_iter=500)
    np.testing.assert_allclose(M[0], ca, atol=1e-6)


def test_mean_shift_wide_kernel_is_weighted_mean():
    """As sigma grows, k -> 1 and one step gives the z-weighted mean of the points."""
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1, (150, 4))
    Z = rng.dirichlet(np.ones(3), size=150)
    M0 = rng.normal(0, 1, (3, 4))
    M1 = extend.mean_shift_step(X, Z, M0, 1e12)
    for l in range(3):
        np.testing.assert_allclose(M1[l], np.average(X, axis=0, weights=Z[:, l]), rtol=1e-9, atol=1e-9)


def test_mean_shift_ascends_the_weighted_density():
    rng = np.random.default_rng(4)
    X = np.vstack([rng.normal(0, 1, (100, 3)), rng.normal(4, 1, (100, 3))])
    Z = rng.dirichlet(np.ones(2), size=200)
    M = rng.normal(2, 2, (2, 3))
    dens = lambda M: (Z * extend.unary_at(X, M, 1.5)).sum(axis=0)
    prev = dens(M)
    for _ in range(30):
        M = extend.mean_shift_step(X, Z, M, 1.5)
        cur = dens(M)
        assert np.all(cur >= prev - 1e-12)
        prev = cur


def test_mean_shift_translation_equivariance():
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (120, 3))
    Z = rng.dirichlet(np.ones(2), size=120)
    M0 = rng.normal(0, 1, (2, 3))
    t = np.array([5.0, -2.0, 0.5])
    a, _ = extend.mean_shift(X, Z, M0, 1.0, tol=1e-12, max_iter=500)
    b, _ = extend.mean_shift(X + t, Z, M0 + t, 1.0, tol=1e-12, max_iter=500)
    np.testing.assert_allclose(b, a + t, atol=1e-7)


def test_fit_ms_final_modes_are_mean_shift_fixed_points():
    inst = gen.gaussian_mixture(n=400, d=4, L=3, K=8, seed=77)
    idx, d2 = slk.knn(inst.X, 8, block=256)
    rp, ci = slk.symmetrize(idx, inst.N)
    s2 = slk.sigma2_from_knn(d2)
    out = extend.fit_ms(inst.X, rp, ci, inst.X[inst.init_modes], s2, 1.0, ms_tol=1e-7)
    assert out["converged"]
    last = out["history"][-1]
    again = extend.mean_shift_step(inst.X, out["last"]["Z"], last["M_next"], s2)
    assert np.sqrt(((again - last["M_next"]) ** 2).sum(axis=1)).max() <= 1e-6 * np.sqrt(s2)
    np.testing.assert_allclose(out["Z"].sum(axis=1), 1.0, atol=1e-12)


def test_planted_mean_shift_mistakes_are_caught(monkeypatch):
    good = extend.mean_shift_step

    def unweighted(X, Z, M, sigma2):      # a dropped z factor
        return good(X, np.ones_like(np.asarray(Z, dtype=float)), M, sigma2)

    monkeypatch.setattr(extend, "mean_shift_step", unweighted)
    with pytest.raises(AssertionError):
        test_mean_shift_wide_kernel_is_weighted_mean()

    def no_kernel(X, Z, M, sigma2):       # the kernel weight left out (plain z-weighted mean)
        return good(X, Z, M, 1e30)

    monkeypatch.setattr(extend, "mean_shift_step", no_kernel)
    with pytest.raises(AssertionError):
        test_mean_shift_climbs_to_the_nearer_group()
