"""Pins of the seeding and exact-mode oracle (oracle/seeding.py): closed forms, the sampling
distribution of K-means++ on points whose squared distances are exact integers, library
routines for the nearest-seed assignment, brute force on tiny inputs, and planted mistakes."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import gen
from oracle import seeding


def line(positions):
    """Points on the first axis of R^3 at integer positions (every squared distance exact)."""
    X = np.zeros((len(positions), 3), dtype=np.float32)
    X[:, 0] = positions
    return X


# ------------------------------------------------------------------- K-means++

def test_kmeanspp_zero_uniforms_take_the_first_new_point():
    """u = 0: the first centre is point 0 and every next one is the first point not yet on a
    centre (the smallest p whose prefix sum of D^2 is positive)."""
    X = gen.gaussian_mixture(n=50, d=4, L=3, seed=1).X
    c, _ = seeding.kmeanspp(X, 7, np.zeros(7))
    assert c.tolist() == list(range(7))


def test_kmeanspp_near_one_uniforms_take_the_last_new_point():
    X = gen.gaussian_mixture(n=50, d=4, L=3, seed=1).X
    c, _ = seeding.kmeanspp(X, 5, np.full(5, 1.0 - 1e-15))
    assert c.tolist() == [49, 48, 47, 46, 45]


def test_kmeanspp_second_centre_follows_d2_sampling():
    """Points at 0, 1, 3, 6, 10 with the first centre at 0: D^2 = 0, 1, 9, 36, 100, so over a
    uniform grid of u the second centre is p with frequency D^2(p) / 146."""
    X = line([0, 1, 3, 6, 10])
    M = 146 * 40
    counts = np.zeros(5)
    for i in range(M):
        c, _ = seeding.kmeanspp(X, 2, np.array([0.0, (i + 0.5) / M]))
        counts[c[1]] += 1
    np.testing.assert_array_equal(counts, np.array([0, 1, 9, 36, 100]) * 40)


def test_kmeanspp_third_centre_uses_the_nearest_chosen_centre():
    """Centres 0 and 10 on the line 0, 1, 3, 6, 10: D^2 = 0, 1, 9, 16, 0 (6 is nearer to 10)."""
    X = line([0, 1, 3, 6, 10])
    M = 26 * 20
    counts = np.zeros(5)
    for i in range(M):
        c, D2 = seeding.kmeanspp(X, 3, np.array([0.0, 0.999, (i + 0.5) / M]))
        assert c[1] == 4
        counts[c[2]] += 1
    np.testing.assert_array_equal(counts, np.array([0, 1, 9, 16, 0]) * 20)


def test_kmeanspp_never_repeats_a_location_while_others_remain():
    rng = np.random.default_rng(3)
    base = rng.integers(-5, 6, size=(12, 3)).astype(np.float32)
    base = np.unique(base, axis=0)
    X = np.vstack([base, base[:5], base[:5]])           # duplicates of some points
    for trial in range(30):
        u = rng.random(len(base))
        c, _ = seeding.kmeanspp(X, len(base), u)
        locs = {tuple(X[i]) for i in c}
        assert len(locs) == len(base)                    # every distinct location exactly once


def test_kmeanspp_all_points_on_centres_falls_back_to_uniform():
    X = line([2, 2, 2, 2])
    c, D2 = seeding.kmeanspp(X, 3, np.array([0.1, 0.6, 0.99]))
    assert c.tolist() == [0, 2, 3] and np.all(D2 == 0)


def test_kmeanspp_translation_invariance_on_integer_points():
    rng = np.random.default_rng(4)
    X = rng.integers(-50, 50, size=(300, 5)).astype(np.float32)
    u = rng.random(9)
    a, _ = seeding.kmeanspp(X, 9, u)
    b, _ = seeding.kmeanspp(X + np.float32(1000), 9, u)
    assert np.array_equal(a, b)


def test_kmeanspp_brute_force_tiny():
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (9, 2)).astype(np.float32)
    u = rng.random(4)
    pts = [[float(v) for v in r] for r in X]
    cent = [min(int(math.floor(u[0] * 9)), 8)]
    for r in range(1, 4):
        d2 = [min(sum((a - b) ** 2 for a, b in zip(p, pts[c])) for c in cent) for p in pts]
        t = u[r] * math.fsum(d2)
        acc = 0.0
        for p, v in enumerate(d2):
            acc += v
            if acc > t:
                cent.append(p)
                break
    c, _ = seeding.kmeanspp(X, 4, u)
    assert c.tolist() == cent


def test_kmeanspp_margin_is_large_for_seeded_draws():
    inst = gen.gaussian_mixture(n=400, d=6, L=5, seed=6)
    u = np.random.default_rng(7).random(5)
    c, _ = seeding.kmeanspp(inst.X, 5, u)
    assert np.all(seeding.kmeanspp_margin(inst.X, c, u) > 2.0 ** -40)


def test_kmeanspp_rejects_bad_uniforms():
    X = line([0, 1, 2])
    with pytest.raises(ValueError):
        seeding.kmeanspp(X, 2, np.array([0.2, 1.0]))
    with pytest.raises(ValueError):
        seeding.kmeanspp(X, 4, np.zeros(4))


# ------------------------------------------------------------------- nearest seed

def test_nearest_labels_match_cdist_and_break_ties_low():
    X = line([0, 1, 2, 3, 4, 5, 6])
    lab = seeding.nearest_labels(X, [4, 2])              # point 3 is equidistant: cluster 0 (seed 4)
    np.testing.assert_array_equal(lab, [1, 1, 1, 0, 0, 0, 0])
    inst = gen.gaussian_mixture(n=500, d=7, L=6, seed=8)
    seeds = np.arange(0, 500, 83)
    ref = np.argmin(cdist(inst.X.astype(np.float64), inst.X[seeds].astype(np.float64), "sqeuclidean"), axis=1)
    np.testing.assert_array_equal(seeding.nearest_labels(inst.X, seeds), ref)


# ------------------------------------------------------------------- modes by definition

def test_narrow_kernel_mode_is_the_largest_membership():
    """With unit-spaced integer points and sigma^2 = 1e-3, k(x_p, x_y) = 1 if p = y and below
    e^-500 otherwise, so P[y, l] = z_yl and the mode is argmax_y z_yl (Eq. (11)'s choice)."""
    rng = np.random.default_rng(9)
    X = rng.permutation(np.arange(200)).reshape(-1, 1).astype(np.float32) * np.ones((1, 2), np.float32)
    Z = rng.dirichlet(np.ones(4), size=200)
    modes, P = seeding.dense_modes(X, Z, 1e-3)
    np.testing.assert_allclose(P, Z, rtol=0, atol=1e-300)
    np.testing.assert_array_equal(modes, np.argmax(Z, axis=0))


def test_wide_kernel_mode_is_the_point_nearest_the_weighted_mean():
    """As sigma grows, P[y, l] = W_l - (W_l ||y - mu_l||^2 + const) / (2 sigma^2) + O(sigma^-4)
    with mu_l the z-weighted mean: the mode is the data point nearest mu_l."""
    rng = np.random.default_rng(10)
    X = rng.normal(0, 3, (300, 4)).astype(np.float32)
    Z = rng.dirichlet(np.ones(3), size=300)
    modes, _ = seeding.dense_modes(X, Z, 1e8)
    X64 = X.astype(np.float64)
    for l in range(3):
        mu = np.average(X64, axis=0, weights=Z[:, l])
        d = ((X64 - mu) ** 2).sum(axis=1)
        srt = np.sort(d)
        assert srt[1] - srt[0] > 1e-3                    # a clear nearest point
        assert modes[l] == np.argmin(d)


def test_proximal_term_equal_pair_breaks_to_the_smaller_index():
    """One member q and previous mode r: P[q] = 1 + k(q, r) = P[r], the rest smaller, so the
    mode is min(q, r); a cluster with no weight keeps its previous mode (k(r, r) = 1).  The
    points are 10 apart, so a point between q and r scores below e^-12."""
    X = line([0, 10, 20, 30, 40, 50])
    Z = np.zeros((6, 2))
    Z[4, 0] = 1.0
    modes, P = seeding.dense_modes(X, Z, 2.0, prev=[1, 3])
    assert P[4, 0] == P[1, 0] and modes.tolist() == [1, 3]
    modes, _ = seeding.dense_modes(X, Z, 2.0, prev=[5, 2])
    assert modes.tolist() == [4, 2]


def test_empty_cluster_keeps_its_seed():
    X = line([0, 1, 2, 3])
    Z = np.zeros((4, 2))
    Z[:, 0] = 1.0
    modes, _ = seeding.dense_modes(X, Z, 1.0, keep=[0, 3])
    assert modes[1] == 3
    with pytest.raises(ValueError):
        seeding.dense_modes(X, Z, 1.0)


def test_dense_modes_brute_force_tiny():
    rng = np.random.default_rng(11)
    X = rng.normal(0, 1, (7, 3)).astype(np.float32)
    Z = rng.dirichlet(np.ones(2), size=7)
    prev = [2, 5]
    s2 = 0.7
    pts = [[float(v) for v in r] for r in X]
    k = lambda a, b: math.exp(-sum((x - y) ** 2 for x, y in zip(a, b)) / (2 * s2))
    for use_prev in (False, True):
        want = []
        for l in range(2):
            vals = [sum(Z[p, l] * k(pts[p], pts[y]) for p in range(7)) + (k(pts[y], pts[prev[l]]) if use_prev else 0)
                    for y in range(7)]
            want.append(int(np.argmax(vals)))
            got_P = seeding.densities(X, Z, s2, prev if use_prev else None)[:, l]
            np.testing.assert_allclose(got_P, vals, rtol=1e-13)
        modes, _ = seeding.dense_modes(X, Z, s2, prev if use_prev else None)
        assert modes.tolist() == want


def test_point_permutation_equivariance():
    inst = gen.gaussian_mixture(n=250, d=5, L=3, seed=12)
    Z = np.random.default_rng(13).dirichlet(np.ones(3), size=250)
    perm = np.random.default_rng(14).permutation(250)
    a, Pa = seeding.dense_modes(inst.X, Z, 20.0)
    b, Pb = seeding.dense_modes(inst.X[perm], Z[perm], 20.0)
    np.testing.assert_allclose(Pa[perm], Pb, rtol=1e-12)
    np.testing.assert_array_equal(perm[b], a)


def test_initial_modes_pipeline():
    inst = gen.gaussian_mixture(n=600, d=5, L=4, seed=15)
    u = np.random.default_rng(16).random(4)
    out = seeding.initial_modes(inst.X, 4, u, 15.0)
    seeds, _ = seeding.kmeanspp(inst.X, 4, u)
    np.testing.assert_array_equal(out["seeds"], seeds)
    np.testing.assert_array_equal(out["labels"], seeding.nearest_labels(inst.X, seeds))
    # every seed is in its own cluster (distance 0); every mode has the largest density
    assert np.all(out["labels"][seeds] == np.arange(4))
    P = out["P"]
    assert np.all(P[out["modes"], np.arange(4)] == P.max(axis=0))


# ------------------------------------------------------------------- planted mistakes

def test_planted_seeding_mistakes_are_caught(monkeypatch):
    good_pp = seeding.kmeanspp

    # '>=' in place of '>' in the prefix rule
    import oracle.seeding as S

    def ge_rule(X, L, u):
        X64 = np.asarray(X, dtype=np.float64)
        XT = np.ascontiguousarray(X64.T)
        N = X64.shape[0]
        cen = [min(int(np.floor(u[0] * N)), N - 1)]
        D2 = np.full(N, np.inf)
        for r in range(1, L + 1):
            D2 = np.minimum(D2, S.sqdist_block(XT, X64[cen[-1]][None, :])[0])
            if r == L:
                break
            cum = np.cumsum(D2)
            cen.append(int(np.searchsorted(cum, u[r] * cum[-1], side="left")))
        return np.asarray(cen), D2

    monkeypatch.setattr(seeding, "kmeanspp", ge_rule)
    with pytest.raises(AssertionError):
        test_kmeanspp_zero_uniforms_take_the_first_new_point()
    monkeypatch.setattr(seeding, "kmeanspp", good_pp)

    def sqrt_weights(X, L, u):                 # D instead of D^2
        X64 = np.asarray(X, dtype=np.float64)
        XT = np.ascontiguousarray(X64.T)
        N = X64.shape[0]
        cen = [min(int(np.floor(u[0] * N)), N - 1)]
        D2 = np.full(N, np.inf)
        for r in range(1, L + 1):
            D2 = np.minimum(D2, S.sqdist_block(XT, X64[cen[-1]][None, :])[0])
            if r == L:
                break
            cum = np.cumsum(np.sqrt(D2))
            cen.append(int(np.searchsorted(cum, u[r] * cum[-1], side="right")))
        return np.asarray(cen), D2

    monkeypatch.setattr(seeding, "kmeanspp", sqrt_weights)
    with pytest.raises(AssertionError):
        test_kmeanspp_second_centre_follows_d2_sampling()
    monkeypatch.setattr(seeding, "kmeanspp", good_pp)

    good_dens = seeding.densities

    def no_z(X, Z, sigma2, prev=None, block=256):          # the z factor dropped
        return good_dens(X, np.ones_like(np.asarray(Z, dtype=float)), sigma2, prev, block)

    monkeypatch.setattr(seeding, "densities", no_z)
    with pytest.raises(AssertionError):
        test_narrow_kernel_mode_is_the_largest_membership()
