"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here re-types an oracle formula and compares it with itself: each test
checks the oracle against a hand-derived fixture (tests/golden), a library routine
computing the same quantity another way, a closed form, an invariant the paper
states, or exhaustive search on tiny inputs.  `test_planted_*` plant plausible
mistakes in the oracle (on the CPU) and check that some pin catches each one.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp
from scipy.spatial import cKDTree
from scipy.spatial.distance import cdist

import gen
from oracle import brute, slk

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def graph(inst, K=None):
    K = K or inst.K
    idx, d2 = slk.knn(inst.X, K, block=512)
    rp, ci = slk.symmetrize(idx, inst.N)
    return idx, d2, rp, ci, slk.sigma2_from_knn(d2)


@pytest.fixture(scope="module")
def small():
    inst = gen.gaussian_mixture(n=300, d=8, L=4, K=6, seed=11)
    return inst, graph(inst)


# ---------------------------------------------------------------- T1: kNN (Section 4.2)

def test_knn_golden_line():
    g = gold("line4_knn.json")
    idx, d2 = slk.knn(np.array(g["X"], dtype=np.float32), g["K"])
    assert idx.tolist() == g["knn_idx"]
    assert d2.tolist() == g["knn_d2"]


def test_knn_matches_kdtree(small):
    inst, (idx, d2, *_rest) = small
    tree = cKDTree(inst.X.astype(np.float64))
    dist, _ = tree.query(inst.X.astype(np.float64), k=inst.K + 1)
    # a library routine on the same points: the multiset of neighbour distances agrees
    np.testing.assert_allclose(np.sort(np.sqrt(d2), axis=1), dist[:, 1:], rtol=1e-12, atol=1e-12)


def test_knn_matches_cdist_bruteforce():
    inst = gen.gaussian_mixture(n=150, d=5, L=3, K=7, seed=3)
    D = cdist(inst.X.astype(np.float64), inst.X.astype(np.float64), "sqeuclidean")
    np.fill_diagonal(D, np.inf)
    idx, d2 = slk.knn(inst.X, 7)
    for p in range(inst.N):
        order = sorted(range(inst.N), key=lambda q: (D[p, q], q))[:7]
        assert idx[p].tolist() == order
        np.testing.assert_allclose(d2[p], D[p, order], rtol=1e-12)


def test_knn_ties_by_index():
    # duplicated points: equal distances are broken by the smaller index, self excluded
    X = np.array([[0, 0], [1, 0], [0, 0], [1, 0], [0, 0], [5, 5]], dtype=np.float32)
    idx, d2 = slk.knn(X, 3)
    assert idx[0].tolist() == [2, 4, 1]
    assert idx[2].tolist() == [0, 4, 1]
    assert idx[1].tolist() == [3, 0, 2]
    assert d2[0].tolist() == [0.0, 0.0, 1.0]


def test_knn_sample_rows_equal_full(small):
    inst, (idx, d2, *_r) = small
    rows = np.array([0, 7, 299, 150])
    i2, dd = slk.knn(inst.X, inst.K, rows=rows)
    assert np.array_equal(i2, idx[rows]) and np.array_equal(dd, d2[rows])


# ---------------------------------------------------------------- T2: symmetric W

def test_symmetrize_golden_line():
    g = gold("line4_knn.json")
    rp, ci = slk.symmetrize(np.array(g["knn_idx"]), 4)
    assert rp.tolist() == g["row_ptr"] and ci.tolist() == g["col_idx"]


def test_symmetrize_dense_or(small):
    inst, (idx, _d2, rp, ci, _s) = small
    N, K = inst.N, inst.K
    M = np.zeros((N, N), dtype=bool)
    M[np.repeat(np.arange(N), K), idx.ravel()] = True
    dense = M | M.T
    np.fill_diagonal(dense, False)
    W = slk.csr_matrix(rp, ci, N).toarray().astype(bool)
    assert np.array_equal(W, dense)
    assert np.all(np.diff(rp) >= K) and len(ci) <= 2 * K * N
    for p in range(N):
        row = ci[rp[p]:rp[p + 1]]
        assert np.all(np.diff(row) > 0)


# ---------------------------------------------------------------- T3: sigma^2 (Section 4.2)

def test_sigma2_golden_line():
    g = gold("line4_knn.json")
    _, d2 = slk.knn(np.array(g["X"], dtype=np.float32), g["K"])
    assert slk.sigma2_from_knn(d2) == g["sigma2"]


def test_sigma2_equals_mean_scipy(small):
    inst, (idx, d2, _rp, _ci, s2) = small
    X = inst.X.astype(np.float64)
    ref = np.mean(np.sum((X[:, None, :] - X[idx]) ** 2, axis=2))
    assert s2 == pytest.approx(ref, rel=1e-13)


# ---------------------------------------------------------------- unary term (Eq. (6a))

def test_unary_vs_cdist(small):
    inst, (*_g, s2) = small
    A = slk.unary(inst.X, inst.init_modes, s2)
    X = inst.X.astype(np.float64)
    ref = np.exp(-cdist(X, X[inst.init_modes], "sqeuclidean") / (2 * s2))
    np.testing.assert_allclose(A, ref, rtol=1e-12, atol=1e-300)
    assert np.allclose(A[inst.init_modes, np.arange(inst.L)], 1.0)


# ---------------------------------------------------------------- T6: softmax / KKT (Eqs. (7)-(8))

def test_softmax_golden():
    g = gold("softmax_kkt.json")
    c = np.array([g["c"]])
    z = slk.softmax_rows(c)
    np.testing.assert_allclose(z[0], g["z"], rtol=1e-14)
    val = float((z * (np.log(z) - c)).sum())
    assert val == pytest.approx(g["min_value"], rel=1e-14)


def test_softmax_is_kkt_minimiser():
    rng = np.random.default_rng(0)
    for L in (2, 3, 5):
        c = rng.normal(size=L) * 3
        f = lambda z: float(np.sum(z * (np.log(np.maximum(z, 1e-300)) - c)))
        cons = ({"type": "eq", "fun": lambda z: np.sum(z) - 1.0},)
        res = scipy.optimize.minimize(f, np.full(L, 1.0 / L), method="SLSQP", constraints=cons,
                                      bounds=[(1e-12, 1.0)] * L, options={"ftol": 1e-14, "maxiter": 500})
        z = slk.softmax_rows(c[None, :])[0]
        np.testing.assert_allclose(z, res.x, atol=2e-5)
        assert f(z) <= res.fun + 1e-12
        assert f(z) == pytest.approx(-scipy.special.logsumexp(c), abs=1e-12)
        # random feasible perturbations never go below the closed form
        for _ in range(50):
            y = rng.dirichlet(np.ones(L))
            assert f(y) >= f(z) - 1e-12


# ---------------------------------------------------------------- T5 / T7: simplex rows and the bound

def _trace_form_bound(Z, A, W, delta, lam, scale=1.0):
    """R(Z) through dense matrices: sum z log z - tr(Z'A) - (s*lam/2) tr(Z'(K + delta I)Z)."""
    Kd = W.toarray() + delta * np.eye(W.shape[0])
    return float(np.sum(scipy.special.xlogy(Z, Z)) - np.trace(Z.T @ A) - 0.5 * scale * lam * np.trace(Z.T @ Kd @ Z))


def test_bound_trace_form_and_tightness(small):
    inst, (_i, _d, rp, ci, s2) = small
    W = slk.csr_matrix(rp, ci, inst.N)
    A = slk.unary(inst.X, inst.init_modes, s2)
    Z = slk.softmax_rows(A)
    for delta in (0.0, 2.0):
        for _ in range(4):
            B = slk.pairwise(W, Z, delta)
            R = slk.relaxed_bound(Z, A, B, 1.3)
            assert R == pytest.approx(_trace_form_bound(Z, A, W, delta, 1.3), rel=1e-12)
            S = A + 1.3 * B
            # tightness A_i(Z^i) = R(Z^i) and descent A_i(Z^{i+1}) <= A_i(Z^i)  (Eq. (4))
            assert slk.aux_value(Z, S, Z, B, 1.3) == pytest.approx(R, rel=1e-12)
            Zn = slk.softmax_rows(S)
            assert slk.aux_at_minimiser(S, Z, B, 1.3) <= R + 1e-9 * abs(R)
            assert slk.aux_value(Zn, S, Z, B, 1.3) == pytest.approx(slk.aux_at_minimiser(S, Z, B, 1.3), rel=1e-12)
            Z = Zn


def test_bound_monotone_with_psd_shift(small):
    # with delta >= max degree, K + delta I is diagonally dominant, hence psd, and the
    # relaxed bound cannot increase between consecutive z-updates (Eq. (4), Prop. 1)
    inst, (_i, _d, rp, ci, s2) = small
    dmax = float(np.max(np.diff(rp)))
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 1.0, delta=dmax, n_inner=25)
    R = np.array(out["R_trace"])
    assert np.all(np.diff(R) <= 1e-10 * np.abs(R[:-1]))
    Aux = np.array(out["Aux_trace"])
    assert np.all(Aux[:-1] >= R[1:] - 1e-10 * np.abs(R[1:]))     # R(Z^{i+1}) <= A_i(Z^{i+1})
    assert np.all(Aux <= R + 1e-10 * np.abs(R))                  # A_i(Z^{i+1}) <= A_i(Z^i) = R(Z^i)
    assert np.allclose(out["Z"].sum(axis=1), 1.0, atol=1e-12) and np.all(out["Z"] >= 0)


def test_bound_with_eq2_scale_is_monotone(small):
    # the update softmax(a + 2 lambda b) is the bound optimizer of Eq. (2) as printed
    inst, (_i, _d, rp, ci, s2) = small
    dmax = float(np.max(np.diff(rp)))
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 0.7, delta=dmax, scale=2.0, n_inner=20)
    R = np.array(out["R_trace"])
    assert np.all(np.diff(R) <= 1e-10 * np.abs(R[:-1]))


# ---------------------------------------------------------------- T8 / T9: energy, identity (3)

def test_energy_golden_two_groups():
    g = gold("two_groups_energy.json")
    X = np.array(g["X"], dtype=np.float32)
    idx, d2 = slk.knn(X, g["K"])
    rp, ci = slk.symmetrize(idx, 4)
    assert slk.sigma2_from_knn(d2) == g["sigma2"]
    A = slk.unary(X, g["modes"], g["sigma2"])
    for c in g["cases"]:
        E, cut = slk.energy(A, c["labels"], rp, ci, g["lam"])
        assert cut == c["cut"]
        assert E == pytest.approx(c["E"], rel=1e-15)


def test_energy_three_ways(small):
    inst, (_i, _d, rp, ci, s2) = small
    rng = np.random.default_rng(1)
    W = slk.csr_matrix(rp, ci, inst.N).toarray()
    A = slk.unary(inst.X, inst.init_modes, s2)
    Lap = np.diag(W.sum(axis=1)) - W
    for _ in range(3):
        lab = rng.integers(0, inst.L, size=inst.N)
        Z = np.eye(inst.L)[lab]
        E, cut = slk.energy(A, lab, rp, ci, 0.8)
        un = -np.sum(A * Z)
        pair = 0.5 * 0.8 * sum(W[p, q] * np.sum((Z[p] - Z[q]) ** 2) for p, q in zip(*np.nonzero(W)))
        assert E == pytest.approx(un + pair, rel=1e-12)
        assert E == pytest.approx(un + 0.8 * np.trace(Z.T @ Lap @ Z), rel=1e-12)      # Eq. (1) = Eq. (3)
        # identity (3): tr(Z'LZ) = sum_p d_p - sum_pq k z_p.z_q for binary Z
        assert np.trace(Z.T @ Lap @ Z) == pytest.approx(W.sum() - np.sum(W * (Z @ Z.T)))
        # diagonal shift: the self terms ||z_p - z_p||^2 vanish, E unchanged (footnote to Prop. 1)
        Wd = W + 3.0 * np.eye(inst.N)
        Lap_d = np.diag(Wd.sum(axis=1)) - Wd
        assert np.trace(Z.T @ Lap_d @ Z) == pytest.approx(np.trace(Z.T @ Lap @ Z))


def test_relaxed_equals_discrete_at_vertices(small):
    # at one-hot Z the entropy vanishes and R = E with lambda halved, minus (lambda/2) sum d_p
    inst, (_i, _d, rp, ci, s2) = small
    A = slk.unary(inst.X, inst.init_modes, s2)
    W = slk.csr_matrix(rp, ci, inst.N)
    lab = np.argmax(A, axis=1)
    Z = np.eye(inst.L)[lab]
    R = slk.relaxed_bound(Z, A, slk.pairwise(W, Z), 1.0)
    E_half, _ = slk.energy(A, lab, rp, ci, 0.5)
    assert R == pytest.approx(E_half - 0.5 * len(ci), rel=1e-12)


# ---------------------------------------------------------------- T4 / T10: modes and brute force

def test_modes_are_points_and_logodds(small):
    inst, (_i, _d, rp, ci, s2) = small
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 1.0)
    m = out["modes_next"]
    assert np.all((m >= 0) & (m < inst.N))
    Z, V = out["Z"], out["V"]
    ok = (Z > 1e-12) & (Z < 1 - 1e-9)
    np.testing.assert_allclose(V[ok], np.log(Z[ok] / (1 - Z[ok])), rtol=1e-6, atol=1e-6)
    for l in range(inst.L):
        assert m[l] in out["ties"][l]
        assert V[m[l], l] == V[:, l].max()
        # Eq. (11) on z itself agrees wherever z has not saturated at the top
        top = Z[:, l].max()
        if top < 1 - 1e-9:
            assert Z[m[l], l] == top


def _tiny_separable():
    # two tight, far-apart groups; kNN edges stay inside each group
    X = np.array([[0, 0], [0.3, 0], [0, 0.3], [0.2, 0.2], [8, 8], [8.3, 8], [8, 8.3], [8.2, 8.25]],
                 dtype=np.float32)
    idx, d2 = slk.knn(X, 2)
    rp, ci = slk.symmetrize(idx, len(X))
    return X, rp, ci, slk.sigma2_from_knn(d2)


def test_bruteforce_separable_reaches_minimum():
    X, rp, ci, s2 = _tiny_separable()
    E_min, lab_min, _ = brute.minimise(X, rp, ci, 2, s2, 1.0)
    out = slk.fit(X, rp, ci, np.array([0, 7]), s2, 1.0)
    G = brute.gram(X, s2)
    E_slk, _ = brute.energy_def(G, rp, ci, out["labels"], 2, 1.0)
    assert E_slk == pytest.approx(E_min, rel=1e-12)
    assert brute.canonical(out["labels"]) == brute.canonical(lab_min)


def test_bruteforce_lower_bounds_slk():
    rng = np.random.default_rng(5)
    for trial in range(4):
        X = rng.normal(size=(7, 2)).astype(np.float32)
        idx, d2 = slk.knn(X, 2)
        rp, ci = slk.symmetrize(idx, 7)
        s2 = slk.sigma2_from_knn(d2)
        L = 3
        E_min, _, _ = brute.minimise(X, rp, ci, L, s2, 0.5)
        out = slk.fit(X, rp, ci, rng.choice(7, L, replace=False), s2, 0.5)
        E_slk, _ = brute.energy_def(brute.gram(X, s2), rp, ci, out["labels"], L, 0.5)
        assert E_slk >= E_min - 1e-12


def test_bruteforce_definition_mode_matches_kde_argmax():
    X, rp, ci, s2 = _tiny_separable()
    G = brute.gram(X, s2)
    lab = [0, 0, 0, 0, 1, 1, 1, 1]
    m = brute.modes_by_definition(G, lab, 2)
    dens0 = [sum(math.exp(-np.sum((X[p].astype(float) - X[y].astype(float)) ** 2) / (2 * s2)) for p in range(4))
             for y in range(8)]
    assert m[0] == int(np.argmax(dens0))


# ---------------------------------------------------------------- T11 / T12: special cases

def test_lambda_zero_is_kernel_kmodes(small):
    inst, (_i, _d, rp, ci, s2) = small
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 0.0)
    X = inst.X.astype(np.float64)
    nearest = np.argmin(cdist(X, X[inst.init_modes], "sqeuclidean"), axis=1)
    assert np.array_equal(out["labels"], nearest)
    assert out["n_pass"] == 2                       # a fixed point after one update
    np.testing.assert_allclose(out["Z"], slk.softmax_rows(out["A"]), rtol=1e-15)


def test_empty_graph_equals_lambda_zero(small):
    inst, (_i, _d, _rp, _ci, s2) = small
    rp0 = np.zeros(inst.N + 1, dtype=np.int64)
    ci0 = np.zeros(0, dtype=np.int64)
    a = slk.assign(inst.X, rp0, ci0, inst.init_modes, s2, 2.0)
    b = slk.assign(inst.X, rp0, ci0, inst.init_modes, s2, 0.0)
    assert np.array_equal(a["Z"], b["Z"]) and a["E"] == b["E"]


def test_single_cluster(small):
    inst, (_i, _d, rp, ci, s2) = small
    out = slk.assign(inst.X, rp, ci, inst.init_modes[:1], s2, 1.0)
    assert np.all(out["Z"] == 1.0)
    assert out["modes_next"][0] == 0
    assert out["cut"] == 0 and out["E"] == pytest.approx(-out["A"][:, 0].sum(), rel=1e-14)


def test_huge_bandwidth_unary_is_flat(small):
    inst, (_i, _d, rp, ci, _s2) = small
    A = slk.unary(inst.X, inst.init_modes, 1e30)
    assert np.all(A == 1.0)


def test_mode_permutation_permutes_columns(small):
    inst, (_i, _d, rp, ci, s2) = small
    perm = np.array([2, 0, 3, 1])
    a = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 1.0, n_inner=6)
    b = slk.assign(inst.X, rp, ci, inst.init_modes[perm], s2, 1.0, n_inner=6)
    np.testing.assert_allclose(b["Z"], a["Z"][:, perm], rtol=1e-12, atol=1e-15)


def test_fit_mixture2k_converges():
    inst = gen.make("mixture-2k")
    idx, d2, rp, ci, s2 = graph(inst)
    out = slk.fit(inst.X, rp, ci, inst.init_modes, s2, inst.lam)
    assert out["converged"] and out["outer_iters"] < 20
    assert np.allclose(out["Z"].sum(axis=1), 1.0, atol=1e-12)
    assert len(np.unique(out["modes"])) == inst.L


# ---------------------------------------------------------------- R10: the inner stop rule

def _sigmoid(t):
    return 1.0 / (1.0 + math.exp(-t))


def _two_point_bounds(alpha, lam, c, passes):
    """Relaxed bound R(Z^0), R(Z^1), ... of a two-point instance, derived by hand.

    Two points joined by one edge, L = 2, and the same unary row a_p = (alpha + c, c) for both.
    By symmetry both rows stay equal, z_p = (u, 1 - u); b_p = z_q gives the logits
    s_p = (alpha + c + lam u, c + lam (1 - u)), so Eq. (8) is the scalar map
    u <- sigmoid(alpha + lam (2u - 1)) from u = sigmoid(alpha) (Z^0 = softmax(a)).  Summed over the
    two points, z_p.log z_p - z_p.a_p - (lam/2) z_p.b_p is
        R(u) = 2 [u log u + (1 - u) log(1 - u) - alpha u - c - (lam/2) (u^2 + (1 - u)^2)].
    The shift c moves every R by -2c and leaves the iterates unchanged."""
    u = _sigmoid(alpha)
    out = []
    for _ in range(passes):
        h = u * math.log(u) + (1.0 - u) * math.log(1.0 - u)
        out.append(2.0 * (h - alpha * u - c - 0.5 * lam * (u * u + (1.0 - u) ** 2)))
        u = _sigmoid(alpha + lam * (2.0 * u - 1.0))
    return out


def _stop_pass(R, tol, rule):
    """Passes run under a stop rule, from the bound trace R: 'rel' is reading R10 (relative change
    between the bounds of consecutive input iterates); 'abs' an absolute change; 'out' the change
    between the bounds of consecutive output iterates (one pass earlier).  Also returns the margin:
    how far the deciding change lies below tol, and the previous one above it."""
    for i in range(1, len(R) - 1):
        if rule == "rel":
            num, den = abs(R[i] - R[i - 1]), tol * abs(R[i - 1])
        elif rule == "abs":
            num, den = abs(R[i] - R[i - 1]), tol
        else:
            num, den = abs(R[i + 1] - R[i]), tol * abs(R[i])
        if num <= den:
            margin = den / max(num, 1e-300)
            if rule == "rel" and i >= 2:
                margin = min(margin, abs(R[i - 1] - R[i - 2]) / (tol * abs(R[i - 2])))
            return i + 1, margin
    raise AssertionError("no stop within the trace")


R10_CASES = [(0.3, 1.0, 0.0, 3e-8), (0.3, 1.0, 1000.0, 3e-8)]


def _two_point_assign(alpha, lam, c, tol):
    A = np.array([[alpha + c, c], [alpha + c, c]])
    rp, ci = np.array([0, 1, 2]), np.array([1, 0])
    return slk.assign(np.zeros((2, 1)), rp, ci, np.array([0, 1]), 1.0, lam, tol=tol, A=A)


def test_r10_two_point_trace_and_stop():
    """The oracle's bound trace equals the hand-derived one, and it stops at the pass the relative
    rule gives: 10 passes unshifted, 6 with the bound shifted by -2000 (the same iterates)."""
    for alpha, lam, c, tol in R10_CASES:
        out = _two_point_assign(alpha, lam, c, tol)
        R = _two_point_bounds(alpha, lam, c, 40)
        n, margin = _stop_pass(R, tol, "rel")
        assert margin >= 1.3, "the case sits too close to the threshold"
        assert out["n_pass"] == n
        np.testing.assert_allclose(out["R_trace"], R[:n], rtol=1e-13, atol=1e-13)
        u = np.full(2, _sigmoid(alpha))
        for _ in range(n):
            u = np.array([_sigmoid(alpha + lam * (2 * u[0] - 1))] * 2)
        np.testing.assert_allclose(out["Z"][:, 0], u, rtol=1e-14)
    assert [_two_point_assign(*cs)["n_pass"] for cs in R10_CASES] == [10, 6]


def test_r10_cases_tell_the_rules_apart():
    """Under an absolute rule both cases would stop together (11 passes); under a rule on the
    output iterates' bounds each would stop one pass earlier (9 and 5)."""
    got = {rule: [_stop_pass(_two_point_bounds(a, l, c, 40), t, rule)[0] for a, l, c, t in R10_CASES]
           for rule in ("rel", "abs", "out")}
    assert got == {"rel": [10, 6], "abs": [11, 11], "out": [9, 5]}


def test_planted_absolute_stop_rule_is_caught(monkeypatch):
    monkeypatch.setattr(slk, "inner_settled", lambda r0, r1, tol: abs(r1 - r0) <= tol)
    assert [_two_point_assign(*cs)["n_pass"] for cs in R10_CASES] != [10, 6]


def test_planted_output_bound_rule_is_caught(monkeypatch):
    # the trace records the bound of each pass's output instead of its input
    orig = slk.relaxed_bound

    def out_bound(Z, A, B, lam, scale=1.0):
        Zn = slk.softmax_rows(A + scale * lam * B)
        W = slk.csr_matrix(np.array([0, 1, 2]), np.array([1, 0]), 2)
        return orig(Zn, A, slk.pairwise(W, Zn), lam, scale)

    monkeypatch.setattr(slk, "relaxed_bound", out_bound)
    assert [_two_point_assign(*cs)["n_pass"] for cs in R10_CASES] != [10, 6]


# ---------------------------------------------------------------- planted mistakes are caught

def test_planted_factor_two_breaks_monotonicity(small, monkeypatch):
    inst, (_i, _d, rp, ci, s2) = small
    dmax = float(np.max(np.diff(rp)))
    # bound with the wrong factor (lambda instead of lambda/2) for the printed update
    orig = slk.bound_rows
    monkeypatch.setattr(slk, "bound_rows", lambda Z, A, B, lam, scale=1.0: orig(Z, A, B, lam, 2.0))
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 1.0, delta=0.0, n_inner=25)
    B = slk.pairwise(slk.csr_matrix(rp, ci, inst.N), out["Z_in"])
    tight = slk.aux_value(out["Z_in"], out["S"], out["Z_in"], B, 1.0)
    # the tightness pin A_i(Z^i) = R(Z^i) of the bound test no longer holds
    assert not np.isclose(tight, out["R_trace"][-1], rtol=1e-9)


def test_planted_sign_error_in_unary_fails_kkt_pin(small, monkeypatch):
    inst, (*_g, s2) = small
    monkeypatch.setattr(slk, "gaussian", lambda d2, sigma2: np.exp(np.asarray(d2) / (2.0 * sigma2)))
    A = slk.unary(inst.X, inst.init_modes, s2)
    X = inst.X.astype(np.float64)
    ref = np.exp(-cdist(X, X[inst.init_modes], "sqeuclidean") / (2 * s2))
    assert not np.allclose(A, ref)


def test_planted_transposed_affinity_fails_dense_or(small, monkeypatch):
    inst, (idx, *_r) = small
    def one_sided(knn_idx, N):
        K = knn_idx.shape[1]
        p = np.repeat(np.arange(N), K)
        keys = np.unique(p * N + knn_idx.ravel())
        rp = np.zeros(N + 1, dtype=np.int64)
        np.cumsum(np.bincount(keys // N, minlength=N), out=rp[1:])
        return rp, keys % N
    rp, ci = one_sided(idx, inst.N)
    W = slk.csr_matrix(rp, ci, inst.N).toarray()
    assert not np.array_equal(W, W.T)      # the symmetry pin would fail


def test_planted_argmin_mode_fails_membership(small):
    inst, (_i, _d, rp, ci, s2) = small
    out = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 1.0)
    wrong = np.argmin(out["V"], axis=0)
    assert any(wrong[l] not in out["ties"][l] for l in range(inst.L))


# ---------------------------------------------------------------- the row-block driver of the full-size tests

@pytest.mark.parametrize("delta,scale", [(0.0, 1.0), (2.0, 2.0)])
def test_row_block_assign_equals_oracle(small, delta, scale):
    import par_oracle
    inst, (_i, _d, rp, ci, s2) = small
    pool = par_oracle.RowPool(threads=3)
    try:
        a = par_oracle.assign(pool, inst.X, rp, ci, inst.init_modes, s2, 0.9, 7, delta=delta, scale=scale)
    finally:
        pool.close()
    b = slk.assign(inst.X, rp, ci, inst.init_modes, s2, 0.9, n_inner=7, delta=delta, scale=scale)
    for k in ("Z", "Z_in", "S", "A", "labels", "modes_next", "V"):
        assert np.array_equal(a[k], b[k]), k
    assert a["R_trace"] == b["R_trace"] and a["E"] == b["E"] and a["cut"] == b["cut"]
    assert all(np.array_equal(x, y) for x, y in zip(a["ties"], b["ties"]))
