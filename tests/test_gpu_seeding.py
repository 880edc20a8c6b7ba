"""K-means++ seeding and exact modes on the GPU (slk_kmeanspp, slk_dense_modes) against the FP64
oracle (oracle/seeding.py).

Bars.  K-means++: D^2 bit-identical (the same fixed-order FP64 sums), the nearest-seed labels
bit-identical, and the centres identical wherever the oracle's target lies more than 2^-40 of
the total away from every prefix boundary (the prefix sums are formed in another order).
Exact modes: the density P within a derived bound of the oracle's, and each mode inside the
oracle's near-tie set under that bound (equal wherever the best is unique by more than it).

Density bound.  The squared distance comes from a centred bf16 hi + lo split with FP32
accumulation: |error| <= 2^-14 (n_p + n_y) with n the centred squared norms, which moves
k = exp(-d^2 / 2 sigma^2) by a relative 2^-14 (n_p + n_y) / (2 sigma^2).  Splitting k and z
into bf16 hi + lo and the FP32 accumulation add at most 2e-5 relative, so
|P_gpu - P| <= (2^-14 max(n_p + n_y) / (2 sigma^2) + 2e-5) P_row_max + 1e-30.  For bf16 points
the Gram product is exact up to FP32 accumulation over the uncentred norms: 2^-20 (n_p + n_y)."""
import numpy as np
import pytest

import gen
from oracle import seeding
from test_gpu_parity import _say, round_bf16, to_dev

pytestmark = pytest.mark.gpu


def uniforms(L, seed):
    return np.random.default_rng(seed).random(L)


# ------------------------------------------------------------------- K-means++

KPP_CASES = [(2000, 16, 5, 1), (1001, 9, 7, 2), (37, 3, 3, 3), (5000, 130, 20, 4), (300, 4, 1, 5),
             (20000, 64, 50, 6), (257, 33, 64, 7)]


def check_kpp(slk, torch, X, L, u, prec="fp32"):
    Xo = round_bf16(X) if prec == "bf16" else X
    cent, lab, d2 = slk.kmeanspp(to_dev(torch, X, torch.float32), L, u, prec=prec)
    ref, rd2 = seeding.kmeanspp(Xo, L, u)
    margin = seeding.kmeanspp_margin(Xo, ref, u)
    assert np.all(margin > 2.0 ** -40), margin.min()
    assert np.array_equal(cent, ref)
    assert np.array_equal(d2.cpu().numpy(), rd2)
    assert np.array_equal(lab.cpu().numpy(), seeding.nearest_labels(Xo, ref))
    return cent


@pytest.mark.parametrize("n,d,L,seed", KPP_CASES)
def test_kmeanspp_matches_oracle(slk, torch, n, d, L, seed):
    inst = gen.gaussian_mixture(n=n, d=d, L=min(L, 8), K=5, seed=seed)
    cent = check_kpp(slk, torch, inst.X, L, uniforms(L, seed))
    _say(f"[kmeans++] n={n} d={d} L={L}: centres {cent[:6].tolist()}...")


def test_kmeanspp_bf16_points(slk, torch):
    inst = gen.gaussian_mixture(n=3000, d=24, L=6, K=5, seed=11)
    check_kpp(slk, torch, inst.X, 12, uniforms(12, 11), prec="bf16")


def test_kmeanspp_edge_uniforms(slk, torch):
    X = gen.gaussian_mixture(n=500, d=6, L=3, K=5, seed=12).X
    x = to_dev(torch, X, torch.float32)
    cent, _, _ = slk.kmeanspp(x, 6, np.zeros(6))
    assert cent.tolist() == list(range(6))
    cent, _, _ = slk.kmeanspp(x, 4, np.full(4, 1.0 - 2.0 ** -53))
    assert cent.tolist() == [499, 498, 497, 496]


def test_kmeanspp_coincident_points_fall_back_to_uniform(slk, torch):
    X = np.full((40, 5), 3.0, dtype=np.float32)
    u = np.array([0.1, 0.6, 0.99, 0.0])
    cent, lab, d2 = slk.kmeanspp(to_dev(torch, X, torch.float32), 4, u)
    assert cent.tolist() == seeding.kmeanspp(X, 4, u)[0].tolist() == [4, 24, 39, 0]
    assert np.all(d2.cpu().numpy() == 0) and np.all(lab.cpu().numpy() == 0)


def test_kmeanspp_duplicates_are_not_repeated(slk, torch):
    rng = np.random.default_rng(13)
    base = np.unique(rng.integers(-5, 6, size=(40, 3)), axis=0).astype(np.float32)
    X = np.vstack([base, base[:20], base[:20]])
    for trial in range(3):
        u = rng.random(len(base))
        cent = check_kpp(slk, torch, X, len(base), u)
        assert len({tuple(X[i]) for i in cent}) == len(base)


def test_kmeanspp_rejects_bad_arguments(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    x = to_dev(torch, np.zeros((10, 2), np.float32), torch.float32)
    with pytest.raises(SlkError):
        slk.kmeanspp(x, 2, np.array([0.5, 1.0]))
    with pytest.raises(SlkError):
        slk.kmeanspp(x, 11, np.zeros(11))


# ------------------------------------------------------------------- exact modes

def density_bound(X, sigma2, prec):
    X64 = np.asarray(X, dtype=np.float64)
    if prec == "bf16":
        X64 = round_bf16(X).astype(np.float64)
        nmax = (X64 ** 2).sum(axis=1).max()
        return 2.0 ** -20 * 2 * nmax / (2 * sigma2) + 2e-5
    Y = X64 - X64.mean(axis=0)
    nmax = (Y ** 2).sum(axis=1).max()
    return 2.0 ** -14 * 2 * nmax / (2 * sigma2) + 2e-5


def check_modes(modes, dens, P, rel):
    """dens within rel * column max of P; each mode inside the near-tie set; modes equal where
    the oracle's best is unique by more than twice the bound."""
    colmax = P.max(axis=0)
    err = np.abs(dens - P).max(axis=0) / colmax
    assert np.all(err <= rel), (err.max(), rel)
    L = P.shape[1]
    srt = np.sort(P, axis=0)
    for l in range(L):
        slack = 2 * rel * colmax[l]
        assert P[modes[l], l] >= colmax[l] - slack, (l, modes[l], P[modes[l], l], colmax[l])
        if L and srt[-1, l] - srt[-2, l] > slack:
            assert modes[l] == np.argmax(P[:, l])
    return err.max()


DM_CASES = [
    ("hard-16", dict(n=1500, d=16, L=5, seed=21), "hard", "fp32"),
    ("soft-ragged", dict(n=1001, d=9, L=7, seed=22), "soft", "fp32"),
    ("wide-d-L40", dict(n=700, d=130, L=40, seed=23), "soft", "fp32"),
    ("tiny", dict(n=37, d=3, L=3, seed=24), "soft", "fp32"),
    ("L64-hard", dict(n=2000, d=64, L=64, seed=25), "hard", "fp32"),
    ("d128-L33", dict(n=1300, d=128, L=33, seed=26), "soft", "fp32"),
    ("bf16-hard", dict(n=1200, d=20, L=6, seed=27), "hard", "bf16"),
    ("bf16-soft-wide", dict(n=900, d=200, L=9, seed=28), "soft", "bf16"),
    ("L1", dict(n=500, d=5, L=1, seed=29), "soft", "fp32"),
    ("d784-hard", dict(n=600, d=784, L=10, seed=30), "hard", "fp32"),
]


@pytest.mark.parametrize("name,kw,kind,prec", DM_CASES)
def test_dense_modes_match_oracle(slk, torch, name, kw, kind, prec):
    inst = gen.gaussian_mixture(n=kw["n"], d=kw["d"], L=min(kw["L"], 8), K=5, seed=kw["seed"])
    L = kw["L"]
    rng = np.random.default_rng(kw["seed"])
    X = inst.X
    x = to_dev(torch, X, torch.float32)
    s2 = 2.0 * kw["d"]
    if kind == "hard":
        lab = rng.integers(0, L, inst.N).astype(np.int32)
        modes, best, dens = slk.dense_modes(x, L, s2, labels=to_dev(torch, lab, torch.int32), prec=prec, density=True)
        Z = np.eye(L)[lab]
    else:
        Z = rng.dirichlet(np.ones(L), size=inst.N).astype(np.float32)
        modes, best, dens = slk.dense_modes(x, L, s2, z=to_dev(torch, Z, torch.float32), prec=prec, density=True)
    Xo = round_bf16(X) if prec == "bf16" else X
    ref, P = seeding.dense_modes(Xo, Z.astype(np.float64), s2)
    rel = density_bound(X, s2, prec)
    err = check_modes(modes, dens.cpu().numpy(), P, rel)
    assert np.allclose(best, dens.cpu().numpy()[modes, np.arange(L)])
    _say(f"[dense modes] {name}: max rel err {err:.2e} (bound {rel:.2e}), equal {np.mean(modes == ref):.3f}")


def test_dense_modes_proximal_term(slk, torch):
    inst = gen.gaussian_mixture(n=1200, d=12, L=6, K=5, seed=31)
    x = to_dev(torch, inst.X, torch.float32)
    rng = np.random.default_rng(31)
    Z = rng.dirichlet(np.ones(6), size=inst.N).astype(np.float32) * 0.05
    prev = rng.choice(inst.N, 6, replace=False)
    s2 = 20.0
    modes, _, dens = slk.dense_modes(x, 6, s2, z=to_dev(torch, Z, torch.float32), prev=prev, density=True)
    ref, P = seeding.dense_modes(inst.X, Z.astype(np.float64), s2, prev=prev)
    check_modes(modes, dens.cpu().numpy(), P, density_bound(inst.X, s2, "fp32"))


def test_dense_modes_empty_cluster(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    inst = gen.gaussian_mixture(n=600, d=5, L=3, K=5, seed=32)
    x = to_dev(torch, inst.X, torch.float32)
    lab = np.where(inst.labels_true == 2, 0, inst.labels_true).astype(np.int32)   # cluster 2 empty
    keep = [0, 1, 577]
    modes, _, _ = slk.dense_modes(x, 3, 10.0, labels=to_dev(torch, lab, torch.int32), keep=keep)
    ref, _ = seeding.dense_modes(inst.X, np.eye(3)[lab], 10.0, keep=keep)
    assert modes[2] == 577 and modes[2] == ref[2]
    with pytest.raises(SlkError):
        slk.dense_modes(x, 3, 10.0, labels=to_dev(torch, lab, torch.int32))
    # Eq. (10): a cluster with no weight keeps its previous mode
    prev = [5, 6, 321]
    modes, _, _ = slk.dense_modes(x, 3, 10.0, labels=to_dev(torch, lab, torch.int32), prev=prev)
    ref, _ = seeding.dense_modes(inst.X, np.eye(3)[lab], 10.0, prev=prev)
    assert modes[2] == 321 == ref[2]
    assert np.array_equal(modes[:2], ref[:2])


def test_dense_modes_larger_ragged(slk, torch):
    """Many tiles and work-groups with a ragged tail: 8,229 points (the oracle's density matrix
    in full)."""
    inst = gen.gaussian_mixture(n=8229, d=48, L=12, K=5, seed=33)
    x = to_dev(torch, inst.X, torch.float32)
    lab = inst.labels_true.astype(np.int32)
    s2 = 60.0
    modes, _, dens = slk.dense_modes(x, 12, s2, labels=to_dev(torch, lab, torch.int32), density=True)
    ref, P = seeding.dense_modes(inst.X, np.eye(12)[lab], s2)
    err = check_modes(modes, dens.cpu().numpy(), P, density_bound(inst.X, s2, "fp32"))
    _say(f"[dense modes] 8229x48 L=12: max rel err {err:.2e}, equal {np.mean(modes == ref):.3f}")


def test_initial_modes_pipeline(slk, torch):
    inst = gen.gaussian_mixture(n=3000, d=16, L=5, K=10, seed=34)
    u = uniforms(5, 34)
    s2 = 13.5
    out = slk.initial_modes(to_dev(torch, inst.X, torch.float32), 5, u, s2)
    ref = seeding.initial_modes(inst.X, 5, u, s2)
    assert np.array_equal(out["seeds"], ref["seeds"])
    assert np.array_equal(out["labels"].cpu().numpy(), ref["labels"])
    check_modes(out["modes"], ref["P"], ref["P"], density_bound(inst.X, s2, "fp32"))


def test_dense_modes_rejects_bad_arguments(slk, torch):
    from paper_1810_13044_amd._lib import SlkError
    x = to_dev(torch, np.random.default_rng(0).normal(size=(50, 3)).astype(np.float32), torch.float32)
    lab = torch.zeros(50, dtype=torch.int32, device="cuda")
    with pytest.raises(SlkError):
        slk.dense_modes(x, 65, 1.0, labels=lab)
    with pytest.raises(SlkError):
        slk.dense_modes(x, 2, 0.0, labels=lab, keep=[0, 1])
    with pytest.raises(SlkError):
        slk.dense_modes(x, 2, 1.0, labels=lab, prev=[0, 50])
