"""Seeded synthetic inputs shaped like the workloads of Scalable Laplacian K-modes.

This module is shared by the oracle-side tests and by the GPU-side tests and
benchmark.  It draws data only: it holds none of the clustering method's
arithmetic (no distances, kernels, graphs, softmax or bounds).

The paper's datasets (Table 1: MNIST variants, LabelMe, YTF, Shuttle, Reuters)
are not available, so each workload below is a seeded stand-in with the shape
of one regime of Table 1.  Every generator draws with
``numpy.random.default_rng(seed)`` in a fixed order: cluster centres, cluster
parameters, labels, noise, then the initial modes (distinct point indices, the
stand-in for the paper's seeding of Section 4.2).

Points are emitted in a random order (cluster labels are shuffled), as a real
dataset would be; any locality ordering is the library's job.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = [
    "Instance", "mixture", "gaussian_mixture", "star_hubs", "manifold_images", "vmf_embeddings",
    "anisotropic_mixture", "job_stream", "init_modes", "make", "WORKLOADS",
]


@dataclass
class Instance:
    """One clustering problem: points, cluster count and the run parameters."""
    name: str
    X: np.ndarray              # N x D float32, row-major
    L: int                     # number of clusters
    K: int                     # neighbours per point for the kNN affinity
    lam: float                 # Laplacian weight lambda
    init_modes: np.ndarray     # L distinct int32 point indices
    labels_true: np.ndarray    # generating component of every point (int32)
    seed: int
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def D(self) -> int:
        return int(self.X.shape[1])


def init_modes(rng: np.random.Generator, n: int, L: int) -> np.ndarray:
    """L distinct point indices, drawn after all data draws."""
    return rng.choice(n, L, replace=False).astype(np.int32)


def _equal_labels(rng: np.random.Generator, n: int, L: int) -> np.ndarray:
    """Exactly floor/ceil(n/L) points per cluster, in a shuffled order."""
    lab = np.arange(n, dtype=np.int64) % L
    rng.shuffle(lab)
    return lab


def _sizes_labels(rng: np.random.Generator, sizes: np.ndarray) -> np.ndarray:
    lab = np.repeat(np.arange(len(sizes), dtype=np.int64), sizes)
    rng.shuffle(lab)
    return lab


def gaussian_mixture(n: int = 2000, d: int = 16, L: int = 5, K: int = 10, lam: float = 1.0,
                     seed: int = 0, box: float = 10.0, noise: float = 1.0,
                     name: str = "mixture") -> Instance:
    """Isotropic Gaussian mixture: centres U[-box, box]^d, N(0, noise^2 I) noise,
    equal cluster weights.  With the defaults this is the 2,000 x 16, L=5 case."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(L, d))
    lab = _equal_labels(rng, n, L)
    eps = rng.standard_normal((n, d)) * noise
    X = (centres[lab] + eps).astype(np.float32)
    modes = init_modes(rng, n, L)
    return Instance(name, X, L, K, lam, modes, lab.astype(np.int32), seed)


# the short name used by tests for arbitrary small mixtures
mixture = gaussian_mixture


def star_hubs(n_background: int = 2000, d: int = 64, L: int = 5, K: int = 10, lam: float = 1.0,
              hub_sizes=(140, 300, 700, 1500), seed: int = 11, name: str = "hubs") -> Instance:
    """A Gaussian mixture (as `gaussian_mixture`) plus star-shaped groups far from it: a
    centre point and m points at distance exactly 1 from it in random directions.  In 64
    dimensions points on the unit sphere are almost never within 1 of each other, so every
    star point has its centre among its nearest neighbours and the centre's row of the
    symmetrised kNN graph has about m entries: hubs of chosen degree.  Star points get the
    label L - 1; the rows are shuffled."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10.0, 10.0, size=(L, d))
    blab = _equal_labels(rng, n_background, L)
    bg = centres[blab] + rng.standard_normal((n_background, d))
    parts, labs = [bg], [blab]
    for h, m in enumerate(hub_sizes):
        c = np.full(d, 100.0 + 10.0 * h)
        u = rng.standard_normal((m, d))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        parts += [c[None, :], c + u]
        labs += [np.full(m + 1, L - 1)]
    X = np.concatenate(parts)
    lab = np.concatenate(labs)
    order = rng.permutation(len(X))
    X, lab = X[order].astype(np.float32), lab[order]
    modes = init_modes(rng, len(X), L)
    return Instance(name, X, L, K, lam, modes, lab.astype(np.int32), seed)


def manifold_images(n: int = 70000, d: int = 784, L: int = 10, K: int = 5, lam: float = 1.0,
                    seed: int = 1, dim: int = 10, scale: float = 1.5, noise: float = 0.05,
                    name: str = "images") -> Instance:
    """Image-like data: cluster l is x = mu_l + scale * Q_l t + eps with mu_l ~ U[0.25, 0.75]^d,
    Q_l an orthonormal d x dim basis (QR of a Gaussian matrix), t ~ U[-1, 1]^dim and
    eps ~ N(0, noise^2); clipped to [0, 1] and quantised to multiples of 1/255 (uint8 codes)."""
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.25, 0.75, size=(L, d))
    Q = np.empty((L, d, dim))
    for l in range(L):
        q, _ = np.linalg.qr(rng.standard_normal((d, dim)))
        Q[l] = q
    lab = _equal_labels(rng, n, L)
    t = rng.uniform(-1.0, 1.0, size=(n, dim))
    eps = rng.standard_normal((n, d)) * noise
    X = np.empty((n, d))
    for l in range(L):
        idx = np.nonzero(lab == l)[0]
        X[idx] = mu[l] + scale * (t[idx] @ Q[l].T) + eps[idx]
    codes = np.rint(np.clip(X, 0.0, 1.0) * 255.0).astype(np.uint8)
    Xf = (codes.astype(np.float32) / np.float32(255.0)).astype(np.float32)
    modes = init_modes(rng, n, L)
    return Instance(name, Xf, L, K, lam, modes, lab.astype(np.int32), seed, {"codes": codes})


def _zipf_sizes(n: int, L: int, s: float) -> np.ndarray:
    """Deterministic cluster sizes proportional to l^-s, largest-remainder rounding to n."""
    w = np.arange(1, L + 1, dtype=np.float64) ** (-s)
    raw = w / w.sum() * n
    sizes = np.floor(raw).astype(np.int64)
    rem = n - int(sizes.sum())
    order = np.argsort(-(raw - sizes), kind="stable")
    sizes[order[:rem]] += 1
    return sizes


def _vmf_cosines(rng: np.random.Generator, kappa: float, m: int, count: int) -> np.ndarray:
    """Wood (1994) rejection sampler for the cosine w = <x, mu> of a von Mises-Fisher draw."""
    b = (-2.0 * kappa + np.sqrt(4.0 * kappa * kappa + (m - 1.0) ** 2)) / (m - 1.0)
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + (m - 1.0) * np.log(1.0 - x0 * x0)
    out = np.empty(count)
    filled = 0
    while filled < count:
        k = max(16, 2 * (count - filled))
        z = rng.beta((m - 1.0) / 2.0, (m - 1.0) / 2.0, size=k)
        u = rng.uniform(size=k)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        ok = kappa * w + (m - 1.0) * np.log(1.0 - x0 * w) - c >= np.log(u)
        acc = w[ok][: count - filled]
        out[filled: filled + len(acc)] = acc
        filled += len(acc)
    return out


def vmf_embeddings(n: int = 100000, d: int = 4096, L: int = 40, K: int = 10, lam: float = 1.0,
                   seed: int = 2, kappa: float = 50.0, zipf: float = 1.1,
                   name: str = "embeddings") -> Instance:
    """Unit-norm embeddings: L von Mises-Fisher clusters (mean directions uniform on the
    sphere, concentration kappa) with Zipf(zipf) cluster sizes."""
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal((L, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    sizes = _zipf_sizes(n, L, zipf)
    lab = _sizes_labels(rng, sizes)
    X = np.empty((n, d), dtype=np.float32)
    for l in range(L):
        idx = np.nonzero(lab == l)[0]
        w = _vmf_cosines(rng, kappa, d, len(idx))
        v = rng.standard_normal((len(idx), d))
        v -= np.outer(v @ mu[l], mu[l])
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        X[idx] = (w[:, None] * mu[l][None, :] + np.sqrt(1.0 - w * w)[:, None] * v).astype(np.float32)
    modes = init_modes(rng, n, L)
    return Instance(name, X, L, K, lam, modes, lab.astype(np.int32), seed, {"sizes": sizes})


def anisotropic_mixture(n: int = 1_000_000, d: int = 128, L: int = 50, K: int = 10,
                        lam: float = 1.0, seed: int = 3, box: float = 10.0,
                        eig_lo: float = 0.2, eig_hi: float = 2.0,
                        name: str = "large") -> Instance:
    """Gaussian mixture with per-cluster covariance Q_l diag(e_l) Q_l^T, e_l ~ U[eig_lo, eig_hi]^d
    and Q_l Haar-distributed (sign-fixed QR); centres U[-box, box]^d, equal weights."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(L, d))
    eig = rng.uniform(eig_lo, eig_hi, size=(L, d))
    Q = np.empty((L, d, d))
    for l in range(L):
        q, r = np.linalg.qr(rng.standard_normal((d, d)))
        Q[l] = q * np.sign(np.diag(r))[None, :]
    lab = _equal_labels(rng, n, L)
    X = np.empty((n, d), dtype=np.float32)
    chunk = 1 << 18
    for s in range(0, n, chunk):
        g = rng.standard_normal((min(chunk, n - s), d))
        lc = lab[s: s + len(g)]
        out = np.empty_like(g)
        for l in np.unique(lc):
            m = lc == l
            out[m] = centres[l] + (g[m] * np.sqrt(eig[l])[None, :]) @ Q[l].T
        X[s: s + len(g)] = out.astype(np.float32)
    modes = init_modes(rng, n, L)
    return Instance(name, X, L, K, lam, modes, lab.astype(np.int32), seed)


@dataclass
class Job:
    job_id: int
    arrival_s: float
    instance: Instance


def job_stream(n_jobs: int = 2000, rate: float = 200.0, seed: int = 5,
               n_lo: int = 500, n_hi: int = 50000, dims=(64, 128, 256),
               L_lo: int = 5, L_hi: int = 50, K: int = 10, lam: float = 1.0):
    """Poisson stream of independent clustering jobs: exponential inter-arrival gaps at
    `rate` jobs/s; N log-uniform in [n_lo, n_hi]; D uniform on `dims`; L uniform on
    [L_lo, L_hi]; each job's data is an isotropic mixture seeded with 10000 + job id.
    Returns a list of (job_id, arrival_s, n, d, L, seed) tuples; `materialise` builds one."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_jobs)
    arr = np.cumsum(gaps)
    ns = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=n_jobs))).astype(np.int64)
    ds = rng.choice(np.asarray(dims), size=n_jobs)
    Ls = rng.integers(L_lo, L_hi + 1, size=n_jobs)
    return [(j, float(arr[j]), int(ns[j]), int(ds[j]), int(Ls[j]), 10000 + j) for j in range(n_jobs)]


def materialise(spec, K: int = 10, lam: float = 1.0) -> Instance:
    j, _arr, n, d, L, seed = spec
    L = min(L, n)
    return gaussian_mixture(n=n, d=d, L=L, K=K, lam=lam, seed=seed, name=f"job{j}")


# The named workloads: (builder, default keyword arguments).
WORKLOADS = {
    "mixture-2k": (gaussian_mixture, dict(n=2000, d=16, L=5, K=10, lam=1.0, seed=0)),
    "images-70k": (manifold_images, dict(n=70000, d=784, L=10, K=5, lam=1.0, seed=1)),
    "embeddings-100k": (vmf_embeddings, dict(n=100000, d=4096, L=40, K=10, lam=1.0, seed=2)),
    "large-1m": (anisotropic_mixture, dict(n=1_000_000, d=128, L=50, K=10, lam=1.0, seed=3)),
}


def make(name: str, **overrides) -> Instance:
    """Build a named workload, optionally at another size (e.g. ``n=20000``)."""
    fn, kw = WORKLOADS[name]
    kw = dict(kw)
    kw.update(overrides)
    return fn(**kw)
