"""MI355X (gfx950) implementation of the Scalable Laplacian K-modes bound-optimizer iteration.

Thin Python layer over libslk (include/slk.h): tensors in, tensors out.  All computation runs
in the library's HIP kernels; this module only marshals arguments.  It raises ImportError on
first use if libslk.so has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import SlkError, PREC_FP32, PREC_BF16, PREC_BF16X, KNN_AUTO, KNN_EXACT, KNN_MFMA  # noqa: F401

__all__ = ["Graph", "fit", "assign", "energy", "unary", "inner_step", "params", "SlkError", "timing_enable",
           "timing_read"]


def _torch():
    import torch
    return torch


def _dev(t, dtype, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _prec(p) -> int:
    if p in (0, "fp32", "float32", None):
        return _lib.PREC_FP32
    if p in (1, "bf16", "bfloat16"):
        return _lib.PREC_BF16
    if p in (2, "bf16x"):
        return _lib.PREC_BF16X
    raise ValueError(f"unknown precision {p!r}")


def params(lam=1.0, sigma2=0.0, delta=0.0, tol=1e-8, max_outer=20, max_inner=1000, fixed_inner=0,
           scale=1, prec="fp32", final_pass=0) -> _lib.Params:
    lib = _lib.load()
    p = _lib.Params()
    _lib.check(lib.slk_params_default(C.byref(p)))
    p.lambda_ = float(lam)
    p.sigma2 = float(sigma2)
    p.delta = float(delta)
    p.bound_tol = float(tol)
    p.max_outer = int(max_outer)
    p.max_inner = int(max_inner)
    p.fixed_inner = int(fixed_inner)
    p.pairwise_scale = int(scale)
    p.prec = _prec(prec)
    p.final_pass = int(final_pass)
    return p


class Graph:
    """Device-resident kNN affinity (Section 4.2): kNN lists, symmetric CSR, sigma^2."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        self._lib = _lib.load()

    @classmethod
    def build_knn(cls, x, k=10, reorder=False, method="auto", prec="fp32", candidates=0):
        lib = _lib.load()
        n, d = x.shape
        o = _lib.KnnOpts()
        _lib.check(lib.slk_knn_opts_default(C.byref(o)))
        o.k = int(k)
        o.reorder = int(bool(reorder))
        o.candidates = int(candidates)
        o.method = {"auto": _lib.KNN_AUTO, "exact": _lib.KNN_EXACT, "mfma": _lib.KNN_MFMA}[method]
        o.prec = _prec(prec)
        h = C.c_void_p()
        _lib.check(lib.slk_build_knn(_dev(x, _torch().float32, "x"), n, d, C.byref(o), _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def build_knn_batched(cls, problems):
        """Graphs of several problems [{"x": tensor, "k": .., "reorder": .., "method": .., "prec": ..}, ...]
        in one call (slk_build_knn_batched); the exact searches share one launch."""
        lib = _lib.load()
        torch = _torch()
        items = (_lib.KnnItem * len(problems))()
        for i, pr in enumerate(problems):
            x = pr["x"]
            n, d = x.shape
            o = _lib.KnnOpts()
            _lib.check(lib.slk_knn_opts_default(C.byref(o)))
            o.k = int(pr.get("k", 10))
            o.reorder = int(bool(pr.get("reorder", False)))
            o.candidates = int(pr.get("candidates", 0))
            o.method = {"auto": _lib.KNN_AUTO, "exact": _lib.KNN_EXACT, "mfma": _lib.KNN_MFMA}[pr.get("method", "auto")]
            o.prec = _prec(pr.get("prec", "fp32"))
            items[i] = _lib.KnnItem(_dev(x, torch.float32, "x").value, n, d, 0, o)
        hs = (C.c_void_p * len(problems))()
        _lib.check(lib.slk_build_knn_batched(items, len(problems), _stream(), hs))
        return [cls(C.c_void_p(h)) for h in hs]

    @classmethod
    def from_knn(cls, knn_idx, knn_d2=None, reorder=False):
        torch = _torch()
        lib = _lib.load()
        n, k = knn_idx.shape
        d2 = _dev(knn_d2, torch.float64, "knn_d2", (n, k)) if knn_d2 is not None else None
        h = C.c_void_p()
        _lib.check(lib.slk_graph_from_knn(n, k, _dev(knn_idx, torch.int32, "knn_idx"), d2, int(bool(reorder)),
                                          _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def from_csr(cls, row_ptr, col_idx, sigma2=0.0, reorder=False):
        torch = _torch()
        lib = _lib.load()
        n = row_ptr.shape[0] - 1
        nnz = col_idx.shape[0]
        h = C.c_void_p()
        _lib.check(lib.slk_graph_from_csr(n, nnz, _dev(row_ptr, torch.int32, "row_ptr"),
                                          _dev(col_idx, torch.int32, "col_idx") if nnz else None,
                                          float(sigma2), int(bool(reorder)), _stream(), C.byref(h)))
        return cls(h)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _lib.GraphInfo()
        _lib.check(self._lib.slk_graph_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in i._fields_}

    def export(self):
        torch = _torch()
        inf = self.info()
        n, k, nnz = inf["n"], inf["k"], inf["nnz"]
        rp = torch.empty(n + 1, dtype=torch.int32, device="cuda")
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        ki = kd = None
        if k > 0:
            ki = torch.empty((n, k), dtype=torch.int32, device="cuda")
            kd = torch.empty((n, k), dtype=torch.float64, device="cuda")
        _lib.check(self._lib.slk_graph_export(self._h, _dev(rp, torch.int32, "rp"), _dev(ci, torch.int32, "ci"),
                                              _dev(ki, torch.int32, "ki") if ki is not None else None,
                                              _dev(kd, torch.float64, "kd") if kd is not None else None,
                                              _dev(perm, torch.int32, "perm"), _stream()))
        return dict(row_ptr=rp, col_idx=ci[:nnz], knn_idx=ki, knn_d2=kd, perm=perm)

    def close(self):
        if self._h:
            self._lib.slk_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _outputs(n, L, labels):
    torch = _torch()
    z = torch.empty((n, L), dtype=torch.float32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda") if labels else None
    return z, lab


def assign(x, graph: Graph, modes, lam=1.0, trace=True, **kw):
    """One outer iteration (z-updates for fixed modes).  Returns dict with z, labels,
    modes_next (numpy), bound_trace (numpy) and the result summary."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    m = _lib.host_i32(modes)
    L = len(m)
    p = params(lam=lam, **kw)
    z, lab = _outputs(n, L, True)
    nxt = np.empty(L, dtype=np.int32)
    cap = max(p.max_inner, p.fixed_inner) if trace else 0
    tr = np.zeros(max(cap, 1), dtype=np.float64)
    r = _lib.Result()
    _lib.check(lib.slk_assign(_dev(x, torch.float32, "x"), n, d, graph.handle, L, _lib.ptr_i32(m), C.byref(p),
                              _stream(), _dev(z, torch.float32, "z"), _dev(lab, torch.int32, "labels"),
                              _lib.ptr_i32(nxt), tr.ctypes.data_as(C.c_void_p) if trace else None, cap, C.byref(r)))
    res = r.as_dict()
    return dict(z=z, labels=lab, modes_next=nxt, bound_trace=tr[: res["inner_iters_last"]] if trace else None,
                result=res)


def fit(x, graph: Graph, init_modes, lam=1.0, **kw):
    """SLK-BO (Algorithm 1).  Returns dict with z, labels, modes (numpy) and the summary."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    m = _lib.host_i32(init_modes)
    L = len(m)
    p = params(lam=lam, **kw)
    z, lab = _outputs(n, L, True)
    out = np.empty(L, dtype=np.int32)
    r = _lib.Result()
    _lib.check(lib.slk_fit(_dev(x, torch.float32, "x"), n, d, graph.handle, L, _lib.ptr_i32(m), C.byref(p),
                           _stream(), _dev(z, torch.float32, "z"), _dev(lab, torch.int32, "labels"),
                           _lib.ptr_i32(out), C.byref(r)))
    return dict(z=z, labels=lab, modes=out, result=r.as_dict())


def energy(x, graph: Graph, labels, modes, lam=1.0, sigma2=0.0, delta=0.0, z=None) -> dict:
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    m = _lib.host_i32(modes)
    o = _lib.EnergyOut()
    _lib.check(lib.slk_energy(_dev(x, torch.float32, "x"), n, d, graph.handle, len(m),
                              _dev(labels, torch.int32, "labels"),
                              _dev(z, torch.float32, "z") if z is not None else None, _lib.ptr_i32(m),
                              float(lam), float(sigma2), float(delta), _stream(), C.byref(o)))
    return {f: getattr(o, f) for f, _ in o._fields_}


def unary(x, modes, sigma2, prec="fp32"):
    """(A, Z0): Gaussian unary affinities to the modes and their row softmax."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    m = _lib.host_i32(modes)
    L = len(m)
    a = torch.empty((n, L), dtype=torch.float32, device="cuda")
    z0 = torch.empty((n, L), dtype=torch.float32, device="cuda")
    _lib.check(lib.slk_unary(_dev(x, torch.float32, "x"), n, d, L, _lib.ptr_i32(m), float(sigma2), _prec(prec),
                             _stream(), _dev(a, torch.float32, "a"), _dev(z0, torch.float32, "z0")))
    return a, z0


def inner_step(graph: Graph, a, z_in, lam=1.0, delta=0.0, scale=1):
    """One z-update from z_in; returns (z_out, bound of z_in)."""
    torch = _torch()
    lib = _lib.load()
    n, L = a.shape
    z_out = torch.empty_like(z_in)
    b = C.c_double(0.0)
    _lib.check(lib.slk_inner_step(graph.handle, L, _dev(a, torch.float32, "a"), _dev(z_in, torch.float32, "z_in"),
                                  float(lam), float(delta), int(scale), _stream(),
                                  _dev(z_out, torch.float32, "z_out"), C.byref(b)))
    return z_out, b.value


def inner_step_noalloc(graph: Graph, a, z_in, z_out, bound=None, lam=1.0, delta=0.0, scale=1):
    """One z-update from z_in into the caller's z_out (may be None) through the allocation-free
    entry point; bound (a one-element float64 device tensor, may be None) receives R(z_in).
    Asynchronous on the current stream."""
    torch = _torch()
    lib = _lib.load()
    n, L = a.shape
    zo = None if z_out is None else _dev(z_out, torch.float32, "z_out", (n, L))
    bd = None if bound is None else _dev(bound, torch.float64, "bound", (1,))
    _lib.check(lib.slk_inner_step_noalloc(graph.handle, L, _dev(a, torch.float32, "a", (n, L)),
                                          _dev(z_in, torch.float32, "z_in", (n, L)), float(lam), float(delta),
                                          int(scale), _stream(), zo, bd))


def inner_step_noalloc_max_rows(L):
    return int(_lib.load().slk_inner_step_noalloc_max_rows(int(L)))


def tune_lookup(n, d, L):
    """Tile shapes the library takes for a problem of n points, d dimensions and L clusters."""
    t = _lib.TuneParams()
    _lib.check(_lib.load().slk_tune_lookup(int(n), int(d), int(L), C.byref(t)))
    return {f: getattr(t, f) for f, _ in t._fields_}


def tune_override(wave_steps):
    """Measurement only: force the z-update's wave_steps (0 = back to the table)."""
    _lib.check(_lib.load().slk_tune_override(int(wave_steps)))


def tune_source():
    return _lib.load().slk_tune_source().decode()


def predict(x, z, modes, y, k=10, lam=1.0, sigma2=0.0, graph=None, method="auto", prec="fp32"):
    """Out-of-sample assignment of the queries y (m x d) against a fit (x, z, modes).
    sigma2 <= 0 takes the estimate of `graph`.  Returns (z_y, labels_y, knn_idx)."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    m = y.shape[0]
    mo = _lib.host_i32(modes)
    L = len(mo)
    if sigma2 <= 0:
        if graph is None:
            raise ValueError("pass sigma2 > 0 or the fit's graph")
        sigma2 = graph.info()["sigma2"]
    zy = torch.empty((m, L), dtype=torch.float32, device="cuda")
    lab = torch.empty(m, dtype=torch.int32, device="cuda")
    nn = torch.empty((m, k), dtype=torch.int32, device="cuda")
    _lib.check(lib.slk_predict(_dev(x, torch.float32, "x"), n, d, _dev(z, torch.float32, "z"), L, _lib.ptr_i32(mo),
                               _dev(y, torch.float32, "y"), m, int(k), float(lam), float(sigma2),
                               {"auto": 0, "exact": 1, "mfma": 2}[method], _prec(prec), _stream(),
                               _dev(zy, torch.float32, "z_out"), _dev(lab, torch.int32, "labels"),
                               _dev(nn, torch.int32, "knn_idx")))
    return zy, lab, nn


def mean_shift(x, z, modes, sigma2, tol=1e-6, max_iter=100, prec="fp32"):
    """SLK-MS mode update (Eq. (9)) from the L x d start vectors `modes` with Z fixed.
    Returns (modes L x d float32 device tensor, steps taken)."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    L = z.shape[1]
    out = torch.empty((L, d), dtype=torch.float32, device="cuda")
    it = C.c_int32(0)
    _lib.check(lib.slk_mean_shift(_dev(x, torch.float32, "x"), n, d, _dev(z, torch.float32, "z"), L,
                                  _dev(modes, torch.float32, "modes", (L, d)), float(sigma2), float(tol),
                                  int(max_iter), _prec(prec), _stream(), _dev(out, torch.float32, "modes_out"),
                                  C.byref(it)))
    return out, it.value


def fit_ms(x, graph: Graph, init_modes, lam=1.0, ms_tol=1e-6, ms_max_iter=100, **kw):
    """SLK-MS (Algorithm 1 with the mean-shift mode update) from L x d start vectors.
    Returns dict with z, labels, modes (after the last mean-shift), modes_used (of the last
    z-updates), ms_steps and the summary."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    L = init_modes.shape[0]
    p = params(lam=lam, **kw)
    z, lab = _outputs(n, L, True)
    mo = torch.empty((L, d), dtype=torch.float32, device="cuda")
    mu = torch.empty((L, d), dtype=torch.float32, device="cuda")
    st = C.c_int32(0)
    r = _lib.Result()
    _lib.check(lib.slk_fit_ms(_dev(x, torch.float32, "x"), n, d, graph.handle, L,
                              _dev(init_modes, torch.float32, "init_modes", (L, d)), C.byref(p), float(ms_tol),
                              int(ms_max_iter), _stream(), _dev(z, torch.float32, "z"),
                              _dev(lab, torch.int32, "labels"), _dev(mo, torch.float32, "modes_out"),
                              _dev(mu, torch.float32, "modes_used"), C.byref(st), C.byref(r)))
    return dict(z=z, labels=lab, modes=mo, modes_used=mu, ms_steps=st.value, result=r.as_dict())


def kmeanspp(x, L, u, prec="fp32"):
    """K-means++ centres for the caller's uniforms u (L values in [0, 1)).  Returns
    (centres numpy int32 [L], labels = nearest centre (device int32 [n]), D^2 (device float64 [n]))."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    uh = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    if uh.shape != (L,):
        raise ValueError("u must hold L uniforms")
    cent = np.empty(L, dtype=np.int32)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    d2 = torch.empty(n, dtype=torch.float64, device="cuda")
    _lib.check(lib.slk_kmeanspp(_dev(x, torch.float32, "x"), n, d, int(L), uh.ctypes.data_as(C.c_void_p),
                                _prec(prec), _stream(), _lib.ptr_i32(cent), _dev(lab, torch.int32, "labels"),
                                _dev(d2, torch.float64, "d2")))
    return cent, lab, d2


def dense_modes(x, L, sigma2, z=None, labels=None, prev=None, keep=None, prec="fp32", density=False):
    """Modes by Eq. (1) (or Eq. (10) with prev): per cluster the point of largest z-weighted
    kernel density.  Pass exactly one of z (n x L) and labels (n).  Returns (modes numpy int32,
    best density numpy float32, density n x L device tensor or None)."""
    torch = _torch()
    lib = _lib.load()
    n, d = x.shape
    modes = np.empty(L, dtype=np.int32)
    best = np.empty(L, dtype=np.float32)
    dens = torch.empty((n, L), dtype=torch.float32, device="cuda") if density else None
    pv = _lib.host_i32(prev) if prev is not None else None
    kp = _lib.host_i32(keep) if keep is not None else None
    _lib.check(lib.slk_dense_modes(_dev(x, torch.float32, "x"), n, d, int(L),
                                   _dev(z, torch.float32, "z", (n, L)) if z is not None else None,
                                   _dev(labels, torch.int32, "labels", (n,)) if labels is not None else None,
                                   float(sigma2), _lib.ptr_i32(pv) if pv is not None else None,
                                   _lib.ptr_i32(kp) if kp is not None else None, _prec(prec), _stream(),
                                   _lib.ptr_i32(modes), best.ctypes.data_as(C.c_void_p),
                                   _dev(dens, torch.float32, "density") if density else None))
    return modes, best, dens


def initial_modes(x, L, u, sigma2, prec="fp32"):
    """The start of Section 4.2: K-means++ seeds, the nearest-seed assignment and the start
    modes by Eq. (1).  Returns dict(seeds, labels (device), modes)."""
    seeds, lab, _ = kmeanspp(x, L, u, prec)
    modes, _, _ = dense_modes(x, L, sigma2, labels=lab, keep=seeds, prec=prec)
    return dict(seeds=seeds, labels=lab, modes=modes)


# ----------------------------------------------------------------------------- served form

def knn_opts(k=10, method="auto", reorder=False, prec="fp32", candidates=0):
    o = _lib.KnnOpts()
    _lib.check(_lib.load().slk_knn_opts_default(C.byref(o)))
    o.k = int(k)
    o.reorder = int(bool(reorder))
    o.candidates = int(candidates)
    o.method = {"auto": 0, "exact": 1, "mfma": 2}[method]
    o.prec = _prec(prec)
    return o


class _JobRec:
    """One submitted job: its C description plus the buffers it points into (kept alive here)."""

    def __init__(self, x, init_modes, lam, k, method, reorder, knn_prec, labels, **kw):
        torch = _torch()
        n, d = x.shape
        self.x = x
        self.modes_in = _lib.host_i32(init_modes)
        L = len(self.modes_in)
        self.z, self.labels = _outputs(n, L, labels)
        self.modes_out = np.zeros(L, dtype=np.int32)
        self.res = _lib.Result()
        self.status = C.c_int(-1)
        j = _lib.Job()
        j.x = _dev(x, torch.float32, "x")
        j.n, j.d, j.L = n, d, L
        j.init_modes_host = _lib.ptr_i32(self.modes_in)
        j.knn = knn_opts(k=k, method=method, reorder=reorder, prec=knn_prec)
        j.params = params(lam=lam, **kw)
        j.z_out = _dev(self.z, torch.float32, "z")
        j.labels_out = _dev(self.labels, torch.int32, "labels") if labels else None
        j.modes_out_host = _lib.ptr_i32(self.modes_out)
        j.result_host = C.cast(C.pointer(self.res), C.c_void_p)
        j.status_host = C.cast(C.pointer(self.status), C.c_void_p)
        self.job = j

    def outcome(self):
        return dict(z=self.z, labels=self.labels, modes=self.modes_out.copy(), result=self.res.as_dict(),
                    status=self.status.value)


class Server:
    """Continuous-batching server (slk_server_*): submit jobs at any time, call step() to
    admit what fits and advance every resident job; finished jobs' outcomes are returned by
    step() and kept in .done."""

    def __init__(self, max_jobs=64, passes_per_step=4, memory_budget=0, builders=0, graph_replay=True):
        self._lib = _lib.load()
        o = _lib.ServerOpts()
        _lib.check(self._lib.slk_server_opts_default(C.byref(o)))
        o.max_jobs, o.passes_per_step, o.memory_budget = int(max_jobs), int(passes_per_step), int(memory_budget)
        o.graph_replay = int(bool(graph_replay))
        if builders:
            o.builders = int(builders)
        h = C.c_void_p()
        _lib.check(self._lib.slk_server_create(C.byref(o), _stream(), C.byref(h)))
        self._h = h
        self._jobs = {}
        self.done = {}
        self._buf = np.zeros(max(int(max_jobs), 1) * 4, dtype=np.int64)

    def submit(self, x, init_modes, lam=1.0, k=10, method="auto", reorder=False, knn_prec="fp32", labels=True,
               **kw) -> int:
        rec = _JobRec(x, init_modes, lam, k, method, reorder, knn_prec, labels, **kw)
        t = C.c_int64(-1)
        _lib.check(self._lib.slk_server_submit(self._h, C.byref(rec.job), C.byref(t)))
        self._jobs[t.value] = rec
        return t.value

    def step(self):
        """One step; returns {ticket: outcome} for the jobs that finished."""
        nd, na, nq = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _lib.check(self._lib.slk_server_step(self._h, self._buf.ctypes.data_as(C.c_void_p), len(self._buf),
                                             C.byref(nd), C.byref(na), C.byref(nq)))
        self.active, self.queued = na.value, nq.value
        out = {}
        for t in self._buf[: nd.value].tolist():
            out[t] = self._jobs.pop(t).outcome()
        self.done.update(out)
        return out

    def pending(self) -> int:
        return len(self._jobs)

    def stats(self):
        st = _lib.ServerStats()
        _lib.check(self._lib.slk_server_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if self._h:
            self._lib.slk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fit_batched(problems, max_jobs=64, passes_per_step=4, **common):
    """Fit a list of problems with slk_fit_batched.  Each problem is a dict with x and
    init_modes (and optionally lam, k, method, reorder, knn_prec and slk_params keywords);
    `common` supplies defaults.  Returns one outcome dict per problem, in order."""
    lib = _lib.load()
    recs = []
    for pr in problems:
        kw = dict(common)
        kw.update(pr)
        x, m = kw.pop("x"), kw.pop("init_modes")
        recs.append(_JobRec(x, m, kw.pop("lam", 1.0), kw.pop("k", 10), kw.pop("method", "auto"),
                            kw.pop("reorder", False), kw.pop("knn_prec", "fp32"), kw.pop("labels", True), **kw))
    arr = (_lib.Job * len(recs))(*[r.job for r in recs])
    o = _lib.ServerOpts()
    _lib.check(lib.slk_server_opts_default(C.byref(o)))
    o.max_jobs, o.passes_per_step = int(max_jobs), int(passes_per_step)
    _lib.check(lib.slk_fit_batched(arr, len(recs), C.byref(o), _stream()))
    return [r.outcome() for r in recs]


def pool_trim() -> None:
    """Return the freed memory held by the library's pool on the current device."""
    _lib.check(_lib.load().slk_pool_trim())


def timing_enable(on: bool = True) -> None:
    """Switch per-kernel HIP-event timing on or off (clears the totals)."""
    _lib.check(_lib.load().slk_timing_enable(int(bool(on))))


def timing_read(kernel: str):
    """(launches, total_ms) accumulated for one kernel name since timing_enable."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _lib.check(_lib.load().slk_timing_read(kernel.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value
