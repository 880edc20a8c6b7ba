"""MI355X (gfx950) implementation of the Scalable Laplacian K-modes bound-optimizer iteration.

Thin Python layer over libslk (include/slk.h): tensors in, tensors out.  All computation runs
in the library's HIP kernels; this module only marshals arguments.  It raises ImportError on
first use if libslk.so has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import SlkError, PREC_FP32, PREC_BF16, KNN_AUTO, KNN_EXACT, KNN_MFMA  # noqa: F401

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
    raise ValueError(f"unknown precision {p!r}")


def params(lam=1.0, sigma2=0.0, delta=0.0, tol=1e-8, max_outer=20, max_inner=1000, fixed_inner=0,
           scale=1, prec="fp32") -> _lib.Params:
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


def timing_enable(on: bool = True) -> None:
    """Switch per-kernel HIP-event timing on or off (clears the totals)."""
    _lib.check(_lib.load().slk_timing_enable(int(bool(on))))


def timing_read(kernel: str):
    """(launches, total_ms) accumulated for one kernel name since timing_enable."""
    n = C.c_int64(0)
    ms = C.c_double(0.0)
    _lib.check(_lib.load().slk_timing_read(kernel.encode(), C.byref(n), C.byref(ms)))
    return n.value, ms.value
