"""The C ABI without a GPU: the library loads, exports every function declared in
include/slk.h, fills defaults, and rejects invalid arguments before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names.update(re.findall(r"\b(slk_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1810_13044_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("slk_build_knn", "slk_fit", "slk_assign", "slk_energy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_defaults(lib):
    from paper_1810_13044_amd import _lib
    p = _lib.Params()
    assert lib.slk_params_default(C.byref(p)) == 0
    assert (p.lambda_, p.sigma2, p.delta, p.bound_tol) == (1.0, 0.0, 0.0, 1e-8)
    assert (p.max_outer, p.max_inner, p.fixed_inner, p.pairwise_scale, p.prec) == (20, 1000, 0, 1, 0)
    o = _lib.KnnOpts()
    assert lib.slk_knn_opts_default(C.byref(o)) == 0
    assert (o.k, o.reorder, o.candidates, o.method, o.prec) == (10, 0, 0, 0, 0)
    assert lib.slk_version().startswith(b"libslk")
    so = _lib.ServerOpts()
    assert lib.slk_server_opts_default(C.byref(so)) == 0
    assert (so.max_jobs, so.passes_per_step, so.memory_budget, so.builders) == (64, 4, 0, 3)


def test_invalid_arguments_rejected_before_launch(lib):
    from paper_1810_13044_amd import _lib
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)        # never dereferenced: validation fails first
    o = _lib.KnnOpts()
    lib.slk_knn_opts_default(C.byref(o))
    assert lib.slk_build_knn(None, 100, 4, C.byref(o), None, C.byref(h)) == 1
    assert b"NULL" in lib.slk_last_error()
    assert lib.slk_build_knn(fake, 1, 4, C.byref(o), None, C.byref(h)) == 1
    assert lib.slk_build_knn(fake, 100, 0, C.byref(o), None, C.byref(h)) == 1
    o.k = 0
    assert lib.slk_build_knn(fake, 100, 4, C.byref(o), None, C.byref(h)) == 1
    o.k = 100
    assert lib.slk_build_knn(fake, 100, 4, C.byref(o), None, C.byref(h)) == 1
    assert b"k must" in lib.slk_last_error()
    o.k = 65
    assert lib.slk_build_knn(fake, 1000, 4, C.byref(o), None, C.byref(h)) == 1
    assert lib.slk_graph_from_knn(100, 0, fake, None, 0, None, C.byref(h)) == 1
    assert lib.slk_graph_from_csr(100, -1, fake, fake, 0.0, 0, None, C.byref(h)) == 1
    p = _lib.Params()
    lib.slk_params_default(C.byref(p))
    modes = np.array([0, 1], dtype=np.int32)
    r = _lib.Result()
    # graph NULL
    assert lib.slk_fit(fake, 100, 4, None, 2, modes.ctypes.data_as(C.c_void_p), C.byref(p), None, fake, None,
                       modes.ctypes.data_as(C.c_void_p), C.byref(r)) == 1
    assert lib.slk_unary(fake, 100, 4, 0, modes.ctypes.data_as(C.c_void_p), 1.0, 0, None, fake, fake) == 1
    assert lib.slk_unary(fake, 100, 4, 2, modes.ctypes.data_as(C.c_void_p), -1.0, 0, None, fake, fake) == 1
    bad = np.array([0, 100], dtype=np.int32)
    assert lib.slk_unary(fake, 100, 4, 2, bad.ctypes.data_as(C.c_void_p), 1.0, 0, None, fake, fake) == 1
    assert b"out of range" in lib.slk_last_error()
    assert lib.slk_unary(fake, 100, 4, 2, modes.ctypes.data_as(C.c_void_p), 1.0, 7, None, fake, fake) == 1
    assert lib.slk_inner_step(None, 2, fake, fake, 1.0, 0.0, 1, None, fake, None) == 1
    assert lib.slk_graph_info(None, None) == 1
    lib.slk_graph_destroy(None)       # a no-op


def test_python_layer_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1810_13044_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load(str(tmp_path / "missing.so"))


def test_extension_entry_points_reject_invalid_arguments(lib):
    """slk_kmeanspp, slk_dense_modes, slk_mean_shift, slk_fit_ms and slk_predict check their
    arguments on the host before any device work."""
    from paper_1810_13044_amd import _lib
    fake = C.c_void_p(0x1000)
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    u = np.array([0.2, 0.5, 1.0], dtype=np.float64)
    cent = np.zeros(3, dtype=np.int32)
    assert lib.slk_kmeanspp(fake, 100, 4, 3, P(u), 0, None, P(cent), None, None) == 1
    assert b"[0, 1)" in lib.slk_last_error()
    u[2] = 0.7
    assert lib.slk_kmeanspp(fake, 100, 4, 101, P(u), 0, None, P(cent), None, None) == 1
    assert lib.slk_kmeanspp(fake, 100, 4, 3, None, 0, None, P(cent), None, None) == 1
    assert lib.slk_kmeanspp(fake, 100, 4, 3, P(u), 9, None, P(cent), None, None) == 1
    modes = np.zeros(65, dtype=np.int32)
    best = np.zeros(65, dtype=np.float32)
    assert lib.slk_dense_modes(fake, 100, 4, 65, fake, None, 1.0, None, None, 0, None, P(modes), P(best), None) == 1
    assert lib.slk_dense_modes(fake, 100, 4, 3, None, None, 1.0, None, None, 0, None, P(modes), P(best), None) == 1
    assert b"exactly one" in lib.slk_last_error()
    assert lib.slk_dense_modes(fake, 100, 4, 3, fake, fake, 1.0, None, None, 0, None, P(modes), P(best), None) == 1
    assert lib.slk_dense_modes(fake, 100, 4, 3, fake, None, 0.0, None, None, 0, None, P(modes), P(best), None) == 1
    prev = np.array([0, 1, 100], dtype=np.int32)
    assert lib.slk_dense_modes(fake, 100, 4, 3, fake, None, 1.0, P(prev), None, 0, None, P(modes), P(best),
                               None) == 1
    assert b"out of range" in lib.slk_last_error()
    it = C.c_int32(0)
    assert lib.slk_mean_shift(fake, 100, 4, fake, 65, fake, 1.0, 1e-6, 10, 0, None, fake, C.byref(it)) == 1
    assert lib.slk_mean_shift(fake, 100, 4, fake, 3, fake, -1.0, 1e-6, 10, 0, None, fake, C.byref(it)) == 1
    assert lib.slk_mean_shift(fake, 100, 4, fake, 3, fake, 1.0, 1e-6, 0, 0, None, fake, C.byref(it)) == 1
    p = _lib.Params()
    lib.slk_params_default(C.byref(p))
    r = _lib.Result()
    assert lib.slk_fit_ms(fake, 100, 4, None, 3, fake, C.byref(p), 1e-6, 10, None, fake, None, fake, None, None,
                          C.byref(r)) == 1
    assert lib.slk_predict(fake, 100, 4, fake, 3, P(prev[:2]), fake, 10, 0, 1.0, 1.0, 0, 0, None, fake, None,
                           None) == 1
    assert b"k must" in lib.slk_last_error()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("n,d,width", [(12289, 20, 4), (9001, 128, 8), (16411, 72, 8), (4095, 2000, 4),
                                       (4096, 2000, 8), (262144, 4, 4), (262145, 4, 8)])
def test_exact_knn_width_rule(n, d, width):
    """The exact kNN's queries per work-group as the library reports them (host lookup, no GPU):
    4 while the points take at most 4 MiB (n d 4 bytes) or there are fewer than 4,096 query rows,
    else 8 - the rule the GPU tests exercise on both sides of each clause."""
    import paper_1810_13044_amd as slk
    t = slk.tune_lookup(n, d, 10)
    assert t["knn_exact_width"] == width
    assert t["wave_steps"] in (1, 2, 4, 8)


@pytest.mark.parametrize("n,long_scan", [(393215, 0), (393216, 1), (2000, 0), (1000000, 1)])
def test_knn_long_scan_rule(n, long_scan):
    """The MFMA candidate search tests each key tile against all of a wave's rows before merging
    from 393,216 keys on (host lookup, no GPU); the GPU tests build graphs on both sides."""
    import paper_1810_13044_amd as slk
    assert slk.tune_lookup(n, 64, 10)["knn_long_scan"] == long_scan
