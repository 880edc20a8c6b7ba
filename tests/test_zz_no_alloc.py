"""The allocation-free z-update (slk_inner_step_noalloc) against slk_inner_step through the C ABI:
two calls in a row on one device, the second with a smaller input, both within the parity bar
(|dZ| <= 1e-5, bound rel. 1e-5) of the existing entry point and of the FP64 oracle; a third with
L > 64; and the size limit rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

import gen
from oracle import slk as orc
from test_gpu_parity import ZTOL, _say, to_dev

pytestmark = pytest.mark.gpu


def _problem(slk, torch, n, d, L, K, seed, reorder):
    inst = gen.gaussian_mixture(n=n, d=d, L=L, K=K, seed=seed)
    idx, d2 = orc.knn(inst.X, K, block=256)
    g = slk.Graph.from_knn(to_dev(torch, idx, torch.int32), to_dev(torch, d2, torch.float64), reorder=reorder)
    rp, ci = orc.symmetrize(idx, n)
    rng = np.random.default_rng(seed)
    A = rng.random((n, L)).astype(np.float32)
    Z = rng.dirichlet(np.ones(L), size=n).astype(np.float32)
    return g, rp, ci, A, Z


def _check(slk, torch, n, d, L, K, seed, reorder, lam, delta, scale):
    g, rp, ci, A, Z = _problem(slk, torch, n, d, L, K, seed, reorder)
    a, z = to_dev(torch, A, torch.float32), to_dev(torch, Z, torch.float32)
    z_na = torch.full_like(z, float("nan"))
    b_na = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    slk.inner_step_noalloc(g, a, z, z_na, b_na, lam=lam, delta=delta, scale=scale)
    torch.cuda.synchronize()
    z_ref, b_ref = slk.inner_step(g, a, z, lam=lam, delta=delta, scale=scale)
    dz = float((z_na - z_ref).abs().max())
    bound = float(b_na.item())
    _say(f"[noalloc] n={n} L={L} reorder={reorder}: |dZ| vs slk_inner_step {dz:.2e}, bound {bound:.10e} vs {b_ref:.10e}")
    assert dz <= ZTOL
    assert abs(bound - b_ref) <= 1e-5 * abs(b_ref) + 1e-6
    W = orc.csr_matrix(rp, ci, n)
    B = orc.pairwise(W, Z.astype(np.float64), delta)
    S = A.astype(np.float64) + scale * lam * B
    assert np.abs(z_na.cpu().numpy() - orc.softmax_rows(S)).max() <= ZTOL
    R = orc.relaxed_bound(Z.astype(np.float64), A.astype(np.float64), B, lam, scale)
    assert abs(bound - R) <= 1e-5 * abs(R) + 1e-6
    # bound only (no Z output)
    b2 = torch.zeros((1,), dtype=torch.float64, device="cuda")
    slk.inner_step_noalloc(g, a, z, None, b2, lam=lam, delta=delta, scale=scale)
    torch.cuda.synchronize()
    assert float(b2.item()) == bound
    g.close()


def test_noalloc_two_calls_then_smaller(slk, torch):
    _check(slk, torch, 6001, 12, 50, 10, 1, True, 1.0, 0.0, 1)     # locality order: rows through the permutation
    _check(slk, torch, 901, 8, 7, 6, 2, False, 0.7, 2.0, 2)        # smaller, ragged L, diagonal shift, scale 2
    _check(slk, torch, 700, 6, 70, 6, 3, True, 1.0, 0.0, 1)        # L > 64


def test_noalloc_limits(slk, torch):
    from paper_1810_13044_amd import _lib
    lib = _lib.load()
    assert slk.inner_step_noalloc_max_rows(50) == 4193792
    assert slk.inner_step_noalloc_max_rows(0) == 0 and slk.inner_step_noalloc_max_rows(257) == 0
    n = slk.inner_step_noalloc_max_rows(50) + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    g = slk.Graph.from_csr(rp, torch.zeros(0, dtype=torch.int32, device="cuda"), sigma2=1.0)
    fake = C.c_void_p(0x1000)         # never dereferenced: the size check fails first
    st = lib.slk_inner_step_noalloc(g.handle, 50, fake, fake, 1.0, 0.0, 1, None, fake, None)
    assert st == 1                    # SLK_ERR_INVALID_ARG
    assert b"allocation-free limit" in lib.slk_last_error()
    g.close()
