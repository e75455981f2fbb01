"""The allocation-free entry point mlpcp_svt_prox_static (workspace and operator in
a static device array) against mlpcp_svt_prox (caller workspace, cached operator),
called through the C ABI on the same seeded inputs: identical rank and L within the
float32 bar (1e-5 relative; the kernels are shared, so the bits agree).  Calls in a
row with shrinking inputs and changing (n, levels), so that the array keeps an
earlier call's contents and the operator is rebuilt in it."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2206_13369_amd as mlp
import synth
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


def _both(M, levels, tau):
    torch, dev = torch_dev()
    L = mlp.lib()
    m, n = M.shape
    s = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    L1 = torch.full((m, n), float("nan"), dtype=torch.float32, device=dev)
    L2 = torch.full((m, n), float("nan"), dtype=torch.float32, device=dev)
    r1, r2 = ctypes.c_int(-1), ctypes.c_int(-1)
    ws = torch.empty(mlp.workspace_bytes(m, n, mlp.default_opts(levels=levels)), dtype=torch.uint8, device=dev)
    st1 = L.mlpcp_svt_prox(m, n, ctypes.c_void_p(M.data_ptr()), M.stride(0), levels, tau,
                           ctypes.c_void_p(L1.data_ptr()), ctypes.byref(r1), ctypes.c_void_p(ws.data_ptr()),
                           ws.numel(), s)
    st2 = L.mlpcp_svt_prox_static(m, n, ctypes.c_void_p(M.data_ptr()), M.stride(0), levels, tau,
                                  ctypes.c_void_p(L2.data_ptr()), ctypes.byref(r2), s)
    torch.cuda.synchronize()
    return st1, st2, to_np(L1), to_np(L2), r1.value, r2.value


def _tau_inside_spectrum(D, levels):
    """A threshold between the 40% and 60% quantiles of the coarse singular values, so
    that the SVT keeps part of the spectrum (the oracle's restriction is used only to
    choose the test's threshold)."""
    X = D.astype(np.float64)
    if levels > 0:
        X = X @ oracle.orthonormal_restriction(D.shape[1], levels)
    s = np.linalg.svd(X, compute_uv=False)
    return float(0.5 * (np.quantile(s, 0.4) + np.quantile(s, 0.6)))


@pytest.mark.parametrize("cases", [
    [(3000, 400, 3), (1200, 250, 2)],        # tall coarse model, then a smaller one
    [(2000, 256, 2), (900, 200, 0)],         # multilevel, then a smaller plain call
    [(4096, 320, 1), (4096, 320, 1), (700, 96, 3)],
])
def test_static_matches_svt_prox(cases):
    for k, (m, n, levels) in enumerate(cases):
        w = synth.gaussian_lowrank_plus_sparse(m, n, 6, seed=70 + k, sparse_frac=0.05, levels=max(levels, 1))
        tau = _tau_inside_spectrum(w.D, levels)
        M = to_dev(w.D)
        say(f"static svt_prox call {k}: {m}x{n} levels {levels} tau {tau}")
        st1, st2, L1, L2, r1, r2 = _both(M, levels, float(tau))
        assert st1 == mlp.MLPCP_OK and st2 == mlp.MLPCP_OK
        say(f"   rank {r2}/{r1} err {rel(L2, L1):.1e} equal {np.array_equal(L1, L2)}")
        assert r1 == r2 and 0 < r1 < mlp.coarse_dim(n, levels)
        assert np.isfinite(L2).all()
        assert rel(L2, L1) <= 1e-5


def test_static_rejects_sizes_beyond_the_array():
    torch, dev = torch_dev()
    m, n = 40000, 1000
    M = torch.zeros((m, n), dtype=torch.float32, device=dev)
    Lo = torch.zeros_like(M)
    r = ctypes.c_int(-1)
    st = mlp.lib().mlpcp_svt_prox_static(m, n, ctypes.c_void_p(M.data_ptr()), n, 0, 1.0,
                                         ctypes.c_void_p(Lo.data_ptr()), ctypes.byref(r), None)
    torch.cuda.synchronize()
    assert st == mlp.MLPCP_E_WORKSPACE and r.value == -1
