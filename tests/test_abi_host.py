"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/mlpcp.h declares, reports coarse widths that match the paper's
composite interpolation, and rejects invalid arguments on the host before any
GPU call (so these calls are safe without a device)."""
import ctypes
import os
import re

import pytest

import oracle
import paper_2206_13369_amd as mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = ctypes.c_void_p(4096)   # never dereferenced: validation fails first


def _declared():
    txt = open(os.path.join(ROOT, "include", "mlpcp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlpcp_[a-z_]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    assert set(_declared()) == set(mlp.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = mlp.lib()
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("n,levels", [(300, 2), (2000, 3), (400, 3), (1000, 2), (200, 4), (25, 1), (1, 0),
                                      (7, 2), (64, 6)])
def test_coarse_dim_matches_oracle(n, levels):
    assert mlp.coarse_dim(n, levels) == oracle.coarse_dim(n, levels)


@pytest.mark.parametrize("n,levels", [(4, -1), (1, 1), (8, 4)])
def test_coarse_dim_rejects_bad_levels(n, levels):
    assert mlp.lib().mlpcp_coarse_dim(n, levels) == mlp.MLPCP_E_LEVELS


def test_default_opts():
    o = mlp.default_opts()
    assert (o.levels, o.tol, o.max_iter, o.rho, o.mu_max_factor, o.prec, o.check_every, o.r_norm, o.svt_method) == \
        (0, 1e-6, 500, 1.5, 1e7, 0, 1, 0, 0)


def test_workspace_bytes():
    o = mlp.default_opts(levels=3)
    a = mlp.workspace_bytes(2000, 2000, o)
    b = mlp.workspace_bytes(4000, 2000, o)
    assert 0 < a <= b
    # the default-mu0 phase (Gram of P_Q D and two squaring buffers, 2048^2 doubles each)
    # shares the workspace, so it bounds the size from below
    assert a >= 3 * 2048 * 2048 * 8
    # two coarse-data buffers M_P, n_H = 13 columns at a leading dimension of 16
    assert mlp.workspace_bytes(262144, 200, mlp.default_opts(levels=4)) >= 262144 * 16 * 4 * 2
    assert mlp.workspace_bytes(10, 20, o) == 0          # m < n
    assert mlp.workspace_bytes(100, 8, mlp.default_opts(levels=4)) == 0


def _pcp(m, n, ldd, lam, mu0, opts=None, D=FAKE, L=ctypes.c_void_p(12288), S=ctypes.c_void_p(8192), ws=None,
         wsb=0):
    return mlp.lib().mlpcp_pcp_solve(m, n, D, ldd, lam, mu0, ctypes.byref(opts) if opts else None, None, None,
                                     L, S, None, ws, wsb, None, None)


def test_pcp_validation():
    assert _pcp(10, 20, 20, 0.1, 1.0) == mlp.MLPCP_E_SHAPE           # wide
    assert _pcp(20, 10, 5, 0.1, 1.0) == mlp.MLPCP_E_SHAPE            # ld < n
    assert _pcp(0, 0, 0, 0.1, 1.0) == mlp.MLPCP_E_SHAPE
    assert _pcp(20, 10, 10, 0.0, 1.0) == mlp.MLPCP_E_INVALID_ARG     # lambda
    assert _pcp(20, 10, 10, 0.1, float("nan")) == mlp.MLPCP_E_INVALID_ARG    # mu0 (<= 0 selects the default)
    assert _pcp(20, 10, 10, 0.1, float("inf")) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, float("-inf")) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, float("nan"), 1.0) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, D=None) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, L=None) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, S=ctypes.c_void_p(12288)) == mlp.MLPCP_E_INVALID_ARG   # L aliases S
    assert _pcp(20, 10, 10, 0.1, 1.0, L=FAKE) == mlp.MLPCP_E_INVALID_ARG   # L aliases D
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(levels=5)) == mlp.MLPCP_E_LEVELS
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(tol=0.0)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(max_iter=0)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(rho=0.5)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(prec=3)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(prec=-1)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(check_every=3)) == mlp.MLPCP_E_UNSUPPORTED
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(r_norm=3)) == mlp.MLPCP_E_UNSUPPORTED
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(r_norm=-1)) == mlp.MLPCP_E_UNSUPPORTED
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(svt_method=2)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, opts=mlp.default_opts(svt_method=-1)) == mlp.MLPCP_E_INVALID_ARG
    assert _pcp(20, 10, 10, 0.1, 1.0, ws=FAKE, wsb=16) == mlp.MLPCP_E_WORKSPACE
    # L stages P_Q D for the default mu0, so it may not alias the initial S0 / Y0
    L_ = ctypes.c_void_p(12288)
    st = mlp.lib().mlpcp_pcp_solve(20, 10, FAKE, 10, 0.1, 0.0, None, L_, None, L_, ctypes.c_void_p(8192), None,
                                   None, 0, None, None)
    assert st == mlp.MLPCP_E_INVALID_ARG
    st = mlp.lib().mlpcp_pcp_solve(20, 10, FAKE, 10, 0.1, 0.0, None, None, L_, L_, ctypes.c_void_p(8192), None,
                                   None, 0, None, None)
    assert st == mlp.MLPCP_E_INVALID_ARG


def test_cpcp_validation():
    L = mlp.lib()
    args = dict(lam=0.1, mu0=1.0)
    st = L.mlpcp_cpcp_solve(20, 10, FAKE, 10, None, 0.1, 1.0, None, None, None, FAKE, ctypes.c_void_p(8192), None,
                            None, 0, None, None)
    assert st == mlp.MLPCP_E_INVALID_ARG       # missing mask
    st = L.mlpcp_cpcp_solve(5, 10, FAKE, 10, FAKE, 0.1, 1.0, None, None, None, FAKE, ctypes.c_void_p(8192), None,
                            None, 0, None, None)
    assert st == mlp.MLPCP_E_SHAPE
    del args


def test_svt_prox_validation():
    L = mlp.lib()
    r = ctypes.c_int(0)
    assert L.mlpcp_svt_prox(10, 20, FAKE, 20, 0, 1.0, FAKE, ctypes.byref(r), None, 0, None) == mlp.MLPCP_E_SHAPE
    assert L.mlpcp_svt_prox(20, 10, FAKE, 10, 0, 0.0, FAKE, ctypes.byref(r), None, 0, None) == \
        mlp.MLPCP_E_INVALID_ARG
    assert L.mlpcp_svt_prox(20, 10, FAKE, 10, 9, 1.0, FAKE, ctypes.byref(r), None, 0, None) == mlp.MLPCP_E_LEVELS
    assert L.mlpcp_svt_prox(20, 10, None, 10, 0, 1.0, FAKE, ctypes.byref(r), None, 0, None) == \
        mlp.MLPCP_E_INVALID_ARG


def test_stream_ops_validation():
    L = mlp.lib()
    assert L.mlpcp_shrink(10, None, 1.0, FAKE, None) == mlp.MLPCP_E_INVALID_ARG
    assert L.mlpcp_shrink(10, FAKE, -1.0, FAKE, None) == mlp.MLPCP_E_INVALID_ARG
    assert L.mlpcp_shrink(0, None, 1.0, None, None) == mlp.MLPCP_OK       # empty is a no-op
    assert L.mlpcp_restrict(4, 10, FAKE, 9, 1, FAKE, 5, None) == mlp.MLPCP_E_SHAPE
    assert L.mlpcp_restrict(4, 10, FAKE, 10, 1, FAKE, 4, None) == mlp.MLPCP_E_SHAPE
    assert L.mlpcp_restrict(4, 10, FAKE, 10, 7, FAKE, 5, None) == mlp.MLPCP_E_LEVELS
    assert L.mlpcp_restrict(0, 10, None, 10, 1, None, 5, None) == mlp.MLPCP_OK
    assert L.mlpcp_prolong(4, 10, FAKE, 4, 1, FAKE, 10, None) == mlp.MLPCP_E_SHAPE
    assert L.mlpcp_prolong(4, 10, FAKE, 5, 1, None, 10, None) == mlp.MLPCP_E_INVALID_ARG


def test_status_strings():
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, 99):
        assert isinstance(mlp.status_string(s), str) and mlp.status_string(s)


# ---- unconstrained CPCP by Frank-Wolfe Thresholding --------------------------------

def _fwt(m, n, ldd, lamL, lamS, levels=2, tol=1e-3, max_iter=10, L=ctypes.c_void_p(12288),
         S=ctypes.c_void_p(8192), ws=None, ws_bytes=0):
    return mlp.lib().mlpcp_cpcp_fwt(m, n, FAKE, ldd, None, lamL, lamS, levels, tol, max_iter, L, S, ws, ws_bytes,
                                    None, None)


@pytest.mark.parametrize("args,status", [
    ((100, 20, 20, 0.0, 0.1), mlp.MLPCP_E_INVALID_ARG),
    ((100, 20, 20, 1.0, -0.1), mlp.MLPCP_E_INVALID_ARG),
    ((100, 20, 20, float("nan"), 0.1), mlp.MLPCP_E_INVALID_ARG),
    ((10, 20, 20, 1.0, 0.1), mlp.MLPCP_E_SHAPE),
    ((100, 20, 10, 1.0, 0.1), mlp.MLPCP_E_SHAPE),
    ((0, 20, 20, 1.0, 0.1), mlp.MLPCP_E_SHAPE),
])
def test_fwt_rejects_bad_arguments(args, status):
    assert _fwt(*args) == status


def test_fwt_rejects_bad_options():
    assert _fwt(100, 20, 20, 1.0, 0.1, tol=0.0) == mlp.MLPCP_E_INVALID_ARG
    assert _fwt(100, 20, 20, 1.0, 0.1, max_iter=0) == mlp.MLPCP_E_INVALID_ARG
    assert _fwt(100, 8, 8, 1.0, 0.1, levels=4) == mlp.MLPCP_E_LEVELS
    assert _fwt(100, 20, 20, 1.0, 0.1, L=ctypes.c_void_p(8192)) == mlp.MLPCP_E_INVALID_ARG   # L aliases S
    assert _fwt(1000, 200, 200, 1.0, 0.1, levels=1) == mlp.MLPCP_E_UNSUPPORTED               # n_H = 100 > 64
    assert _fwt(100000, 30000, 30000, 1.0, 0.1, levels=9) == mlp.MLPCP_E_UNSUPPORTED         # m n >= 2^31
    assert _fwt(20000, 10000, 10000, 1.0, 0.1, levels=0) == mlp.MLPCP_E_UNSUPPORTED          # power path n > 8192
    assert _fwt(1000, 200, 200, 1.0, 0.1, levels=3, ws=ctypes.c_void_p(4096), ws_bytes=1024) == \
        mlp.MLPCP_E_WORKSPACE


def test_fwt_workspace_bytes():
    a = mlp.fwt_workspace_bytes(1000, 500, 3, True)
    b = mlp.fwt_workspace_bytes(2000, 500, 3, True)
    assert 0 < a < b
    assert mlp.fwt_workspace_bytes(1000, 500, 3, False) < a          # no mask bits
    assert mlp.fwt_workspace_bytes(1000, 500, 0, True) > a           # dense L gradient and power buffers
    assert mlp.fwt_workspace_bytes(10, 20, 0, True) == 0              # m < n
    assert mlp.fwt_workspace_bytes(1000, 200, 1, True) == 0           # n_H > 64


@pytest.mark.slow
def test_validation_under_host_sanitizers(tmp_path):
    """Every host-side rejection path of the C ABI (tests/abi_host_check.c), run against a
    build whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer: the
    statuses match and neither sanitizer reports anything."""
    import shutil
    import subprocess
    from paper_2206_13369_amd.build import build_host_sanitized
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    exe = build_host_sanitized(str(tmp_path / "san"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "abi host checks passed" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
