"""Python binding of libmlpcp: multilevel PCP / CPCP on AMD MI355X.

Argument marshalling only.  Every step of the solver runs in the HIP kernels of
libmlpcp.so behind the C ABI declared in include/mlpcp.h; PyTorch supplies
device memory (tensors, the caching allocator for workspaces) and the current
HIP stream.  There is no CPU fallback: if the library is missing, importing the
functions that need it raises.

Entry points (same names as the C ABI, minus the ``mlpcp_`` prefix):
    pcp_solve, cpcp_solve, svt_prox, shrink, restrict, prolong,
    coarse_dim, workspace_bytes, default_opts, status_string,
    cpcp_fwt, fwt_workspace_bytes
and the raw ctypes handle ``lib()`` for tests that call the C ABI directly.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlpcp.so")

MLPCP_OK = 0
MLPCP_NOT_CONVERGED = 1
MLPCP_E_INVALID_ARG = -1
MLPCP_E_SHAPE = -2
MLPCP_E_LEVELS = -3
MLPCP_E_NONFINITE = -4
MLPCP_E_EIG = -5
MLPCP_E_WORKSPACE = -6
MLPCP_E_HIP = -7
MLPCP_E_UNSUPPORTED = -8

EXPORTED = (
    "mlpcp_default_opts", "mlpcp_coarse_dim", "mlpcp_workspace_bytes", "mlpcp_pcp_solve",
    "mlpcp_cpcp_solve", "mlpcp_svt_prox", "mlpcp_shrink", "mlpcp_restrict", "mlpcp_prolong",
    "mlpcp_status_string", "mlpcp_profile_enable", "mlpcp_profile_read", "mlpcp_step_workspace_bytes",
    "mlpcp_ialm_step", "mlpcp_ialm_step_vjp", "mlpcp_fwt_workspace_bytes", "mlpcp_cpcp_fwt",
    "mlpcp_svt_prox_static",
)


class Opts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("rho", ctypes.c_double), ("mu_max_factor", ctypes.c_double), ("prec", ctypes.c_int),
                ("check_every", ctypes.c_int), ("r_norm", ctypes.c_int), ("svt_method", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("fg", ctypes.c_double), ("rank", ctypes.c_int),
                ("mu_final", ctypes.c_double), ("tau_margin", ctypes.c_double), ("eig_sweeps", ctypes.c_int),
                ("fg_history", ctypes.POINTER(ctypes.c_double)), ("rank_history", ctypes.POINTER(ctypes.c_int)),
                ("history_len", ctypes.c_int), ("gram_bf16_iters", ctypes.c_int),
                ("gram_split_iters", ctypes.c_int), ("sweeps_history", ctypes.POINTER(ctypes.c_int)),
                ("mu0", ctypes.c_double), ("partial_eig_iters", ctypes.c_int), ("msvt_iters", ctypes.c_int),
                ("msvt_flags", ctypes.c_int), ("msvt_products", ctypes.c_int)]


class FwtInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("f", ctypes.c_double),
                ("t_L", ctypes.c_double), ("t_S", ctypes.c_double), ("rel_change", ctypes.c_double),
                ("gap", ctypes.c_double), ("power_steps", ctypes.c_longlong),
                ("f_history", ctypes.POINTER(ctypes.c_double)), ("alpha_history", ctypes.POINTER(ctypes.c_double)),
                ("beta_history", ctypes.POINTER(ctypes.c_double)), ("sigma_history", ctypes.POINTER(ctypes.c_double)),
                ("history_len", ctypes.c_int)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_longlong), ("total_ms", ctypes.c_double)]


class MLPCPError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} (status {status})")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmlpcp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2206_13369_amd.build` "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, d, f, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_size_t
    L.mlpcp_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.mlpcp_default_opts.restype = None
    L.mlpcp_coarse_dim.argtypes = [i, i]
    L.mlpcp_coarse_dim.restype = i
    L.mlpcp_workspace_bytes.argtypes = [i, i, ctypes.POINTER(Opts)]
    L.mlpcp_workspace_bytes.restype = sz
    L.mlpcp_pcp_solve.argtypes = [i, i, vp, i, f, d, ctypes.POINTER(Opts), vp, vp, vp, vp, vp, vp, sz,
                                  ctypes.POINTER(Info), vp]
    L.mlpcp_pcp_solve.restype = i
    L.mlpcp_cpcp_solve.argtypes = [i, i, vp, i, vp, f, d, ctypes.POINTER(Opts), vp, vp, vp, vp, vp, vp, sz,
                                   ctypes.POINTER(Info), vp]
    L.mlpcp_cpcp_solve.restype = i
    L.mlpcp_svt_prox.argtypes = [i, i, vp, i, i, f, vp, ctypes.POINTER(i), vp, sz, vp]
    L.mlpcp_svt_prox.restype = i
    L.mlpcp_svt_prox_static.argtypes = [i, i, vp, i, i, f, vp, ctypes.POINTER(i), vp]
    L.mlpcp_svt_prox_static.restype = i
    L.mlpcp_shrink.argtypes = [sz, vp, f, vp, vp]
    L.mlpcp_shrink.restype = i
    L.mlpcp_restrict.argtypes = [i, i, vp, i, i, vp, i, vp]
    L.mlpcp_restrict.restype = i
    L.mlpcp_prolong.argtypes = [i, i, vp, i, i, vp, i, vp]
    L.mlpcp_prolong.restype = i
    L.mlpcp_status_string.argtypes = [i]
    L.mlpcp_status_string.restype = ctypes.c_char_p
    L.mlpcp_profile_enable.argtypes = [i]
    L.mlpcp_profile_enable.restype = i
    L.mlpcp_profile_read.argtypes = [ctypes.POINTER(KernelTime), i]
    L.mlpcp_profile_read.restype = i
    L.mlpcp_step_workspace_bytes.argtypes = [i, i, i]
    L.mlpcp_step_workspace_bytes.restype = sz
    L.mlpcp_ialm_step.argtypes = [i, i, i, vp, i, vp, vp, f, d, vp, vp, vp, ctypes.POINTER(i), vp, sz, vp]
    L.mlpcp_ialm_step.restype = i
    L.mlpcp_ialm_step_vjp.argtypes = [i, i, i, vp, i, vp, vp, f, d, vp, vp, vp, vp, vp, vp,
                                      ctypes.POINTER(d), vp, sz, vp]
    L.mlpcp_ialm_step_vjp.restype = i
    L.mlpcp_fwt_workspace_bytes.argtypes = [i, i, i, i]
    L.mlpcp_fwt_workspace_bytes.restype = sz
    L.mlpcp_cpcp_fwt.argtypes = [i, i, vp, i, vp, f, f, i, d, i, vp, vp, vp, sz, ctypes.POINTER(FwtInfo), vp]
    L.mlpcp_cpcp_fwt.restype = i
    _lib = L
    return L


KERNEL_CLASSES = ("init_restrict", "gram", "coarse_CGC", "jacobi_pairs", "jacobi_apply", "jacobi_misc",
                  "svt_prep", "epilogue", "reduce", "finalize", "coarse_svt_small", "fw_pass", "fw_power",
                  "fw_small", "fw_top", "msvt_mm", "recon_gemm", "other")


def profile_enable(on=True) -> None:
    """Per-kernel-class HIP-event timing: True = all classes, False = off, or an
    iterable of class names to time only those.  Resets the counters."""
    if on is True:
        mask = -1
    elif not on:
        mask = 0
    else:
        mask = 0
        for name in on:
            mask |= 1 << KERNEL_CLASSES.index(name)
    lib().mlpcp_profile_enable(mask)


def profile_read() -> dict:
    """{kernel class: (launches, total milliseconds)} accumulated since profile_enable."""
    buf = (KernelTime * 32)()
    k = lib().mlpcp_profile_read(buf, 32)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(min(k, 32))}


def status_string(status: int) -> str:
    return lib().mlpcp_status_string(int(status)).decode()


def coarse_dim(n: int, levels: int) -> int:
    r = lib().mlpcp_coarse_dim(int(n), int(levels))
    if r < 0:
        raise MLPCPError(r, "coarse_dim")
    return r


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().mlpcp_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def workspace_bytes(m: int, n: int, opts: Optional[Opts] = None) -> int:
    return int(lib().mlpcp_workspace_bytes(int(m), int(n), ctypes.byref(opts) if opts is not None else None))


# ---- torch marshalling -------------------------------------------------------------

def _torch():
    import torch
    return torch


def _check_dev(t, name, dtype=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t


def _check_mn(t, name, m, n):
    """Optional (None) or a contiguous m x n float32 device tensor."""
    if t is None:
        return
    _check_dev(t, name, _torch().float32)
    if tuple(t.shape) != (m, n) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous m x n tensor")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(_torch().cuda.current_stream(device).cuda_stream)


@dataclasses.dataclass
class SolveResult:
    L: object
    S: object
    Y: object
    status: int
    iters: int
    fg: float
    rank: int
    mu_final: float
    tau_margin: float
    eig_sweeps: int
    fg_history: list
    rank_history: list
    gram_bf16_iters: int = 0
    gram_split_iters: int = 0
    sweeps_history: list = dataclasses.field(default_factory=list)
    mu0: float = 0.0
    partial_eig_iters: int = 0
    msvt_iters: int = 0
    msvt_flags: int = 0
    msvt_products: int = 0


PRECISIONS = {"fp32": 0, "bf16": 1, "bf16x3": 2}


def _prec(p) -> int:
    if isinstance(p, str):
        if p not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        return PRECISIONS[p]
    return int(p)


def _solve(D, Q, lam, mu0, levels, tol, max_iter, rho, mu_max_factor, S0, Y0, want_y, workspace, history,
           prec="fp32", r_norm=0, svt_method=0):
    torch = _torch()
    _check_dev(D, "D", torch.float32)
    if D.dim() != 2 or D.stride(1) != 1:
        raise ValueError("D must be a 2-D row-major tensor")
    m, n = D.shape
    dev = D.device
    L = torch.empty((m, n), dtype=torch.float32, device=dev)
    S = torch.empty((m, n), dtype=torch.float32, device=dev)
    Y = torch.empty((m, n), dtype=torch.float32, device=dev) if want_y else None
    for name, t in (("S0", S0), ("Y0", Y0)):
        if t is not None:
            _check_dev(t, name, torch.float32)
            if not t.is_contiguous() or tuple(t.shape) != (m, n):
                raise ValueError(f"{name} must be a contiguous m x n tensor")
    o = default_opts(levels=levels, tol=tol, max_iter=max_iter, rho=rho, mu_max_factor=mu_max_factor,
                     prec=_prec(prec), r_norm=int(r_norm), svt_method=int(svt_method))
    wsb = workspace_bytes(m, n, o)
    if workspace is None:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    else:
        ws = workspace
        if ws.numel() < wsb:
            raise ValueError(f"workspace needs {wsb} bytes")
    info = Info()
    fh = (ctypes.c_double * history)() if history else None
    rh = (ctypes.c_int * history)() if history else None
    sh = (ctypes.c_int * history)() if history else None
    if history:
        info.fg_history = fh
        info.rank_history = rh
        info.sweeps_history = sh
        info.history_len = history
    ld = D.stride(0)
    mu0 = 0.0 if mu0 is None else float(mu0)
    if Q is None:
        st = lib().mlpcp_pcp_solve(m, n, _ptr(D), ld, float(lam), float(mu0), ctypes.byref(o), _ptr(S0), _ptr(Y0),
                                   _ptr(L), _ptr(S), _ptr(Y), _ptr(ws), ws.numel(), ctypes.byref(info),
                                   _stream(dev))
    else:
        _check_dev(Q, "Q", torch.uint8)
        if not Q.is_contiguous() or tuple(Q.shape) != (m, n):
            raise ValueError("Q must be a contiguous m x n uint8 tensor")
        st = lib().mlpcp_cpcp_solve(m, n, _ptr(D), ld, _ptr(Q), float(lam), float(mu0), ctypes.byref(o), _ptr(S0),
                                    _ptr(Y0), _ptr(L), _ptr(S), _ptr(Y), _ptr(ws), ws.numel(), ctypes.byref(info),
                                    _stream(dev))
    if st < 0:
        raise MLPCPError(st, "cpcp_solve" if Q is not None else "pcp_solve")
    k = min(info.iters, history) if history else 0
    return SolveResult(L, S, Y, st, info.iters, info.fg, info.rank, info.mu_final, info.tau_margin, info.eig_sweeps,
                       [fh[i] for i in range(k)] if history else [], [rh[i] for i in range(k)] if history else [],
                       info.gram_bf16_iters, info.gram_split_iters,
                       [sh[i] for i in range(k)] if history else [], info.mu0, info.partial_eig_iters,
                       info.msvt_iters, info.msvt_flags, info.msvt_products)


def pcp_solve(D, lam: float, mu0: Optional[float] = None, *, levels: int = 0, tol: float = 1e-6, max_iter: int = 500,
              rho: float = 1.5, mu_max_factor: float = 1e7, S0=None, Y0=None, want_y: bool = True,
              workspace=None, history: int = 0, prec="fp32", r_norm: int = 0, svt_method: int = 0) -> SolveResult:
    """Robust PCA by (multilevel) inexact ALM; D is an m x n float32 tensor on the GPU.
    mu0: initial penalty; None or <= 0 selects 1.25 / ||D||_2, computed on the device.
    prec: "fp32", "bf16" or "bf16x3" (the arithmetic of the coarse SVT's products).
    r_norm: restriction normalisation, 0 orthonormal (default), 1 P / ||P||_2, 2 P.
    svt_method: 0 matrix-function coarse SVT where eligible, 1 eigensolver only."""
    return _solve(D, None, lam, mu0, levels, tol, max_iter, rho, mu_max_factor, S0, Y0, want_y, workspace, history,
                  prec, r_norm, svt_method)


def cpcp_solve(D, Q, lam: float, mu0: Optional[float] = None, *, levels: int = 0, tol: float = 1e-6, max_iter: int = 500,
               rho: float = 1.5, mu_max_factor: float = 1e7, S0=None, Y0=None, want_y: bool = True,
               workspace=None, history: int = 0, prec="fp32", r_norm: int = 0,
               svt_method: int = 0) -> SolveResult:
    """Compressive PCP (constrained form) by masked (multilevel) inexact ALM; Q uint8 mask.
    mu0: initial penalty; None or <= 0 selects 1.25 / ||P_Q D||_2, computed on the device.
    prec: "fp32", "bf16" or "bf16x3" (the arithmetic of the coarse SVT's products).
    r_norm: restriction normalisation, 0 orthonormal (default), 1 P / ||P||_2, 2 P.
    svt_method: 0 matrix-function coarse SVT where eligible, 1 eigensolver only."""
    return _solve(D, Q, lam, mu0, levels, tol, max_iter, rho, mu_max_factor, S0, Y0, want_y, workspace, history,
                  prec, r_norm, svt_method)


def svt_prox(M, tau: float, levels: int = 0, workspace=None):
    """L = SVT_tau(M R) R^T and the number of singular values kept."""
    torch = _torch()
    _check_dev(M, "M", torch.float32)
    m, n = M.shape
    L = torch.empty((m, n), dtype=torch.float32, device=M.device)
    o = default_opts(levels=levels)
    wsb = workspace_bytes(m, n, o)
    ws = workspace if workspace is not None else torch.empty(max(wsb, 1), dtype=torch.uint8, device=M.device)
    r = ctypes.c_int(0)
    st = lib().mlpcp_svt_prox(m, n, _ptr(M), M.stride(0), levels, float(tau), _ptr(L), ctypes.byref(r), _ptr(ws),
                              ws.numel(), _stream(M.device))
    if st < 0:
        raise MLPCPError(st, "svt_prox")
    return L, r.value


def shrink(X, tau: float, out=None):
    torch = _torch()
    _check_dev(X, "X", torch.float32)
    if not X.is_contiguous():
        raise ValueError("X must be contiguous")
    Y = torch.empty_like(X) if out is None else out
    st = lib().mlpcp_shrink(X.numel(), _ptr(X), float(tau), _ptr(Y), _stream(X.device))
    if st < 0:
        raise MLPCPError(st, "shrink")
    return Y


def restrict(X, levels: int):
    torch = _torch()
    _check_dev(X, "X", torch.float32)
    m, n = X.shape
    nH = coarse_dim(n, levels)
    XH = torch.empty((m, nH), dtype=torch.float32, device=X.device)
    st = lib().mlpcp_restrict(m, n, _ptr(X), X.stride(0), levels, _ptr(XH), nH, _stream(X.device))
    if st < 0:
        raise MLPCPError(st, "restrict")
    return XH


def prolong(XH, n: int, levels: int):
    torch = _torch()
    _check_dev(XH, "XH", torch.float32)
    m, nH = XH.shape
    X = torch.empty((m, n), dtype=torch.float32, device=XH.device)
    st = lib().mlpcp_prolong(m, n, _ptr(XH), XH.stride(0), levels, _ptr(X), n, _stream(XH.device))
    if st < 0:
        raise MLPCPError(st, "prolong")
    return X


# ---- differentiation form ------------------------------------------------------------

def step_workspace(m: int, n: int, levels: int, device):
    torch = _torch()
    return torch.empty(max(int(lib().mlpcp_step_workspace_bytes(m, n, levels)), 1), dtype=torch.uint8,
                       device=device)


def ialm_step(D, S, Y, lam: float, mu: float, levels: int, workspace=None):
    """One explicit (multilevel) inexact-ALM iteration; S, Y may be None (zeros).
    Returns (L, S_next, Y_next, rank)."""
    torch = _torch()
    _check_dev(D, "D", torch.float32)
    if D.dim() != 2 or D.stride(1) != 1:
        raise ValueError("D must be a 2-D row-major tensor")
    m, n = D.shape
    _check_mn(S, "S", m, n)
    _check_mn(Y, "Y", m, n)
    L = torch.empty((m, n), dtype=torch.float32, device=D.device)
    Sn = torch.empty_like(L)
    Yn = torch.empty_like(L)
    ws = workspace if workspace is not None else step_workspace(m, n, levels, D.device)
    r = ctypes.c_int(0)
    st = lib().mlpcp_ialm_step(m, n, levels, _ptr(D), D.stride(0), _ptr(S), _ptr(Y), float(lam), float(mu), _ptr(L),
                               _ptr(Sn), _ptr(Yn), ctypes.byref(r), _ptr(ws), ws.numel(), _stream(D.device))
    if st < 0:
        raise MLPCPError(st, "ialm_step")
    return L, Sn, Yn, r.value


def ialm_step_vjp(D, S, Y, lam: float, mu: float, levels: int, L_bar, S_bar, Y_bar, D_bar, workspace=None):
    """Adjoint of ialm_step: accumulates into D_bar, returns (S_bar_prev, Y_bar_prev, lambda_bar).
    D_bar must have D's shape and row stride (the C ABI addresses both with D's leading
    dimension)."""
    torch = _torch()
    _check_dev(D, "D", torch.float32)
    if D.dim() != 2 or D.stride(1) != 1:
        raise ValueError("D must be a 2-D row-major tensor")
    m, n = D.shape
    _check_dev(D_bar, "D_bar", torch.float32)
    if tuple(D_bar.shape) != (m, n) or D_bar.stride(1) != 1 or D_bar.stride(0) != D.stride(0):
        raise ValueError("D_bar must be m x n with D's row stride")
    for name, t in (("S", S), ("Y", Y), ("L_bar", L_bar), ("S_bar", S_bar), ("Y_bar", Y_bar)):
        _check_mn(t, name, m, n)
    Sbp = torch.empty((m, n), dtype=torch.float32, device=D.device)
    Ybp = torch.empty_like(Sbp)
    ws = workspace if workspace is not None else step_workspace(m, n, levels, D.device)
    lb = ctypes.c_double(0.0)
    st = lib().mlpcp_ialm_step_vjp(m, n, levels, _ptr(D), D.stride(0), _ptr(S), _ptr(Y), float(lam), float(mu),
                                   _ptr(L_bar), _ptr(S_bar), _ptr(Y_bar), _ptr(D_bar), _ptr(Sbp), _ptr(Ybp),
                                   ctypes.byref(lb), _ptr(ws), ws.numel(), _stream(D.device))
    if st < 0:
        raise MLPCPError(st, "ialm_step_vjp")
    return Sbp, Ybp, lb.value


# ---- unconstrained CPCP by (multilevel) Frank-Wolfe Thresholding ----------------------

@dataclasses.dataclass
class FwtResult:
    L: object
    S: object
    status: int
    iters: int
    converged: bool
    f: float
    t_L: float
    t_S: float
    rel_change: float
    gap: float
    power_steps: int
    f_history: list
    alpha_history: list
    beta_history: list
    sigma_history: list


def fwt_workspace_bytes(m: int, n: int, levels: int, masked: bool) -> int:
    return int(lib().mlpcp_fwt_workspace_bytes(int(m), int(n), int(levels), 1 if masked else 0))


def cpcp_fwt(D, Q, lam_L: float, lam_S: float, *, levels: int = 0, tol: float = 1e-3, max_iter: int = 1000,
             workspace=None, history: int = 0) -> FwtResult:
    """min 1/2 ||P_Q[L + S - D]||^2 + lam_L ||L||_* + lam_S ||S||_1 by FW-T (levels = 0)
    or ML-FWT (levels > 0); D m x n float32 on the GPU, Q uint8 mask or None."""
    torch = _torch()
    _check_dev(D, "D", torch.float32)
    if D.dim() != 2 or D.stride(1) != 1:
        raise ValueError("D must be a 2-D row-major tensor")
    m, n = D.shape
    dev = D.device
    if Q is not None:
        _check_dev(Q, "Q", torch.uint8)
        if not Q.is_contiguous() or tuple(Q.shape) != (m, n):
            raise ValueError("Q must be a contiguous m x n uint8 tensor")
    L = torch.empty((m, n), dtype=torch.float32, device=dev)
    S = torch.empty((m, n), dtype=torch.float32, device=dev)
    wsb = fwt_workspace_bytes(m, n, levels, Q is not None)
    if wsb == 0:
        raise MLPCPError(MLPCP_E_SHAPE, "cpcp_fwt")
    if workspace is None:
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    else:
        ws = workspace
        if ws.numel() < wsb:
            raise ValueError(f"workspace needs {wsb} bytes")
    info = FwtInfo()
    hs = [(ctypes.c_double * history)() for _ in range(4)] if history else None
    if history:
        info.f_history, info.alpha_history, info.beta_history, info.sigma_history = hs
        info.history_len = history
    st = lib().mlpcp_cpcp_fwt(m, n, _ptr(D), D.stride(0), _ptr(Q), float(lam_L), float(lam_S), int(levels),
                              float(tol), int(max_iter), _ptr(L), _ptr(S), _ptr(ws), ws.numel(), ctypes.byref(info),
                              _stream(dev))
    if st < 0:
        raise MLPCPError(st, "cpcp_fwt")
    k = min(info.iters, history) if history else 0
    hist = [[h[i] for i in range(k)] for h in hs] if history else [[], [], [], []]
    return FwtResult(L, S, st, info.iters, bool(info.converged), info.f, info.t_L, info.t_S, info.rel_change,
                     info.gap, int(info.power_steps), *hist)
