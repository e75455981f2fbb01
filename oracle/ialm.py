"""Inexact ALM (Alg. 1), multilevel inexact ALM (Alg. 4) and their masked form.

The iteration, in the paper's notation, for k = 0, 1, ...:

    M_H   = (D - S_k + Y_k / mu_k) R              coarse data        (Alg. 4)
    L_H   = U_H S_{1/mu_k}[Sigma_H] V_H^T         coarse SVT         (Alg. 4)
    L     = L_H R^T                               prolongation       (Alg. 4)
    S     = S_{lam/mu_k}[D - L + Y_k / mu_k]      sparse update      (Alg. 1/4)
    Y     = Y_k + mu_k (D - L - S)                dual update        (Alg. 1/4)
    mu    = mu_{k+1}                              penalty update

With levels = 0 the restriction is the identity and this is Alg. 1.

Readings (each also listed in the design notes):

* Penalty schedule: the paper only asks for an increasing sequence.  Reading:
  mu_{k+1} = min(rho mu_k, mu_max) with rho = 1.5 and mu_max = 1e7 mu_0, the
  customary inexact-ALM parameterisation; mu_0 is an input (Alg. 1 requires it).
* Initial S, Y: inputs (Alg. 1 / Alg. 4 requirements); zero by default.
* Stopping: the feasibility gap FG = ||P_Q(D - L - S)||_F / ||P_Q D||_F of the
  experiments section, tested after every iteration.
* Restriction: the orthonormalised interpolation operator (see restriction.py); any
  other n x n_H operator can be passed as R (the literal interpolation operator for the
  ablation of that reading).
* Compressive (masked) form.  The paper states the constrained problem
  P_Q[L + S] = P_Q[D] but solves it only with Frank-Wolfe.  Reading: inexact
  ALM on  min ||L||_* + lam ||P_Q S||_1  s.t. L + S = P_Q D, where S is free
  (unpenalised) off Q.  Its S-step leaves S = -L + Y/mu off Q, so Y stays zero
  there and the next coarse data off Q is the previous L.  Returned S is the
  on-Q part (zero off Q).  With Q = everything this is exactly PCP.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .prox import shrink, svt
from .restriction import orthonormal_restriction


@dataclasses.dataclass
class IALMResult:
    L: np.ndarray
    S: np.ndarray
    Y: np.ndarray
    rank: int
    iters: int
    fg: float
    mu: float                      # penalty used by the last iteration
    converged: bool
    history: list                  # per-iteration dicts


def default_schedule(mu0: float, iters: int, rho: float = 1.5, mu_max_factor: float = 1e7):
    """mu_0, mu_1, ... with mu_{k+1} = min(rho mu_k, mu_max)."""
    mus = [mu0]
    for _ in range(iters - 1):
        mus.append(min(rho * mus[-1], mu_max_factor * mu0))
    return mus


def ialm(D, lam: float, mu0: float, *, Q: Optional[np.ndarray] = None, levels: int = 0,
         rho: float = 1.5, mu_max_factor: float = 1e7, tol: float = 1e-7, max_iter: int = 500,
         S0=None, Y0=None, fixed_iters: Optional[int] = None, R: Optional[np.ndarray] = None,
         record: bool = False, keep_iterates: bool = False) -> IALMResult:
    """Plain (levels = 0) or multilevel inexact ALM, optionally masked.

    fixed_iters: run exactly that many iterations, ignoring ``tol``.
    R: override the restriction (n x n_H); default is the orthonormalised
       interpolation operator for ``levels``.
    keep_iterates: store (L, S, Y, Yhat, U_r, V_r, the coarse iterate L_H) per iteration
       in the history, for invariant checks on small inputs.
    """
    D = np.asarray(D, dtype=np.float64)
    m, n = D.shape
    if Q is None:
        Qb = np.ones((m, n), dtype=bool)
    else:
        Qb = np.asarray(Q, dtype=bool)
    if R is None:
        R = None if levels == 0 else orthonormal_restriction(n, levels)
    PD = np.where(Qb, D, 0.0)
    nrmD = np.linalg.norm(PD)
    S = np.zeros((m, n)) if S0 is None else np.where(Qb, np.asarray(S0, dtype=np.float64), 0.0)
    Y = np.zeros((m, n)) if Y0 is None else np.where(Qb, np.asarray(Y0, dtype=np.float64), 0.0)
    L = np.zeros((m, n))
    mu = float(mu0)
    mu_max = mu_max_factor * mu0
    hist = []
    n_iter = fixed_iters if fixed_iters is not None else max_iter
    fg = np.inf
    rank = 0
    converged = False
    k = 0
    for k in range(1, n_iter + 1):
        mu_k = mu
        # coarse data: D - S + Y/mu on Q, previous L off Q
        Mk = np.where(Qb, D - S + Y / mu_k, L)
        LH = None
        if R is None:
            L_new, rank, sig = svt(Mk, 1.0 / mu_k)
            Ur = Vr = None
            if keep_iterates:
                U, s, Vt = np.linalg.svd(Mk, full_matrices=False)
                Ur, Vr = U[:, :rank], Vt[:rank].T
        else:
            MH = Mk @ R
            LH, rank, sig = svt(MH, 1.0 / mu_k)
            L_new = LH @ R.T
            Ur = Vr = None
            if keep_iterates:
                U, s, Vt = np.linalg.svd(MH, full_matrices=False)
                Ur, Vr = U[:, :rank], Vt[:rank].T
        # sparse step on Q
        S_new = np.where(Qb, shrink(D - L_new + Y / mu_k, lam / mu_k), 0.0)
        Z = np.where(Qb, D - L_new - S_new, 0.0)
        Y_new = Y + mu_k * Z
        fg = float(np.linalg.norm(Z) / nrmD)
        if record or keep_iterates:
            h = dict(k=k, mu=mu_k, rank=rank, fg=fg, sigma=sig.copy())
            if keep_iterates:
                Yhat = Y + mu_k * (D - S - L_new)
                h.update(L=L_new.copy(), S=S_new.copy(), Y=Y_new.copy(), Yprev=Y.copy(), Sprev=S.copy(),
                         Yhat=Yhat, Ur=Ur, Vr=Vr, LH=None if LH is None else LH.copy())
            hist.append(h)
        L, S, Y = L_new, S_new, Y_new
        mu = min(rho * mu_k, mu_max)
        if fixed_iters is None and fg <= tol:
            converged = True
            break
    return IALMResult(L=L, S=S, Y=Y, rank=rank, iters=k, fg=fg, mu=mu_k if k else mu0,
                      converged=converged, history=hist)
