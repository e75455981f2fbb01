"""Frank-Wolfe Thresholding (Alg. 3) and multilevel Frank-Wolfe Thresholding
(Alg. 6) for the unconstrained CPCP problem (eq. cpcp)

    min_{L,S}  1/2 ||P_Q[L + S - D]||_F^2 + lam_L ||L||_* + lam_S ||S||_1

in its epigraph form (eq. cpcp-epi, eq. cpcp-fw): variables (L, S, t_L, t_S) with
||L||_* <= t_L <= U_L and ||S||_1 <= t_S <= U_S, objective

    f(L, S, t_L, t_S) = 1/2 ||P_Q[L + S - D]||_F^2 + lam_L t_L + lam_S t_S.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy float64,
LAPACK SVD for the top singular pair.

One iteration, for k = 1, 2, ... (Alg. 3, with Alg. 6's coarse nuclear oracle
when levels > 0):

    G     = P_Q[L + S - D]                                   eq. (cpcp-grad-LS)
    M_L   = -u v^T, (u, sigma, v) the top singular triple of G          (fine)
          = -u (R v_H)^T / ||R||_2, (u, sigma, v_H) top triple of G R  (coarse)
    M_S   = -sign(G_ij) e_i e_j^T at (i, j) = argmax |G_ij|
    V_L, V_tL = 0, 0        if lam_L >= -<G, M_L>,  else U_L M_L, U_L
    V_S, V_tS = 0, 0        if lam_S >= -<G, M_S>,  else U_S M_S, U_S
    (alpha, beta) = argmin over [0, 1]^2 of f along
          L + alpha (V_L - L), t_L + alpha (V_tL - t_L),
          S + beta  (V_S - S), t_S + beta  (V_tS - t_S)          (exact line search)
    L, t_L      <- the alpha point;   S_half, t_S_half <- the beta point
    S     = S_{lam_S}[S_half - P_Q[L + S_half - D]],  t_S = ||S||_1
    U_L   = f / lam_L,  U_S = f / lam_S

initialised with L = S = 0, t_L = t_S = 0, U_L = f_0 / lam_L, U_S = f_0 / lam_S.

Readings (each also listed in the design notes):

* The thresholding step is written with L^(k+1/2); no such iterate exists, the
  only new L of the iteration is the line-search point L^(k+1), which is used.
* The bound update is written with a function g that is never defined, with
  garbled parentheses; it is read as the objective f at the new iterate.
* The coarse ball radius is written 1/||R||_* ; the bound that makes the lifted
  atom feasible is ||M_H R^T||_* <= ||R||_2 ||M_H||_*, so the radius is read as
  1/||R||_2.  With the orthonormalised restriction R~ (restriction.py) the
  radius is 1 and the lifted atom -u (R~ v_H)^T has nuclear norm exactly 1.
* Stopping: the paper runs to a 1e-3 tolerance without defining it.  Reading:
  the relative decrease of the objective, |f_{k-1} - f_k| / f_{k-1} <= tol,
  tested after every iteration (f_0 = 1/2 ||P_Q D||^2).
* Line search: the minimiser of a convex quadratic over the unit square is
  taken over the candidates (origin, corners, the minimiser of each edge, the
  interior stationary point); among equal values the first in that order wins,
  so a direction that changes nothing (zero curvature and zero slope) keeps
  step 0.
* Gradient after a threshold step: on Q the new S is S_{lam_S}[D - L] (the two
  S_half terms of its argument cancel), hence L + S - D = -clamp(D - L, -lam_S,
  lam_S) exactly and |G| <= lam_S, which keeps the l1 oracle's gate closed from
  the second iteration on.  G is evaluated in that clipped form; the literal sum
  can exceed lam_S by a rounding error, which would open the gate and add a
  spike of height U_S with a vanishing step (noise, not the method).
* The step of the threshold is 1 (the Lipschitz constant of the gradient in S
  alone), so the threshold is lam_S itself.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .prox import shrink
from .restriction import orthonormal_restriction


@dataclasses.dataclass
class FWTResult:
    L: np.ndarray
    S: np.ndarray
    t_L: float
    t_S: float
    f: float                       # objective f(L, S, t_L, t_S) at the returned iterate
    iters: int
    converged: bool
    history: list                  # per-iteration dicts


def objective(D, Q, L, S, t_L, t_S, lam_L, lam_S) -> float:
    """f of eq. (cpcp-fw)."""
    R = np.where(Q, L + S - D, 0.0)
    return 0.5 * float(np.sum(R * R)) + lam_L * t_L + lam_S * t_S


def cpcp_value(D, Q, L, S, lam_L, lam_S) -> float:
    """The unconstrained CPCP objective of eq. (cpcp): f with t_L = ||L||_*, t_S = ||S||_1."""
    nuc = float(np.sum(np.linalg.svd(L, compute_uv=False)))
    return objective(D, Q, L, S, nuc, float(np.abs(S).sum()), lam_L, lam_S)


def top_singular_triple(A):
    """(u, sigma_1, v) of A by LAPACK SVD."""
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    return U[:, 0].copy(), float(s[0]), Vt[0].copy()


def nuclear_lmo(G):
    """argmin over ||M||_* <= 1 of <G, M>:  -u v^T; returns (u, v, <G, M>) with
    <G, M> = -sigma_1(G) (the nuclear ball's support function is the spectral norm)."""
    u, s, v = top_singular_triple(G)
    return u, v, -s


def coarse_nuclear_lmo(G, R):
    """Alg. 6: argmin over ||M_H||_* <= 1/||R||_2 of <G R, M_H>, lifted by R^T.
    Returns (u, w, <G, M_L>) with M_L = -u w^T, w = R v_H / ||R||_2."""
    u, s, vH = top_singular_triple(G @ R)
    r2 = float(np.linalg.norm(R, 2))
    return u, (R @ vH) / r2, -s / r2


def l1_lmo(G):
    """argmin over ||M||_1 <= 1 of <G, M>:  -sign(G_ij) e_i e_j^T at the entry of
    largest magnitude (first in row-major order among equals); returns
    (i, j, sign, <G, M>) with <G, M> = -max |G|."""
    flat = int(np.argmax(np.abs(G)))
    i, j = divmod(flat, G.shape[1])
    g = float(G[i, j])
    sgn = 1.0 if g > 0 else (-1.0 if g < 0 else 0.0)
    return i, j, sgn, -abs(g)


def box_qp(haa: float, hab: float, hbb: float, ga: float, gb: float):
    """argmin over (a, b) in [0, 1]^2 of 1/2 (haa a^2 + 2 hab a b + hbb b^2) + ga a + gb b
    for a positive semidefinite Hessian.  Exact: the minimum of a convex
    quadratic over the square is attained at a corner, at the minimiser of one
    edge or at the interior stationary point, and all of them are compared."""
    def phi(a, b):
        return 0.5 * (haa * a * a + 2.0 * hab * a * b + hbb * b * b) + ga * a + gb * b

    def clamp01(x):
        return min(1.0, max(0.0, x))

    cands = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (1.0, 1.0)]
    for b in (0.0, 1.0):                       # edges b = const: minimise over a
        if haa > 0.0:
            cands.append((clamp01(-(ga + hab * b) / haa), b))
    for a in (0.0, 1.0):                       # edges a = const: minimise over b
        if hbb > 0.0:
            cands.append((a, clamp01(-(gb + hab * a) / hbb)))
    det = haa * hbb - hab * hab
    if det > 0.0:
        a = (-ga * hbb + gb * hab) / det
        b = (-gb * haa + ga * hab) / det
        if 0.0 <= a <= 1.0 and 0.0 <= b <= 1.0:
            cands.append((a, b))
    best, bv = cands[0], phi(*cands[0])
    for c in cands[1:]:
        v = phi(*c)
        if v < bv:
            best, bv = c, v
    return best


def fwt(D, lam_L: float, lam_S: float, *, Q: Optional[np.ndarray] = None, levels: int = 0,
        tol: float = 1e-3, max_iter: int = 1000, fixed_iters: Optional[int] = None,
        R: Optional[np.ndarray] = None, keep_iterates: bool = False) -> FWTResult:
    """FW-T (levels = 0, Alg. 3) or ML-FWT (levels > 0, Alg. 6) for eq. (cpcp).

    fixed_iters: run exactly that many iterations, ignoring ``tol``.
    R: override the restriction (n x n_H); default is the orthonormalised
       interpolation operator for ``levels``.
    keep_iterates: store L, S and the gradient of each iteration in the history.
    """
    D = np.asarray(D, dtype=np.float64)
    m, n = D.shape
    Qb = np.ones((m, n), dtype=bool) if Q is None else np.asarray(Q, dtype=bool)
    if lam_L <= 0 or lam_S <= 0:
        raise ValueError("lam_L and lam_S must be positive")
    if R is None and levels > 0:
        R = orthonormal_restriction(n, levels)

    L = np.zeros((m, n))
    S = np.zeros((m, n))
    t_L = t_S = 0.0
    f = objective(D, Qb, L, S, t_L, t_S, lam_L, lam_S)
    U_L, U_S = f / lam_L, f / lam_S
    history = []
    iters, converged = 0, False
    if f == 0.0:
        return FWTResult(L, S, t_L, t_S, f, 0, True, history)
    limit = fixed_iters if fixed_iters is not None else max_iter
    thresholded = False
    for k in range(1, limit + 1):
        if thresholded:
            # after a threshold step S = S_{lam_S}[D - L] on Q, so the residual there
            # is L + S - D = -clamp(D - L, -lam_S, lam_S): evaluated in that form
            G = np.where(Qb, -np.clip(D - L, -lam_S, lam_S), 0.0)
        else:
            G = np.where(Qb, L + S - D, 0.0)
        # linear oracles (steps 3-4 of Alg. 3, step 3 of Alg. 6)
        if R is None:
            u, w, gML = nuclear_lmo(G)
        else:
            u, w, gML = coarse_nuclear_lmo(G, R)
        i, j, sgn, gMS = l1_lmo(G)
        # gates (steps 5-16)
        takeL = not (lam_L >= -gML)
        takeS = not (lam_S >= -gMS)
        V_L = -U_L * np.outer(u, w) if takeL else np.zeros((m, n))
        V_tL = U_L if takeL else 0.0
        V_S = np.zeros((m, n))
        if takeS:
            V_S[i, j] = -U_S * sgn
        V_tS = U_S if takeS else 0.0
        # exact line search over the two segments (step 17)
        A = np.where(Qb, V_L - L, 0.0)
        B = np.where(Qb, V_S - S, 0.0)
        haa, hab, hbb = float(np.sum(A * A)), float(np.sum(A * B)), float(np.sum(B * B))
        ga = float(np.sum(G * A)) + lam_L * (V_tL - t_L)
        gb = float(np.sum(G * B)) + lam_S * (V_tS - t_S)
        alpha, beta = box_qp(haa, hab, hbb, ga, gb)
        gap = -(ga + gb)               # Frank-Wolfe gap <grad f, x - v> at x_k
        L = L + alpha * (V_L - L)
        t_L = t_L + alpha * (V_tL - t_L)
        S_half = S + beta * (V_S - S)
        # thresholding step (steps 18-19)
        S = shrink(S_half - np.where(Qb, L + S_half - D, 0.0), lam_S)
        t_S = float(np.abs(S).sum())
        thresholded = True
        f_prev = f
        f = objective(D, Qb, L, S, t_L, t_S, lam_L, lam_S)
        # bound update (steps 20-21)
        U_L, U_S = f / lam_L, f / lam_S
        iters = k
        rec = dict(k=k, sigma=-gML, gmax=-gMS, takeL=takeL, takeS=takeS, spike=(i, j),
                   alpha=alpha, beta=beta, f=f, gap=gap, t_L=t_L, t_S=t_S,
                   rel_change=abs(f_prev - f) / f_prev if f_prev > 0 else 0.0)
        if keep_iterates:
            rec.update(G=G, L=L.copy(), S=S.copy(), u=u, w=w)
        history.append(rec)
        if fixed_iters is None and rec["rel_change"] <= tol:
            converged = True
            break
    return FWTResult(L, S, t_L, t_S, f, iters, converged, history)
