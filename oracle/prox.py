"""The two closed-form subproblem solutions of inexact ALM (Alg. 1).

* Elementwise soft threshold S_tau[x] = sign(x) max(|x| - tau, 0): the minimiser
  over S of the augmented Lagrangian (eq. aug-lagr) for fixed L, Y.  The paper
  uses S_tau without defining it; this is the standard proximal map of
  tau ||.||_1.
* Singular value thresholding U S_tau[Sigma] V^T: the minimiser over L, and, on
  the coarse model, the minimiser of the coarse augmented Lagrangian
  (eq. coarse-aug-lagr), lifted back with the prolongation (Alg. 4).
  Ranks count singular values strictly above tau.
"""
from __future__ import annotations

import numpy as np

from .restriction import orthonormal_restriction


def shrink(X, tau):
    """S_tau[X] = sign(X) * max(|X| - tau, 0), elementwise, float64."""
    X = np.asarray(X, dtype=np.float64)
    return np.sign(X) * np.maximum(np.abs(X) - tau, 0.0)


def svt(M, tau):
    """Returns (U S_tau[Sigma] V^T, rank, singular values) via LAPACK SVD."""
    M = np.asarray(M, dtype=np.float64)
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    r = int(np.count_nonzero(s > tau))
    L = (U[:, :r] * (s[:r] - tau)) @ Vt[:r]
    return L, r, s


def svt_prox(M, tau, levels: int):
    """Coarse SVT lifted back: SVT_tau(M R~) R~^T (Alg. 4 steps 3-6 with the
    S/Y dependence folded into M).  levels = 0 is the plain SVT of M."""
    M = np.asarray(M, dtype=np.float64)
    if levels == 0:
        return svt(M, tau)[:2]
    R = orthonormal_restriction(M.shape[1], levels)
    LH, r, _ = svt(M @ R, tau)
    return LH @ R.T, r
