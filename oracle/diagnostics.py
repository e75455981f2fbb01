"""Diagnostics of the multilevel analysis (Sec. 3.2) for a given restriction R, and the
literal interpolation operator as an alternative to the orthonormalised one.
TEST INFRASTRUCTURE ONLY (see the package docstring).  NumPy float64.

* epsilon (Thm. LH-eps): eps = sum_{k <= r_H} sigma_k(L_H) (1 - sigma_{n_H - k + 1}(R)),
  r_H = rank(L_H); the theorem gives ||L_H R^T||_* >= ||L_H||_* - eps.
* delta (Lemma 3): Delta = <L_H (R^T R - I), L_H - L_H*>, for a coarse iterate L_H and a
  coarse solution L_H*.
* literal_restriction: the composite interpolation operator P itself (scaled = False)
  or P / ||P||_2 (scaled = True, the largest scaling with ||R||_2 <= 1).

For an orthonormal R both quantities vanish identically.
"""
from __future__ import annotations

import numpy as np

from .restriction import composite_interp


def numerical_rank(A, rtol: float = 1e-12) -> int:
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return int(np.count_nonzero(s > rtol * (s[0] if s.size else 0.0)))


def epsilon(LH, R, rtol: float = 1e-12) -> float:
    """Thm. LH-eps: sum over the r_H nonzero singular values of L_H, paired with the
    smallest singular values of R in reverse order."""
    sL = np.linalg.svd(np.asarray(LH, dtype=np.float64), compute_uv=False)
    sR = np.linalg.svd(np.asarray(R, dtype=np.float64), compute_uv=False)
    nH = sR.size
    rH = int(np.count_nonzero(sL > rtol * (sL[0] if sL.size else 0.0)))
    return float(sum(sL[k] * (1.0 - sR[nH - 1 - k]) for k in range(rH)))


def delta(LH, LH_star, R) -> float:
    """Lemma 3: <L_H (R^T R - I), L_H - L_H*> (Frobenius inner product)."""
    R = np.asarray(R, dtype=np.float64)
    E = R.T @ R - np.eye(R.shape[1])
    LH = np.asarray(LH, dtype=np.float64)
    return float(np.sum((LH @ E) * (LH - np.asarray(LH_star, dtype=np.float64))))


def literal_restriction(n: int, levels: int, scaled: bool = True) -> np.ndarray:
    P = composite_interp(n, levels)
    return P / np.linalg.norm(P, 2) if scaled else P
