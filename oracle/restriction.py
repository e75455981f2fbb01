"""Restriction / prolongation operators of the coarse model (Sec. 3.1).

Readings taken here (each also listed in the design notes):

* One level (eq. (Rx) and the worked n = 6 example of Sec. 3.1): for even n the
  operator is n x n/2, its first two rows both pick coarse point 0, odd rows
  2k+1 pick coarse point k and even rows 2k (k >= 1) average coarse points k-1
  and k.  The printed general matrix ends in a row "... 1 2" which disagrees
  with the worked example (last row = last coarse point alone); the example is
  followed.
* Odd n is not covered by the paper.  Reading: vertex-centred interpolation
  without the duplicated row, coarse points at fine rows 0, 2, ..., n-1 and
  midpoints at odd rows; n_H = (n + 1) / 2.  Rows still sum to one and the
  columns stay independent (Assumption 1).
* "levels" counts halvings: the composite is P_n P_{n_1} ... (levels factors),
  n_{i+1} = n_H(n_i) (Sec. 3.1, the product of interpolation operators).
* Normalisation (Assumption 4 is garbled: a nuclear norm can never be below
  the spectral norm).  Reading: the coarse model uses the orthonormalised
  operator R~ = P (P^T P)^{-1/2}, which has the same column range as the
  paper's P and satisfies ||R~||_2 = 1 and R~^T R~ = I, the case in which the
  nuclear-norm gap of Theorem LH-eps vanishes (epsilon = 0) and Delta_k of
  Lemma 3 is identically zero.
"""
from __future__ import annotations

import numpy as np


def coarse_dim(n: int, levels: int) -> int:
    """n_H after ``levels`` halvings (even n -> n/2, odd n -> (n+1)/2)."""
    if levels < 0:
        raise ValueError("levels must be >= 0")
    for _ in range(levels):
        if n < 2:
            raise ValueError("too many levels for this n")
        n = n // 2 if n % 2 == 0 else (n + 1) // 2
    return n


def interp_level(n: int) -> np.ndarray:
    """One interpolation operator P_n (n x n_H), Sec. 3.1 eq. (Rx) read through
    the worked example.  Entries are 0, 1/2 or 1."""
    if n < 2:
        raise ValueError("need n >= 2")
    if n % 2 == 0:
        nH = n // 2
        P = np.zeros((n, nH))
        P[0, 0] = 1.0                      # duplicated first row of the example
        for k in range(nH):
            P[2 * k + 1, k] = 1.0          # fine point coincides with coarse point k
        for k in range(1, nH):
            P[2 * k, k - 1] = 0.5          # midpoint between coarse k-1 and k
            P[2 * k, k] = 0.5
    else:
        nH = (n + 1) // 2
        P = np.zeros((n, nH))
        for k in range(nH):
            P[2 * k, k] = 1.0
        for k in range(nH - 1):
            P[2 * k + 1, k] = 0.5
            P[2 * k + 1, k + 1] = 0.5
    return P


def composite_interp(n: int, levels: int) -> np.ndarray:
    """P = P_n P_{n_1} ... P_{n_{levels-1}}  (n x n_H); identity for levels = 0."""
    P = np.eye(n)
    cur = n
    for _ in range(levels):
        Pl = interp_level(cur)
        P = P @ Pl
        cur = Pl.shape[1]
    return P


def orthonormal_restriction(n: int, levels: int) -> np.ndarray:
    """R~ = P (P^T P)^{-1/2}: orthonormal columns spanning range(P)."""
    P = composite_interp(n, levels)
    if levels == 0:
        return P
    w, V = np.linalg.eigh(P.T @ P)
    C = (V / np.sqrt(w)) @ V.T
    return P @ C


def restrict(X: np.ndarray, levels: int) -> np.ndarray:
    """X R~  (m x n -> m x n_H), the coarse-model map applied to rows."""
    return X @ orthonormal_restriction(X.shape[1], levels)


def prolong(XH: np.ndarray, n: int, levels: int) -> np.ndarray:
    """X_H R~^T  (m x n_H -> m x n), the lift back to the fine dimension."""
    R = orthonormal_restriction(n, levels)
    if XH.shape[1] != R.shape[1]:
        raise ValueError("coarse width does not match n and levels")
    return XH @ R.T
