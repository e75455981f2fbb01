"""Spectral norm of the observed data, used for the customary initial penalty
mu_0 = 1.25 / ||P_Q D||_2 of inexact ALM.  LAPACK singular values in float64."""
from __future__ import annotations

from typing import Optional

import numpy as np


def spectral_norm(D, Q: Optional[np.ndarray] = None) -> float:
    X = np.asarray(D, dtype=np.float64)
    if Q is not None:
        X = np.where(Q, X, 0.0)
    return float(np.linalg.svd(X, compute_uv=False)[0])
