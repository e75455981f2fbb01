"""K unrolled (multilevel) inexact-ALM iterations in PyTorch float64 on the CPU, for
reference gradients of a recovery loss.  Test infrastructure only.

The forward pass is the iteration of Alg. 4 (Alg. 1 at levels = 0) with a fixed
penalty schedule mu_0 .. mu_{K-1} (held fixed, not recomputed from D):

    M = D - S + Y/mu;  L = SVT_{1/mu}(M R) R^T;  S <- S_{lam/mu}[D - L + Y/mu];
    Y <- Y + mu (D - L - S)

starting from S = Y = 0.  The loss is ||L_K - L0||_F^2.  Gradients with respect to D
and lam come from torch.autograd, i.e. from PyTorch's own SVD backward (an
implementation independent of the GPU adjoint), and are pinned in the tests against
central finite differences in float64.
"""
from __future__ import annotations

import numpy as np
import torch

from .restriction import orthonormal_restriction


def _svt(A: torch.Tensor, tau: float):
    """(SVT_tau(A), number of singular values above tau)."""
    U, s, Vh = torch.linalg.svd(A, full_matrices=False)
    return (U * torch.clamp(s - tau, min=0.0)) @ Vh, int((s.detach() > tau).sum())


def _shrink(X: torch.Tensor, tau) -> torch.Tensor:
    return torch.sign(X) * torch.clamp(torch.abs(X) - tau, min=0.0)


def restriction(n: int, levels: int):
    """The orthonormal restriction as a float64 tensor (None for levels = 0)."""
    return None if levels == 0 else torch.from_numpy(orthonormal_restriction(n, levels))


def step(D, S, Y, lam, mu: float, R, ranks: list | None = None):
    """One explicit iteration of Alg. 4 (Alg. 1 when R is None) at penalty mu:
    returns (L, S', Y').  Differentiable in every tensor argument (forward and
    reverse mode).  ranks: if a list is given, the rank kept by the SVT is appended."""
    M = D - S + Y / mu
    if R is None:
        L, r = _svt(M, 1.0 / mu)
    else:
        LH, r = _svt(M @ R, 1.0 / mu)
        L = LH @ R.T
    if ranks is not None:
        ranks.append(r)
    S_next = _shrink(D - L + Y / mu, lam / mu)
    Y_next = Y + mu * (D - L - S_next)
    return L, S_next, Y_next


def unrolled(D, lam, mus, levels: int, supports: list | None = None):
    """Returns (L_K, S_K, Y_K, ranks) for float64 tensors D (m x n) and lam (scalar
    tensor).  supports: if a list is given, the support of S after every iteration is
    appended to it (boolean arrays), the active set of the soft threshold."""
    m, n = D.shape
    R = restriction(n, levels)
    S = torch.zeros_like(D)
    Y = torch.zeros_like(D)
    L = None
    ranks = []
    for mu in mus:
        L, S, Y = step(D, S, Y, lam, mu, R, ranks)
        if supports is not None:
            supports.append((S != 0).detach().numpy().copy())
    return L, S, Y, ranks


def loss_and_grad(D, L0, lam: float, mus, levels: int):
    """FP64 loss ||L_K - L0||_F^2 and its gradients (dL/dD, dL/dlam) via autograd."""
    Dt = torch.tensor(np.asarray(D, dtype=np.float64), requires_grad=True)
    lt = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    L, _, _, ranks = unrolled(Dt, lt, mus, levels)
    loss = ((L - torch.from_numpy(np.asarray(L0, dtype=np.float64))) ** 2).sum()
    gD, gl = torch.autograd.grad(loss, (Dt, lt))
    return float(loss.detach()), gD.detach().numpy(), float(gl.detach()), ranks


def loss_only(D, L0, lam: float, mus, levels: int, supports: list | None = None):
    """(loss, S_K, per-iteration ranks) without gradients; see unrolled() for supports."""
    with torch.no_grad():
        L, S, _, ranks = unrolled(torch.tensor(np.asarray(D, dtype=np.float64)),
                                  torch.tensor(float(lam), dtype=torch.float64), mus, levels, supports)
        return float(((L - torch.from_numpy(np.asarray(L0, dtype=np.float64))) ** 2).sum()), S.numpy(), ranks
