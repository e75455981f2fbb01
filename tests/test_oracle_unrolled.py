"""Pins of the FP64 reference gradient of K unrolled (multilevel) inexact-ALM
iterations: its forward pass equals the NumPy oracle's iteration (Alg. 1 / Alg. 4),
and its gradients with respect to D and lambda match central finite differences in
float64 along seeded unit-Frobenius directions (directions whose perturbation
changes an active set -- the support of S or a rank at some step -- are rejected)."""
import numpy as np
import pytest

import oracle
from oracle import unrolled as U
import synth


def _work(levels, seed=3, m=48, n=40):
    w = synth.gaussian_lowrank_plus_sparse(m, n, 3, seed=seed, sparse_frac=0.05, levels=levels)
    mus = oracle.default_schedule(w.mu0, 8)
    return w, mus


@pytest.mark.parametrize("levels", [0, 1])
def test_forward_equals_numpy_oracle(levels):
    w, mus = _work(levels)
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, fixed_iters=len(mus))
    import torch
    L, S, Y, ranks = U.unrolled(torch.tensor(w.D.astype(np.float64)), torch.tensor(w.lam, dtype=torch.float64),
                                mus, levels)
    assert np.allclose(L.numpy(), ref.L, atol=1e-12, rtol=0)
    assert np.allclose(S.numpy(), ref.S, atol=1e-12, rtol=0)
    assert np.allclose(Y.numpy(), ref.Y, atol=1e-9, rtol=0)


def _support_and_ranks(D, w, mus, levels):
    _, S, ranks = U.loss_only(D, w.L0, w.lam, mus, levels)
    return S != 0, ranks


@pytest.mark.parametrize("levels", [0, 1])
def test_gradient_matches_central_differences(levels):
    w, mus = _work(levels)
    D = w.D.astype(np.float64)
    loss, gD, gl, ranks = U.loss_and_grad(D, w.L0, w.lam, mus, levels)
    assert np.isfinite(gD).all() and np.isfinite(gl)
    rng = np.random.default_rng(0)
    h = 1e-6
    supp0, r0 = _support_and_ranks(D, w, mus, levels)
    used = 0
    for _ in range(40):
        E = rng.normal(size=D.shape)
        E /= np.linalg.norm(E)
        sp, rp = _support_and_ranks(D + h * E, w, mus, levels)
        sm, rm = _support_and_ranks(D - h * E, w, mus, levels)
        if not (np.array_equal(sp, supp0) and np.array_equal(sm, supp0) and rp == r0 and rm == r0):
            continue
        fp = U.loss_only(D + h * E, w.L0, w.lam, mus, levels)[0]
        fm = U.loss_only(D - h * E, w.L0, w.lam, mus, levels)[0]
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gD * E))
        assert abs(fd - an) <= 1e-4 * max(abs(fd), 1e-3 * np.linalg.norm(gD)), (fd, an)
        used += 1
        if used == 12:
            break
    assert used >= 8
    # lambda
    fp = U.loss_only(D, w.L0, w.lam + h, mus, levels)[0]
    fm = U.loss_only(D, w.L0, w.lam - h, mus, levels)[0]
    fd = (fp - fm) / (2 * h)
    assert abs(fd - gl) <= 1e-4 * max(abs(fd), 1e-8)
