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
        assert abs(fd - an) <= 1e-4 * max(abs(fd), abs(an)), (fd, an)
        used += 1
        if used == 12:
            break
    assert used >= 8
    # lambda
    fp = U.loss_only(D, w.L0, w.lam + h, mus, levels)[0]
    fm = U.loss_only(D, w.L0, w.lam - h, mus, levels)[0]
    fd = (fp - fm) / (2 * h)
    assert abs(fd - gl) <= 1e-4 * max(abs(fd), 1e-8)


def _active(D, w, mus, levels, lam=None):
    sup = []
    f, _, ranks = U.loss_only(D, w.L0, w.lam if lam is None else lam, mus, levels, supports=sup)
    return f, sup, ranks


def _same_sets(a, b):
    return len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.slow
def test_c4_gradient_central_differences():
    """The 1000 x 1000 differentiated workload (rank 20, 5% +-1, K = 20, 2 levels): FP64
    central differences along 32 accepted seeded unit-Frobenius directions agree with
    the reference gradient to 1e-4 relative, direction by direction.  mu_k is held
    fixed.  A direction is rejected (and a new one drawn) when D +- hE changes an
    active set: the support of S after any of the K iterations or any rank; rejections
    are counted and bounded.  lambda gets one central difference (step 1e-9) under the
    same guard.

    Step h = 2e-7.  At h = 1e-6 no direction keeps every active set (measured: 0 of 40;
    each flips one to three of the 2 * 10^7 shrinkage decisions, and the kink puts up
    to 2e-3 into the quotient); at 1e-7 the FP64 rounding of the loss, about 1e-14
    relative, reaches 1e-4 of a directional derivative.  At 2e-7 about 60% of the
    directions are kept and the worst error measured was 1.9e-5."""
    w = synth.config("c4")
    K = 20
    mus = oracle.default_schedule(w.mu0, K)
    D = w.D.astype(np.float64)
    _, gD, gl, _ = U.loss_and_grad(D, w.L0, w.lam, mus, w.levels)
    _, sup0, r0 = _active(D, w, mus, w.levels)
    h = 2e-7
    rng = np.random.default_rng(2024)
    accepted, rejected, worst = 0, 0, 0.0
    while accepted < 32:
        assert rejected <= 48, f"{rejected} directions rejected before 32 were accepted"
        E = rng.normal(size=D.shape)
        E /= np.linalg.norm(E)
        fp, sp, rp = _active(D + h * E, w, mus, w.levels)
        fm, sm, rm = _active(D - h * E, w, mus, w.levels)
        if not (_same_sets(sp, sup0) and _same_sets(sm, sup0) and rp == r0 and rm == r0):
            rejected += 1
            continue
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gD * E))
        err = abs(fd - an) / max(abs(fd), abs(an))
        assert err <= 1e-4, (accepted, fd, an)
        worst = max(worst, err)
        accepted += 1
    print(f"c4 central differences: {accepted} directions accepted, {rejected} rejected, "
          f"worst relative error {worst:.2e}")
    # lambda moves every threshold lam / mu_k at once: step 1e-9 (at 1e-8 one of the
    # 2 * 10^7 decisions flips; the quotient's rounding at 1e-9 is ~1e-7 relative)
    hl = 1e-9
    fp, sp, rp = _active(D, w, mus, w.levels, lam=w.lam + hl)
    fm, sm, rm = _active(D, w, mus, w.levels, lam=w.lam - hl)
    assert _same_sets(sp, sup0) and _same_sets(sm, sup0) and rp == r0 and rm == r0
    fd = (fp - fm) / (2 * hl)
    assert abs(fd - gl) <= 1e-4 * max(abs(fd), abs(gl)), (fd, gl)


@pytest.mark.parametrize("levels", [0, 2])
def test_step_dot_product(levels):
    """<J v, w> = <v, J^T w> for one explicit iteration (D, S, Y, lambda) -> (L, S', Y'):
    forward-mode derivatives (torch.func.jvp) against reverse-mode ones
    (torch.autograd), both in float64, for random tangents v and cotangents w."""
    import torch
    from torch.func import jvp
    w = synth.gaussian_lowrank_plus_sparse(64, 48, 3, seed=5, sparse_frac=0.05, levels=levels)
    rng = np.random.default_rng(11)
    m, n = w.D.shape
    D = torch.tensor(w.D.astype(np.float64))
    S = torch.tensor(0.05 * rng.normal(size=(m, n)))
    Y = torch.tensor(np.clip(0.2 * rng.normal(size=(m, n)), -w.lam, w.lam))
    lam = torch.tensor(w.lam, dtype=torch.float64)
    mu = 3.0 * w.mu0
    R = U.restriction(n, levels)
    v = [torch.tensor(rng.normal(size=(m, n))) for _ in range(3)] + [torch.tensor(0.7, dtype=torch.float64)]
    c = [torch.tensor(rng.normal(size=(m, n))) for _ in range(3)]

    def f(D_, S_, Y_, l_):
        return U.step(D_, S_, Y_, l_, mu, R)

    _, Jv = jvp(f, (D, S, Y, lam), tuple(v))
    ins = [t.clone().requires_grad_(True) for t in (D, S, Y, lam)]
    outs = f(*ins)
    JTw = torch.autograd.grad(outs, ins, grad_outputs=c)
    lhs = sum(float((a * b).sum()) for a, b in zip(Jv, c))
    rhs = sum(float((a * b).sum()) for a, b in zip(v, JTw))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), abs(rhs)), (lhs, rhs)
