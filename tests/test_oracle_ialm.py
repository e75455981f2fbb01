"""Pins of the oracle's inexact ALM (Alg. 1), multilevel inexact ALM (Alg. 4)
and its masked (compressive) form, against what the paper and convex analysis
fix: exact recovery, Lemma 1 optimality invariants at every iteration, the
Lyapunov inequality of Lemma 4 (eq. b_k), KKT certificates at convergence and
exact special-case reductions."""
import math

import numpy as np
import pytest

import oracle
import synth


def _small_pcp(m=120, n=100, rank=5, seed=11, frac=0.05, observed=None):
    return synth.gaussian_lowrank_plus_sparse(m, n, rank, seed=seed, sparse_frac=frac,
                                              observed_frac=observed, levels=2)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_plain_exact_recovery_c1():
    # Thm. 1 (convergence of IALM) with the exact-recovery regime of PCP:
    # 300 x 300, rank 10, 5% gross errors is recovered exactly.
    w = synth.config("c1")
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=0, tol=1e-7)
    assert r.converged and r.fg <= 1e-7
    assert r.rank == 10
    assert _rel(r.L, w.L0) < 5e-6
    assert _rel(r.S, w.S0) < 5e-6


def test_multilevel_recovers_when_assumption3_holds():
    # Assumption 3 (L* = L_H* R^T) made exact: rows of L0 lie in range(P).
    # Then the coarse model loses nothing and ML-IALM recovers L0 (Thm. 3 with
    # epsilon = Delta = 0 for the orthonormal restriction).
    n, lv = 120, 2
    P = oracle.composite_interp(n, lv)
    w = synth.range_conforming_lowrank_plus_sparse(150, n, 5, P, seed=5, sparse_frac=0.05, levels=lv)
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=lv, tol=1e-8)
    assert r.converged
    assert r.rank == 5
    assert _rel(r.L, w.L0) < 1e-5
    assert _rel(r.S, w.S0) < 1e-5


def test_levels_zero_equals_identity_restriction():
    w = _small_pcp()
    a = oracle.ialm(w.D, w.lam, w.mu0, levels=0, fixed_iters=12)
    b = oracle.ialm(w.D, w.lam, w.mu0, R=np.eye(w.n), fixed_iters=12)
    assert np.allclose(a.L, b.L, rtol=0, atol=1e-12)
    assert np.allclose(a.S, b.S, rtol=0, atol=1e-12)


@pytest.mark.parametrize("levels", [0, 2])
def test_full_mask_equals_pcp(levels):
    # CPCP with Q = the entire space is PCP (Sec. 2).
    w = _small_pcp()
    a = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, fixed_iters=15)
    b = oracle.ialm(w.D, w.lam, w.mu0, Q=np.ones(w.D.shape, bool), levels=levels, fixed_iters=15)
    assert np.array_equal(a.L, b.L) and np.array_equal(a.S, b.S) and np.array_equal(a.Y, b.Y)


@pytest.mark.parametrize("levels,observed", [(0, None), (2, None), (0, 0.6), (2, 0.6)])
def test_lemma1_sparse_optimality_every_iteration(levels, observed):
    # Lemma 1.2 (with its typo read as the subdifferential of lam||S||_1):
    # Y^{k+1} in d(lam ||S^{k+1}||_1): |Y| <= lam everywhere and Y = lam sign(S)
    # where S != 0.  Masked form: S = 0 and Y = 0 off Q.
    w = _small_pcp(observed=observed)
    r = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=levels, fixed_iters=20, keep_iterates=True)
    for h in r.history:
        Y, S = h["Y"], h["S"]
        assert np.abs(Y).max() <= w.lam * (1 + 1e-10)
        nz = S != 0
        assert np.allclose(Y[nz], w.lam * np.sign(S[nz]), rtol=1e-9, atol=0)
        if w.Q is not None:
            assert not S[~w.Q].any() and not Y[~w.Q].any()


@pytest.mark.parametrize("levels", [0, 2])
def test_lemma1_coarse_optimality_every_iteration(levels):
    # Lemma 1.1 with R^T R = I:  Yhat R in d||L_H||_*, where
    # Yhat^{k+1} = Y^k + mu_k (D - S^k - L^{k+1})  (eq. Yhat).  For
    # L_H = U_r Sig V_r^T this means Yhat R = U_r V_r^T + W, U_r^T W = 0,
    # W V_r = 0, ||W||_2 <= 1.
    w = _small_pcp()
    R = np.eye(w.n) if levels == 0 else oracle.orthonormal_restriction(w.n, levels)
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, fixed_iters=20, keep_iterates=True)
    checked = 0
    for h in r.history:
        G = h["Yhat"] @ R
        U, V = h["Ur"], h["Vr"]
        if U.shape[1] == 0:
            assert np.linalg.norm(G, 2) <= 1 + 1e-9
            continue
        W = G - U @ V.T
        assert np.abs(U.T @ W).max() < 1e-8
        assert np.abs(W @ V).max() < 1e-8
        assert np.linalg.norm(W, 2) <= 1 + 1e-8
        checked += 1
    assert checked > 5


def test_feasibility_gap_identity():
    # Proof of Thm. 3: ||D - L^k - S^k||_F = mu_{k-1}^{-1} ||Y^k - Y^{k-1}||_F.
    w = _small_pcp()
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=2, fixed_iters=15, keep_iterates=True)
    D = w.D.astype(np.float64)
    for h in r.history:
        lhs = np.linalg.norm(D - h["L"] - h["S"])
        rhs = np.linalg.norm(h["Y"] - h["Yprev"]) / h["mu"]
        assert abs(lhs - rhs) <= 1e-10 * max(lhs, 1e-300) + 1e-14
        assert abs(h["fg"] - lhs / np.linalg.norm(D)) <= 1e-12


@pytest.mark.parametrize("levels", [0, 2])
def test_lyapunov_monotone(levels):
    # Lemma 4, eq. (b_k) with epsilon = 0 and Delta = 0 (orthonormal restriction):
    # ||S^{k+1} - S*||^2 + mu_{k+1}^{-2}||Y^{k+1} - Y*||^2 is non-increasing,
    # for a saddle point (S*, Y*) of the (coarse-constrained) problem, taken
    # from a long run.  The penalty is uncapped here only in the sense that the
    # comparison uses the mu actually used at each step.
    w = _small_pcp()
    star = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, tol=1e-12, max_iter=400)
    assert star.fg < 1e-9
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, fixed_iters=25, keep_iterates=True)
    mus = [h["mu"] for h in r.history]
    phi = []
    for k, h in enumerate(r.history):
        mu_next = min(1.5 * mus[k], 1e7 * w.mu0)
        phi.append(np.sum((h["S"] - star.S) ** 2) + np.sum((h["Y"] - star.Y) ** 2) / mu_next ** 2)
    scale = phi[0]
    for a, b in zip(phi, phi[1:]):
        assert b <= a + 1e-9 * scale


def _nuc(A):
    return np.linalg.svd(A, compute_uv=False).sum()


@pytest.mark.parametrize("levels", [0, 2])
def test_converged_point_minimises_pcp_objective(levels):
    # eq. (rpca): min ||L||_* + lam ||S||_1 s.t. D = L + S (for levels > 0 also
    # L = L R~ R~^T, the coarse-model constraint).  Convex, so a point that no
    # feasible direction improves is the global minimiser.  Feasible moves:
    # (L + tE, S - tE) with E in the row range of the restriction.
    w = _small_pcp()
    # (with mu capped at 1e7 mu_0 the gap stalls near 1e-10, so stop at 1e-9)
    r = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, tol=1e-9, max_iter=400)
    assert r.converged
    D = w.D.astype(np.float64)
    assert np.linalg.norm(D - r.L - r.S) <= 1e-9 * np.linalg.norm(D)
    R = np.eye(w.n) if levels == 0 else oracle.orthonormal_restriction(w.n, levels)
    L = r.L
    S = D - L                              # exact feasibility (moves S by ~1e-9)

    def f(Lx, Sx):
        return _nuc(Lx) + w.lam * np.abs(Sx).sum()

    f0 = f(L, S)
    rng = np.random.default_rng(0)
    for t in (1e-2, 1e-4):
        for _ in range(40):
            E = rng.normal(size=D.shape) @ R @ R.T
            E *= t / np.linalg.norm(E)
            assert f(L + E, S - E) >= f0 - 1e-7 * f0
    # and the multiplier bound of Lemma 1.2; rounding of Y + mu (D - L - S)
    # grows like mu * eps * |D|
    assert np.abs(r.Y).max() <= w.lam + r.mu * 1e-14 * np.abs(D).max()


def test_converged_point_minimises_cpcp_objective():
    # Constrained CPCP (Sec. 2): P_Q[L + S] = P_Q[D] with S supported on Q.
    # Feasible moves: (L + tE, S - t P_Q E).  Y vanishes off Q.
    w = _small_pcp(observed=0.7)
    r = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=0, tol=1e-9, max_iter=400)
    assert r.converged
    D = w.D.astype(np.float64)
    assert np.linalg.norm(np.where(w.Q, D - r.L - r.S, 0)) <= 1e-9 * np.linalg.norm(np.where(w.Q, D, 0))
    assert not r.Y[~w.Q].any() and not r.S[~w.Q].any()
    L = r.L
    S = np.where(w.Q, D - L, 0.0)

    def f(Lx, Sx):
        return _nuc(Lx) + w.lam * np.abs(Sx).sum()

    f0 = f(L, S)
    rng = np.random.default_rng(1)
    for t in (1e-2, 1e-4):
        for _ in range(40):
            E = rng.normal(size=D.shape)
            E *= t / np.linalg.norm(E)
            assert f(L + E, S - np.where(w.Q, E, 0.0)) >= f0 - 1e-7 * f0


def test_masked_recovers_low_rank_from_partial_observations():
    # Compressive PCP with 70% observed entries and 5% gross errors still
    # recovers the low-rank part (plain path).
    w = _small_pcp(m=200, n=160, rank=4, observed=0.7)
    r = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=0, tol=1e-8)
    assert r.converged and r.rank == 4
    assert _rel(r.L, w.L0) < 1e-4


def test_warm_start_resume():
    # S^(0), Y^(0) are inputs (Alg. 1): resuming from the iterate after k steps
    # with mu_k continues the same sequence.
    w = _small_pcp()
    full = oracle.ialm(w.D, w.lam, w.mu0, levels=2, fixed_iters=10)
    first = oracle.ialm(w.D, w.lam, w.mu0, levels=2, fixed_iters=6)
    mu6 = min(1.5 * first.mu, 1e7 * w.mu0)
    rest = oracle.ialm(w.D, w.lam, mu6, levels=2, fixed_iters=4, S0=first.S, Y0=first.Y,
                       mu_max_factor=1e7 * w.mu0 / mu6)
    assert np.allclose(rest.L, full.L, atol=1e-12) and np.allclose(rest.S, full.S, atol=1e-12)


def test_penalty_schedule():
    mus = oracle.default_schedule(2.0, 50)
    assert mus[0] == 2.0 and mus[1] == 3.0
    assert all(b >= a for a, b in zip(mus, mus[1:]))
    assert max(mus) == pytest.approx(2.0e7)
