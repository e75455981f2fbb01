"""Pins of the oracle's proximal maps: soft threshold and singular value
thresholding (Alg. 1 steps), and the coarse SVT of Alg. 4 against a direct
minimisation of the coarse augmented Lagrangian (eq. coarse-aug-lagr)."""
import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar

import oracle


def test_shrink_brute_force_1d():
    # S_tau[x] = argmin_s 0.5 (s - x)^2 + tau |s|, found by a bounded scalar search
    rng = np.random.default_rng(0)
    for _ in range(200):
        x = rng.normal() * 3
        tau = rng.uniform(0.01, 2.0)
        res = minimize_scalar(lambda s: 0.5 * (s - x) ** 2 + tau * abs(s),
                              bounds=(-20, 20), method="bounded", options={"xatol": 1e-12})
        assert abs(oracle.shrink(x, tau) - res.x) < 1e-6


def test_shrink_special_values():
    x = np.array([-3.0, -1.0, -0.5, 0.0, 0.5, 1.0, 3.0])
    assert np.array_equal(oracle.shrink(x, 1.0), np.array([-2.0, 0, 0, 0, 0, 0, 2.0]))
    assert np.array_equal(oracle.shrink(x, 0.0), x)


def test_svt_diagonal_closed_form():
    d = np.array([5.0, 3.0, 1.0, 0.2])
    M = np.zeros((6, 4))
    M[:4, :4] = np.diag(d)
    L, r, _ = oracle.svt(M, 0.5)
    E = np.zeros((6, 4))
    E[:4, :4] = np.diag([4.5, 2.5, 0.5, 0.0])
    assert r == 3
    assert np.allclose(L, E, atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_svt_subgradient_certificate(seed):
    # L = SVT_tau(M) iff M - L in tau * d||L||_*, i.e. M - L = tau (U V^T + W)
    # with U^T W = 0, W V = 0, ||W||_2 <= 1 (U, V singular vectors of L).
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(30, 12)) + 3 * rng.normal(size=(30, 2)) @ rng.normal(size=(2, 12))
    tau = 2.0
    L, r, _ = oracle.svt(M, tau)
    U, s, Vt = np.linalg.svd(L, full_matrices=False)
    U, V = U[:, :r], Vt[:r].T
    W = (M - L) / tau - U @ V.T
    assert np.abs(U.T @ W).max() < 1e-10
    assert np.abs(W @ V).max() < 1e-10
    assert np.linalg.norm(W, 2) <= 1 + 1e-10


@pytest.mark.parametrize("seed", range(3))
def test_svt_is_minimiser_under_perturbation(seed):
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(15, 10))
    tau = 1.0

    def F(X):
        return 0.5 * np.sum((X - M) ** 2) + tau * np.linalg.svd(X, compute_uv=False).sum()

    L = oracle.svt(M, tau)[0]
    f0 = F(L)
    for _ in range(50):
        E = rng.normal(size=M.shape)
        assert F(L + 1e-3 * E / np.linalg.norm(E)) >= f0 - 1e-12


def test_svt_brute_force_tiny():
    # direct minimisation of 0.5||X - M||^2 + tau ||X||_* over 3 x 2 matrices
    rng = np.random.default_rng(7)
    M = rng.normal(size=(3, 2)) * 2
    tau = 0.7

    def F(x):
        X = x.reshape(3, 2)
        return 0.5 * np.sum((X - M) ** 2) + tau * np.linalg.svd(X, compute_uv=False).sum()

    best = None
    for start in (M.ravel(), np.zeros(6), rng.normal(size=6)):
        res = minimize(F, start, method="Powell", options={"xtol": 1e-10, "ftol": 1e-14, "maxfev": 200000})
        res = minimize(F, res.x, method="Nelder-Mead", options={"xatol": 1e-10, "fatol": 1e-15, "maxfev": 200000})
        if best is None or res.fun < best.fun:
            best = res
    L = oracle.svt(M, tau)[0]
    assert F(L.ravel()) <= best.fun + 1e-9
    assert np.allclose(L.ravel(), best.x, atol=1e-4)


def test_coarse_step_minimises_coarse_augmented_lagrangian():
    # Alg. 4: L_H = U_H S_{1/mu}[Sigma_H] V_H^T with U_H Sigma_H V_H^T = (D - S + Y/mu) R
    # must minimise the coarse augmented Lagrangian of eq. (coarse-aug-lagr):
    #   ||L||_* + lam||S||_1 + <Y, [(D - S)R - L] R^T> + mu/2 ||(D - S)R - L||_F^2
    # written out term by term and minimised directly over a tiny coarse L.
    rng = np.random.default_rng(3)
    m, n, lv = 3, 4, 1
    R = oracle.orthonormal_restriction(n, lv)
    nH = R.shape[1]
    D = rng.normal(size=(m, n))
    S = rng.normal(size=(m, n)) * 0.3
    Y = rng.normal(size=(m, n)) * 0.5
    mu, lam = 1.7, 0.4

    def LHfun(x):
        LH = x.reshape(m, nH)
        A = (D - S) @ R - LH
        return (np.linalg.svd(LH, compute_uv=False).sum() + lam * np.abs(S).sum()
                + np.sum(Y * (A @ R.T)) + 0.5 * mu * np.sum(A ** 2))

    best = None
    for start in (np.zeros(m * nH), ((D - S) @ R).ravel(), rng.normal(size=m * nH)):
        res = minimize(LHfun, start, method="Powell", options={"xtol": 1e-11, "ftol": 1e-15, "maxfev": 400000})
        res = minimize(LHfun, res.x, method="Nelder-Mead", options={"xatol": 1e-11, "fatol": 1e-15, "maxfev": 400000})
        if best is None or res.fun < best.fun:
            best = res
    MH = (D - S + Y / mu) @ R
    LH, _, _ = oracle.svt(MH, 1.0 / mu)
    assert LHfun(LH.ravel()) <= best.fun + 1e-9
    assert np.allclose(LH.ravel(), best.x, atol=1e-4)
    # and the lifted step equals the oracle's svt_prox
    Lf, _ = oracle.svt_prox(D - S + Y / mu, 1.0 / mu, lv)
    assert np.allclose(Lf, LH @ R.T, atol=1e-13)


def test_coarse_svt_equals_svt_of_projected_data():
    # With R~ orthonormal, SVT(M R~) R~^T = SVT(M R~ R~^T): the lift commutes with
    # thresholding (a plausible mistake -- lifting with P instead of R~, or not
    # lifting at all -- breaks it).
    rng = np.random.default_rng(4)
    M = rng.normal(size=(40, 24))
    R = oracle.orthonormal_restriction(24, 2)
    L1, r1 = oracle.svt_prox(M, 0.8, 2)
    L2, r2, _ = oracle.svt(M @ R @ R.T, 0.8)
    assert r1 == r2
    assert np.allclose(L1, L2, atol=1e-12)
