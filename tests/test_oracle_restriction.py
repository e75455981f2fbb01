"""Pins of the oracle's restriction operators (Sec. 3.1, eq. (Rx), Thm. LH-eps).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own construction."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_n6_exact():
    # Sec. 3.1 worked example: the printed 6 x 3 operator, entry by entry.
    P6 = np.loadtxt(os.path.join(GOLDEN, "interp_n6.txt"))
    assert np.array_equal(oracle.interp_level(6), P6)


def test_worked_example_rank_one_background():
    # Sec. 3.1: a matrix of ones on the coarse grid lifts to ones on the fine grid.
    P6 = np.loadtxt(os.path.join(GOLDEN, "interp_n6.txt"))
    LH = np.ones((7, 3))
    assert np.array_equal(LH @ oracle.interp_level(6).T, np.ones((7, 6)))
    assert np.array_equal(LH @ P6.T, np.ones((7, 6)))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 13, 25, 50, 100, 101, 200, 250, 400])
def test_single_level_structure(n):
    P = oracle.interp_level(n)
    nH = oracle.coarse_dim(n, 1)
    assert P.shape == (n, nH)
    assert nH == (n + 1) // 2
    # interpolation weights: each fine point is a convex combination of coarse points
    assert np.allclose(P.sum(axis=1), 1.0, atol=0, rtol=0)
    assert set(np.unique(P)).issubset({0.0, 0.5, 1.0})
    assert (np.count_nonzero(P, axis=1) <= 2).all()
    # Assumption 1: linearly independent columns
    assert np.linalg.matrix_rank(P) == nH


@pytest.mark.parametrize("n", [4, 6, 8, 50, 100, 250, 400, 2000])
def test_condition_bound_one_level(n):
    # Sec. 3.1 (after Thm. LH-eps): sigma_1(R) / sigma_nH(R) <= 2 for the
    # interpolation operator.
    s = np.linalg.svd(oracle.interp_level(n), compute_uv=False)
    assert s[0] / s[-1] <= 2.0


@pytest.mark.parametrize("n,levels,nH", [(300, 2, 75), (2000, 3, 250), (400, 3, 50), (1000, 2, 250),
                                         (200, 4, 13), (25, 1, 13), (7, 2, 2)])
def test_composite_dims(n, levels, nH):
    assert oracle.coarse_dim(n, levels) == nH
    P = oracle.composite_interp(n, levels)
    assert P.shape == (n, nH)
    # composite of interpolations still interpolates: rows sum to one
    assert np.allclose(P.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert np.linalg.matrix_rank(P) == nH


def test_composite_is_product_of_levels():
    # The multi-level operator is the product of single-level ones (Sec. 3.1).
    P = oracle.interp_level(200) @ oracle.interp_level(100) @ oracle.interp_level(50) @ oracle.interp_level(25)
    assert np.array_equal(oracle.composite_interp(200, 4), P)


def test_composite_piecewise_linear_reproduces_linear_functions():
    # Interpolation reproduces affine data: lifting coarse samples of a linear
    # function gives a fine function with slope 1/2^levels, except at the start,
    # where each level repeats its first point (the duplicated first row of the
    # worked example), so the first 2^levels fine values are flat.
    n, lv = 64, 3
    P = oracle.composite_interp(n, lv)
    f = P @ np.arange(P.shape[1], dtype=float)
    d = np.diff(f)
    flat = 2 ** lv - 1
    assert np.allclose(d[:flat - 1], 0.0)
    assert np.allclose(d[flat:], 1.0 / 2 ** lv)


@pytest.mark.parametrize("n,levels", [(300, 2), (2000, 3), (400, 3), (200, 4), (25, 1)])
def test_orthonormal_restriction_range_and_orthonormality(n, levels):
    R = oracle.orthonormal_restriction(n, levels)
    P = oracle.composite_interp(n, levels)
    nH = P.shape[1]
    assert np.allclose(R.T @ R, np.eye(nH), atol=1e-12)
    # same column range as P: least-squares projection onto range(P) (an
    # independent route) equals R R^T
    rng = np.random.default_rng(0)
    X = rng.normal(size=(n, 5))
    coef = np.linalg.lstsq(P, X, rcond=None)[0]
    assert np.allclose(P @ coef, R @ (R.T @ X), atol=1e-10)
    # symmetric orthogonalisation: R^T P is symmetric positive definite
    M = R.T @ P
    assert np.allclose(M, M.T, atol=1e-12)
    assert np.linalg.eigvalsh(M).min() > 0


def test_levels_zero_is_identity():
    assert np.array_equal(oracle.orthonormal_restriction(10, 0), np.eye(10))
    X = np.arange(12.0).reshape(3, 4)
    assert np.array_equal(oracle.restrict(X, 0), X)


def test_restrict_prolong_adjoint():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(9, 50))
    Z = rng.normal(size=(9, oracle.coarse_dim(50, 2)))
    lhs = np.sum(oracle.restrict(X, 2) * Z)
    rhs = np.sum(X * oracle.prolong(Z, 50, 2))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def _nuc(A):
    return np.linalg.svd(A, compute_uv=False).sum()


@pytest.mark.parametrize("seed", range(4))
def test_theorem_LH_eps(seed):
    # Thm. LH-eps: ||L_H R^T||_* >= ||L_H||_* - eps with
    # eps = sum_k sigma_k(L_H)(1 - sigma_{nH-k+1}(R)), and <= ||L_H||_* when
    # ||R||_2 <= 1.  For the orthonormal R~ both hold with equality (eps = 0).
    rng = np.random.default_rng(seed)
    n, lv, m = 40, 2, 60
    P = oracle.composite_interp(n, lv)
    nH = P.shape[1]
    LH = rng.normal(size=(m, 3)) @ rng.normal(size=(3, nH))
    Rs = P / np.linalg.norm(P, 2)
    sR = np.linalg.svd(Rs, compute_uv=False)
    sL = np.linalg.svd(LH, compute_uv=False)
    rH = np.linalg.matrix_rank(LH)
    eps = sum(sL[k] * (1 - sR[nH - k - 1]) for k in range(rH))
    assert _nuc(LH @ Rs.T) >= _nuc(LH) - eps - 1e-10
    assert _nuc(LH @ Rs.T) <= _nuc(LH) + 1e-10
    Ro = oracle.orthonormal_restriction(n, lv)
    assert abs(_nuc(LH @ Ro.T) - _nuc(LH)) <= 1e-10 * _nuc(LH)
