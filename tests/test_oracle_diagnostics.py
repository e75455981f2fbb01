"""Pins of the multilevel diagnostics (Thm. LH-eps, Lemma 3) and of the oracle with the
literal interpolation operator.

* Thm. LH-eps holds: ||L_H R^T||_* >= ||L_H||_* - eps on random inputs for the literal
  operator (scaled and not), and is tight, with the closed form eps = (1 - c) ||L_H||_*,
  for R = c R~ (every singular value of R equal to c); eps = 0 for orthonormal R.
* Delta vanishes for orthonormal R and equals (c^2 - 1) <L_H, L_H - L_H*> for R = c R~.
* One interpolation operator (eq. Rx) has sigma_1 / sigma_{n_H} <= 2 (the remark after
  Thm. LH-eps), so P / ||P||_2 has its singular values in [1/2, 1]; the composite of
  three or more levels exceeds 2 slightly (2.096 at 3 levels), recorded here.
* The oracle with an explicit R: R = c R~ turns the coarse model into a scaled one, and
  with c = 1 it is the default multilevel solve.
"""
import numpy as np
import pytest

import oracle
from oracle import diagnostics as dg
from oracle.restriction import orthonormal_restriction


def _nuc(A):
    return float(np.linalg.svd(A, compute_uv=False).sum())


@pytest.mark.parametrize("n,levels", [(16, 2), (30, 1), (64, 3), (25, 2)])
@pytest.mark.parametrize("scaled", [True, False])
def test_epsilon_bound_holds(n, levels, scaled):
    rng = np.random.default_rng(n + levels)
    R = dg.literal_restriction(n, levels, scaled)
    nH = R.shape[1]
    for r in (1, 3, nH):
        LH = rng.normal(size=(40, r)) @ rng.normal(size=(r, nH))
        eps = dg.epsilon(LH, R)
        assert _nuc(LH @ R.T) >= _nuc(LH) - eps - 1e-9 * _nuc(LH)


def test_epsilon_tight_and_delta_closed_forms():
    rng = np.random.default_rng(3)
    Rt = orthonormal_restriction(32, 2)
    nH = Rt.shape[1]
    LH = rng.normal(size=(20, 4)) @ rng.normal(size=(4, nH))
    LHs = rng.normal(size=(20, nH))
    assert abs(dg.epsilon(LH, Rt)) < 1e-12 * _nuc(LH)
    assert abs(dg.delta(LH, LHs, Rt)) < 1e-10 * np.linalg.norm(LH) ** 2
    for c in (0.5, 0.9):
        R = c * Rt
        eps = dg.epsilon(LH, R)
        assert np.isclose(eps, (1 - c) * _nuc(LH), rtol=1e-10)
        assert np.isclose(_nuc(LH @ R.T), _nuc(LH) - eps, rtol=1e-10)
        assert np.isclose(dg.delta(LH, LHs, R), (c * c - 1) * np.sum(LH * (LH - LHs)), rtol=1e-10)


@pytest.mark.parametrize("n", [6, 7, 64, 300, 2000, 401])
def test_interpolation_singular_value_ratio(n):
    s = np.linalg.svd(dg.literal_restriction(n, 1, scaled=False), compute_uv=False)
    assert s[0] / s[-1] <= 2.0 + 1e-12
    t = np.linalg.svd(dg.literal_restriction(n, 1, scaled=True), compute_uv=False)
    assert np.isclose(t[0], 1.0) and t[-1] >= 0.5 - 1e-12


def test_composite_singular_value_ratio():
    ratio = {}
    for levels in (2, 3, 4):
        s = np.linalg.svd(dg.literal_restriction(2000, levels, scaled=False), compute_uv=False)
        ratio[levels] = s[0] / s[-1]
    assert ratio[2] <= 2.0 and 2.09 < ratio[3] < 2.10 and ratio[4] > 2.0


def test_oracle_with_explicit_restriction():
    rng = np.random.default_rng(4)
    m, n = 60, 32
    D = rng.normal(size=(m, 3)) @ rng.normal(size=(3, n)) / 3
    D[rng.random((m, n)) < 0.05] += 2.0
    lam = 1 / np.sqrt(m)
    Rt = orthonormal_restriction(n, 2)
    a = oracle.ialm(D, lam, 0.5, levels=2, fixed_iters=6)
    b = oracle.ialm(D, lam, 0.5, levels=2, fixed_iters=6, R=Rt)
    assert np.allclose(a.L, b.L, atol=1e-13) and np.allclose(a.S, b.S, atol=1e-13)
    # the coarse iterates are recorded and lift to L
    h = oracle.ialm(D, lam, 0.5, levels=2, fixed_iters=3, keep_iterates=True).history
    assert all(np.allclose(x["LH"] @ Rt.T, x["L"], atol=1e-12) for x in h)
