"""Pins of the FP64 Frank-Wolfe Thresholding oracle (Alg. 3, Alg. 6) against facts
that do not come from the oracle itself:

* the exact line search against a dense grid and scipy's bounded minimiser;
* the linear oracles against their support-function values and brute force over
  the extreme points of the nuclear and l1 balls;
* the monotone decrease of f that the exact line search and the proximal threshold
  guarantee (the line search contains the step (0, 0); the threshold is the proximal
  step of the S-block with step 1/Lipschitz);
* weak duality against an independent solver of eq. (cpcp): accelerated proximal
  gradient (FISTA with singular value thresholding, written here), giving F*;
  every FW iterate satisfies F* <= F(L, S) <= f <= F* + gap and the sublinear bound
  of the FW theorem with Lipschitz constant 2 and the diameter bound of the epigraph
  reformulation.  For ML-FWT the same holds with the optimum over matrices whose
  rows lie in range(R) (Thm. for ML-FW);
* the l1-free case (lam_S above every residual, Q = all): the optimum is the SVT of D,
  a closed form;
* the gradient identity behind the clipped evaluation of G.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle.fwt as fw
from oracle.prox import shrink, svt
from oracle.restriction import composite_interp, orthonormal_restriction


def _problem(m=30, n=20, r=2, seed=0, obs=0.8, sparse=0.05, delta=0.05):
    rng = np.random.default_rng(seed)
    L0 = rng.normal(size=(m, r)) @ rng.normal(size=(r, n))
    S0 = np.zeros(m * n)
    idx = rng.choice(m * n, int(sparse * m * n), replace=False)
    S0[idx] = rng.uniform(-5, 5, idx.size)
    D = L0 + S0.reshape(m, n)
    Q = rng.random((m, n)) < obs
    lam_L = delta * np.linalg.norm(np.where(Q, D, 0.0), 2)
    lam_S = lam_L / np.sqrt(max(m, n))
    return D, Q, lam_L, lam_S


def _fista(D, Q, lam_L, lam_S, iters=4000, R=None):
    """min 1/2 ||P_Q[L + S - D]||^2 + lam_L ||L||_* + lam_S ||S||_1 by accelerated
    proximal gradient on (X, S), L = X (or X R^T with orthonormal R, where
    ||X R^T||_* = ||X||_*).  The smooth part has a 2-Lipschitz gradient: step 1/2."""
    m, n = D.shape
    X = np.zeros((m, n if R is None else R.shape[1]))
    S = np.zeros((m, n))
    Yx, Ys, t = X.copy(), S.copy(), 1.0
    for _ in range(iters):
        L = Yx if R is None else Yx @ R.T
        G = np.where(Q, L + Ys - D, 0.0)
        gx = G if R is None else G @ R
        Xn = svt(Yx - gx / 2.0, lam_L / 2.0)[0]
        Sn = shrink(Ys - G / 2.0, lam_S / 2.0)
        tn = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        Yx = Xn + ((t - 1.0) / tn) * (Xn - X)
        Ys = Sn + ((t - 1.0) / tn) * (Sn - S)
        X, S, t = Xn, Sn, tn
    L = X if R is None else X @ R.T
    return fw.cpcp_value(D, Q, L, S, lam_L, lam_S)


# ---- line search --------------------------------------------------------------------

def _phi(c, a, b):
    haa, hab, hbb, ga, gb = c
    return 0.5 * (haa * a * a + 2 * hab * a * b + hbb * b * b) + ga * a + gb * b


def _random_qps(rng, count):
    out = []
    for k in range(count):
        M = rng.normal(size=(2, 2)) * rng.uniform(0.1, 10)
        H = M @ M.T
        if k % 5 == 0:                    # singular Hessian
            v = rng.normal(size=2)
            H = np.outer(v, v)
        if k % 7 == 0:                    # one direction without curvature
            H = np.diag([rng.uniform(0.1, 5), 0.0])
        g = rng.normal(size=2) * rng.uniform(0.1, 20)
        out.append((H[0, 0], H[0, 1], H[1, 1], g[0], g[1]))
    return out


def test_box_qp_beats_grid_and_matches_scipy():
    rng = np.random.default_rng(7)
    grid = np.linspace(0.0, 1.0, 401)
    A, B = np.meshgrid(grid, grid, indexing="ij")
    for c in _random_qps(rng, 60):
        a, b = fw.box_qp(*c)
        assert 0.0 <= a <= 1.0 and 0.0 <= b <= 1.0
        v = _phi(c, a, b)
        assert v <= _phi(c, A, B).min() + 1e-12 * (1 + abs(v))
        res = minimize(lambda x: _phi(c, x[0], x[1]), x0=[0.5, 0.5], bounds=[(0, 1), (0, 1)],
                       method="L-BFGS-B", options=dict(ftol=1e-15, gtol=1e-12))
        assert v <= res.fun + 1e-9 * (1 + abs(res.fun))


def test_box_qp_interior_and_degenerate():
    # interior optimum of a strictly convex quadratic: the stationary point
    a, b = fw.box_qp(2.0, 0.5, 1.0, -0.6, -0.3)
    x = np.linalg.solve([[2.0, 0.5], [0.5, 1.0]], [0.6, 0.3])
    assert np.allclose([a, b], x, atol=1e-15)
    # nothing to gain: the origin
    assert fw.box_qp(0.0, 0.0, 0.0, 0.0, 0.0) == (0.0, 0.0)
    # pure descent along a without curvature: the far edge
    assert fw.box_qp(0.0, 0.0, 1.0, -1.0, 0.0) == (1.0, 0.0)


# ---- linear oracles -------------------------------------------------------------------

def test_nuclear_lmo_support_function_and_extreme_points():
    rng = np.random.default_rng(3)
    G = rng.normal(size=(9, 6))
    u, v, val = fw.nuclear_lmo(G)
    M = -np.outer(u, v)
    assert np.isclose(np.sum(G * M), val, rtol=1e-13)
    assert np.isclose(val, -np.linalg.norm(G, 2), rtol=1e-13)
    assert np.isclose(np.linalg.svd(M, compute_uv=False).sum(), 1.0, rtol=1e-13)
    # extreme points of the unit nuclear ball are x y^T with unit x, y
    for _ in range(2000):
        x = rng.normal(size=9)
        y = rng.normal(size=6)
        x /= np.linalg.norm(x)
        y /= np.linalg.norm(y)
        assert np.sum(G * np.outer(x, y)) >= val - 1e-12


def test_coarse_nuclear_lmo():
    rng = np.random.default_rng(4)
    G = rng.normal(size=(12, 16))
    R = orthonormal_restriction(16, 2)
    u, w, val = fw.coarse_nuclear_lmo(G, R)
    M = -np.outer(u, w)
    assert np.isclose(np.sum(G * M), val, rtol=1e-12)
    assert np.isclose(val, -np.linalg.norm(G @ R, 2), rtol=1e-12)
    assert np.linalg.svd(M, compute_uv=False).sum() <= 1.0 + 1e-12      # feasible for the fine ball
    assert val >= fw.nuclear_lmo(G)[2] - 1e-12                         # a restricted oracle
    nH = R.shape[1]
    for _ in range(2000):                                              # coarse extreme points, lifted
        x = rng.normal(size=12)
        y = rng.normal(size=nH)
        x /= np.linalg.norm(x)
        y /= np.linalg.norm(y)
        assert np.sum(G * np.outer(x, R @ y)) >= val - 1e-12
    # a restriction that is not orthonormal (the literal interpolation operator,
    # ||P||_2 > 1): the radius 1/||P||_2 keeps the lifted atom in the unit ball
    P = composite_interp(16, 2)
    p2 = np.linalg.norm(P, 2)
    assert p2 > 1.5
    u3, w3, val3 = fw.coarse_nuclear_lmo(G, P)
    M3 = -np.outer(u3, w3)
    assert np.isclose(np.sum(G * M3), val3, rtol=1e-12)
    assert np.isclose(val3, -np.linalg.norm(G @ P, 2) / p2, rtol=1e-12)
    assert np.linalg.svd(M3, compute_uv=False).sum() <= 1.0 + 1e-12
    # identity restriction: the fine oracle
    u2, w2, val2 = fw.coarse_nuclear_lmo(G, np.eye(16))
    u1, v1, val1 = fw.nuclear_lmo(G)
    assert np.isclose(val1, val2, rtol=1e-13)
    assert np.allclose(np.outer(u1, v1), np.outer(u2, w2), atol=1e-12)


def test_l1_lmo_brute_force():
    rng = np.random.default_rng(5)
    G = rng.normal(size=(7, 5))
    i, j, sgn, val = fw.l1_lmo(G)
    best = min(s * G[a, b] for a in range(7) for b in range(5) for s in (-1.0, 1.0))
    assert np.isclose(val, best, rtol=1e-15)
    assert np.isclose(-sgn * G[i, j], best, rtol=1e-15)


# ---- the whole iteration ----------------------------------------------------------------

@pytest.mark.parametrize("levels", [0, 2])
def test_objective_monotone_and_bounds_feasible(levels):
    D, Q, lam_L, lam_S = _problem(seed=1, n=24)
    res = fw.fwt(D, lam_L, lam_S, Q=Q, levels=levels, fixed_iters=80, keep_iterates=True)
    f0 = 0.5 * float(np.sum(np.where(Q, D, 0.0) ** 2))
    prev = f0
    for h in res.history:
        assert h["f"] <= prev * (1 + 1e-13)
        prev = h["f"]
        nuc = np.linalg.svd(h["L"], compute_uv=False).sum()
        assert nuc <= h["t_L"] * (1 + 1e-10) + 1e-12              # epigraph constraint
        assert np.isclose(h["t_S"], np.abs(h["S"]).sum(), rtol=1e-14)
    # f at the returned iterate recomputed from its parts
    assert np.isclose(res.f, fw.objective(D, Q, res.L, res.S, res.t_L, res.t_S, lam_L, lam_S), rtol=1e-14)


def test_weak_duality_and_rate_against_fista():
    D, Q, lam_L, lam_S = _problem(seed=2)
    Fstar = _fista(D, Q, lam_L, lam_S)
    res = fw.fwt(D, lam_L, lam_S, Q=Q, fixed_iters=300, keep_iterates=True)
    f0 = 0.5 * float(np.sum(np.where(Q, D, 0.0) ** 2))
    diam2 = 5.0 * ((f0 / lam_L) ** 2 + (f0 / lam_S) ** 2)
    fprev = f0
    for h in res.history:
        # the gap of iteration k bounds f(x_k) - F* (x_k: the point before the step)
        assert fprev - Fstar <= h["gap"] * (1 + 1e-9) + 1e-9
        F = fw.cpcp_value(D, Q, h["L"], h["S"], lam_L, lam_S)
        assert Fstar - 1e-8 * abs(Fstar) <= F <= h["f"] * (1 + 1e-12)
        assert h["f"] - Fstar <= 2 * 2.0 * diam2 / (h["k"] + 2)
        fprev = h["f"]
    assert (res.f - Fstar) / Fstar < 0.05     # O(1/k) progress after 300 iterations


def test_ml_weak_duality_against_restricted_optimum():
    D, Q, lam_L, lam_S = _problem(seed=3, n=32)
    R = orthonormal_restriction(32, 2)
    FH = _fista(D, Q, lam_L, lam_S, R=R)
    Fstar = _fista(D, Q, lam_L, lam_S)
    assert FH >= Fstar - 1e-8 * Fstar          # a restricted problem
    res = fw.fwt(D, lam_L, lam_S, Q=Q, levels=2, fixed_iters=200, keep_iterates=True)
    fprev = 0.5 * float(np.sum(np.where(Q, D, 0.0) ** 2))
    for h in res.history:
        assert fprev - FH <= h["gap"] * (1 + 1e-9) + 1e-9
        assert np.allclose(h["L"], h["L"] @ R @ R.T, atol=1e-9 * (1 + np.abs(h["L"]).max()))  # rows in range(R)
        assert fw.cpcp_value(D, Q, h["L"], h["S"], lam_L, lam_S) >= FH - 1e-8 * FH
        fprev = h["f"]


def test_l1_free_case_reaches_svt_closed_form():
    rng = np.random.default_rng(6)
    D = rng.normal(size=(12, 3)) @ np.diag([5.0, 2.0, 1.0]) @ rng.normal(size=(3, 8))
    lam_L = 1.5
    lam_S = 1e6                                 # above every residual: S stays zero
    Lstar = svt(D, lam_L)[0]
    Fstar = 0.5 * np.sum((Lstar - D) ** 2) + lam_L * np.linalg.svd(Lstar, compute_uv=False).sum()
    res = fw.fwt(D, lam_L, lam_S, fixed_iters=2000)
    assert np.all(res.S == 0.0)
    assert res.f - Fstar >= -1e-9 * Fstar
    assert (res.f - Fstar) / Fstar < 1e-3
    assert np.linalg.norm(res.L - Lstar) / np.linalg.norm(Lstar) < 0.05


def test_clipped_gradient_identity():
    rng = np.random.default_rng(8)
    D = rng.normal(size=(20, 10)) * 3
    L = rng.normal(size=(20, 10))
    Q = rng.random((20, 10)) < 0.7
    lam_S = 0.8
    S_half = np.where(Q, rng.normal(size=(20, 10)), 0.0)
    S = shrink(S_half - np.where(Q, L + S_half - D, 0.0), lam_S)
    literal = np.where(Q, L + S - D, 0.0)
    clipped = np.where(Q, -np.clip(D - L, -lam_S, lam_S), 0.0)
    assert np.allclose(literal, clipped, atol=1e-14)
    assert np.all(S[~Q] == 0.0)


def test_zero_data():
    res = fw.fwt(np.zeros((5, 4)), 1.0, 0.5)
    assert res.iters == 0 and res.f == 0.0 and np.all(res.L == 0) and np.all(res.S == 0)


def test_tolerance_stop():
    D, Q, lam_L, lam_S = _problem(seed=9)
    res = fw.fwt(D, lam_L, lam_S, Q=Q, tol=1e-3)
    assert res.converged and res.history[-1]["rel_change"] <= 1e-3
    assert all(h["rel_change"] > 1e-3 for h in res.history[:-1])


@pytest.mark.parametrize("lam_L,lam_S", [(0.3, 0.7), (0.7, 0.3)])
def test_first_iteration_closed_form(lam_L, lam_S):
    """Alg. 3 from its initial point on D = d e_1 e_1^T (Q = all), worked by hand.
    Start: L = S = 0, t_L = t_S = 0, f_0 = d^2 / 2, U_L = f_0 / lam_L, U_S = f_0 / lam_S.
    G = -D, so both linear oracles return the atom e_1 e_1^T with <G, M> = -d; both
    gates open (lam < d).  Along V_L = U_L e_1 e_1^T and V_S = U_S e_1 e_1^T the
    objective is 1/2 (alpha U_L + beta U_S - d)^2 + lam_L alpha U_L + lam_S beta U_S, a
    function of x = alpha U_L + beta U_S plus a cost that makes the cheaper weight win:
    with lam_L < lam_S, x = d - lam_L on the alpha edge, alpha = (d - lam_L) / U_L, beta = 0;
    otherwise alpha = 0, beta = (d - lam_S) / U_S.  The Frank-Wolfe gap at the start is
    U_L (d - lam_L) + U_S (d - lam_S).  Step sizes and gap therefore fix both initial
    bounds (a swap of U_L and U_S changes them)."""
    d = 2.0
    D = np.zeros((5, 4))
    D[0, 0] = d
    res = fw.fwt(D, lam_L, lam_S, fixed_iters=1)
    h = res.history[0]
    f0 = 0.5 * d * d
    UL, US = f0 / lam_L, f0 / lam_S
    assert h["takeL"] and h["takeS"]
    assert h["sigma"] == pytest.approx(d, rel=1e-14) and h["gmax"] == pytest.approx(d, rel=1e-14)
    assert h["gap"] == pytest.approx(UL * (d - lam_L) + US * (d - lam_S), rel=1e-13)
    E11 = np.zeros_like(D)
    E11[0, 0] = 1.0
    if lam_L < lam_S:
        assert h["alpha"] == pytest.approx((d - lam_L) / UL, rel=1e-13) and h["beta"] == 0.0
        # L = (d - lam_L) e_1 e_1^T; the threshold of D - L = lam_L at lam_S leaves S = 0
        assert np.allclose(res.L, (d - lam_L) * E11, atol=1e-14) and not res.S.any()
        assert res.t_L == pytest.approx(d - lam_L, rel=1e-14) and res.t_S == 0.0
        assert res.f == pytest.approx(0.5 * lam_L ** 2 + lam_L * (d - lam_L), rel=1e-14)
    else:
        assert h["alpha"] == 0.0 and h["beta"] == pytest.approx((d - lam_S) / US, rel=1e-13)
        # S_half = (d - lam_S) e_1 e_1^T; the threshold step gives S = S_{lam_S}[D] = (d - lam_S) e_1 e_1^T
        assert not res.L.any() and np.allclose(res.S, (d - lam_S) * E11, atol=1e-14)
        assert res.t_L == 0.0 and res.t_S == pytest.approx(d - lam_S, rel=1e-14)
        assert res.f == pytest.approx(0.5 * lam_S ** 2 + lam_S * (d - lam_S), rel=1e-14)
