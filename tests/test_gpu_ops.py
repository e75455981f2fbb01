"""GPU parity of the streaming operators and the coarse SVT against the FP64 oracle,
called through the C ABI (Python binding).  Sizes span several tiles and ragged
tails; tolerances follow from float32 arithmetic."""
import numpy as np
import pytest

import oracle
import paper_2206_13369_amd as mlp
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


def test_shrink_matches_float32_formula_exactly():
    torch, dev = torch_dev()
    rng = np.random.default_rng(0)
    x = rng.normal(size=100003).astype(np.float32) * 3
    x[:6] = [0.0, -0.0, 0.5, -0.5, np.inf, -np.inf]
    for tau in (0.0, 0.5, 1.0, 2.75):
        say("shrink", tau)
        y = to_np(mlp.shrink(to_dev(x), tau))
        ref = np.sign(x) * np.maximum(np.abs(x) - np.float32(tau), np.float32(0))
        assert y.dtype == np.float32
        assert np.array_equal(y, ref.astype(np.float32))
    # NaN propagates, in place works
    xn = np.array([np.nan, 1.0, -3.0], dtype=np.float32)
    t = to_dev(xn)
    mlp.shrink(t, 0.5, out=t)
    got = to_np(t)
    assert np.isnan(got[0]) and got[1] == 0.5 and got[2] == -2.5


@pytest.mark.parametrize("m,n,levels", [(37, 50, 2), (130, 200, 4), (65, 25, 1), (9, 300, 2), (300, 2000, 3),
                                        (64, 64, 0), (77, 64, 2), (33, 128, 3), (50, 252, 4), (17, 256, 5)])
def test_restrict_prolong(m, n, levels):
    say("restrict/prolong", m, n, levels)
    rng = np.random.default_rng(m + n)
    X = rng.normal(size=(m, n)).astype(np.float32)
    XH = to_np(mlp.restrict(to_dev(X), levels))
    ref = oracle.restrict(X.astype(np.float64), levels)
    assert XH.shape == ref.shape
    assert rel(XH, ref) < 2e-6
    Z = rng.normal(size=ref.shape).astype(np.float32)
    Xf = to_np(mlp.prolong(to_dev(Z), n, levels))
    ref2 = oracle.prolong(Z.astype(np.float64), n, levels)
    assert rel(Xf, ref2) < 2e-6
    if levels == 0:
        assert np.array_equal(XH, X) and np.array_equal(Xf, Z)


@pytest.mark.parametrize("m,n,levels,rank", [(50, 20, 0, 3), (120, 64, 0, 5), (300, 300, 2, 10), (500, 100, 0, 8),
                                             (400, 200, 4, 6), (257, 250, 1, 12), (90, 33, 0, 4),
                                             (700, 520, 0, 12), (2000, 2000, 3, 30),
                                             (1200, 1100, 0, 12),    # width >= 1024: partial certificate
                                             (640, 512, 0, 10),      # widest split apply step (A alternates)
                                             (100, 16, 0, 3), (300, 60, 2, 4), (130, 7, 0, 2)])   # one-wave sweeps
def test_svt_prox_matches_oracle(m, n, levels, rank):
    say("svt_prox", m, n, levels, rank)
    rng = np.random.default_rng(m * 7 + n)
    M = (rng.normal(size=(m, rank)) @ rng.normal(size=(rank, n)) + 0.05 * rng.normal(size=(m, n))).astype(np.float32)
    s = np.linalg.svd(oracle.restrict(M.astype(np.float64), levels), compute_uv=False)
    # threshold in a gap of the coarse spectrum, so the rank is well defined
    gaps = s[:-1] / s[1:]
    k = int(np.argmax(gaps[: max(1, min(len(gaps), rank + 2))]))
    tau = float(np.sqrt(s[k] * s[k + 1]))
    L, r = mlp.svt_prox(to_dev(M), tau, levels)
    Lref, rref = oracle.svt_prox(M.astype(np.float64), tau, levels)
    assert r == rref
    assert rel(to_np(L), Lref) < 1e-5


def test_svt_prox_thresholds_everything():
    torch, dev = torch_dev()
    rng = np.random.default_rng(3)
    M = rng.normal(size=(80, 40)).astype(np.float32)
    L, r = mlp.svt_prox(to_dev(M), 1e6, 1)
    assert r == 0 and not to_np(L).any()


@pytest.mark.parametrize("m,n,tau,levels", [(600, 520, 1e6, 0), (600, 520, 1e6, 2), (600, 520, 1e-3, 0),
                                             (600, 520, 1e-3, 2), (1100, 1030, 1e6, 0), (1100, 1030, 1e-3, 0)])
def test_svt_prox_blocked_extremes(m, n, tau, levels):
    # widths above 64 take the blocked eigensolver: a threshold above the whole spectrum
    # certifies every index at once (no sweep, rank 0); one below it certifies none
    # (width 1030 pads to 1088, where the certificate also takes its partial form)
    say("svt_prox extremes", m, n, tau, levels)
    rng = np.random.default_rng(17 + levels + n)
    M = rng.normal(size=(m, n)).astype(np.float32)
    L, r = mlp.svt_prox(to_dev(M), tau, levels)
    Lref, rref = oracle.svt_prox(M.astype(np.float64), tau, levels)
    assert r == rref
    if rref == 0:
        assert not to_np(L).any()
    else:
        assert rref == oracle.restrict(M.astype(np.float64), levels).shape[1]   # full coarse rank
        assert rel(to_np(L), Lref) < 1e-5


def test_shrink_unaligned_and_tails():
    """The vector path (16-byte groups) and the scalar path (misaligned views, tails)
    give the float32 formula's bits."""
    torch, dev = torch_dev()
    rng = np.random.default_rng(3)
    x = (rng.normal(size=4 * 65536 + 7) * 2).astype(np.float32)
    t = to_dev(x)
    for off, cnt in ((0, x.size), (1, x.size - 1), (2, 4 * 65536), (3, 10)):
        say("shrink offset", off, cnt)
        y = to_np(mlp.shrink(t[off:off + cnt], 0.7))
        ref = np.sign(x[off:off + cnt]) * np.maximum(np.abs(x[off:off + cnt]) - np.float32(0.7), np.float32(0))
        assert np.array_equal(y, ref.astype(np.float32))


@pytest.mark.parametrize("m,n,levels,pad", [(1000, 200, 4, 0), (513, 203, 3, 5), (77, 1000, 2, 3), (40, 1024, 1, 0),
                                             (300, 96, 3, 4), (61, 200, 4, 8)])
def test_restrict_prolong_padded_rows(m, n, levels, pad):
    """Row-padded inputs (ld > n, also not a multiple of 4) and widths whose coarse
    tiles take the fallback kernels (n_H = 512 at 1024 / 1 level)."""
    torch, dev = torch_dev()
    say("restrict/prolong padded", m, n, levels, pad)
    rng = np.random.default_rng(m + 3 * n)
    X = rng.normal(size=(m, n + pad)).astype(np.float32)
    Xd = to_dev(X)[:, :n]
    XH = to_np(mlp.restrict(Xd, levels))
    ref = oracle.restrict(X[:, :n].astype(np.float64), levels)
    assert rel(XH, ref) < 2e-6
    nH = ref.shape[1]
    Z = rng.normal(size=(m, nH + pad)).astype(np.float32)
    Xf = to_np(mlp.prolong(to_dev(Z)[:, :nH], n, levels))
    assert rel(Xf, oracle.prolong(Z[:, :nH].astype(np.float64), n, levels)) < 2e-6


def test_restrict_prolong_full_hyperspectral_size():
    """262144 x 200, 4 levels (n_H = 13), the size the streaming kernels are measured at:
    every row on the GPU, the FP64 oracle on a seeded sample of rows (the maps act row
    by row)."""
    torch, dev = torch_dev()
    m, n, levels = 262144, 200, 4
    rng = np.random.default_rng(11)
    X = rng.normal(size=(m, n)).astype(np.float32)
    say("restrict/prolong full size")
    XH = to_np(mlp.restrict(to_dev(X), levels))
    rows = np.sort(rng.choice(m, 4096, replace=False))
    rows = np.concatenate([rows, [0, m - 1]])
    assert rel(XH[rows], oracle.restrict(X[rows].astype(np.float64), levels)) < 2e-6
    Z = rng.normal(size=(m, XH.shape[1])).astype(np.float32)
    Xf = to_np(mlp.prolong(to_dev(Z), n, levels))
    assert rel(Xf[rows], oracle.prolong(Z[rows].astype(np.float64), n, levels)) < 2e-6
