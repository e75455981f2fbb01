"""GPU parity of the PCP / CPCP solvers against the FP64 oracle on the same seeded
inputs (D rounded to float32 once; the oracle consumes the rounded values).

FP32 tolerance: relative Frobenius error <= 1e-5 in L and S, identical rank.
Checked at a fixed iteration count (the oracle's own stopping iteration) and at
each side's own stop."""
import numpy as np
import pytest

import oracle
import paper_2206_13369_amd as mlp
import synth
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def _run_gpu(w, levels, tol=None, fixed=None, masked=None, S0=None, Y0=None):
    torch, dev = torch_dev()
    D = to_dev(w.D)
    kw = dict(levels=levels, tol=tol if tol is not None else 1e-30, max_iter=fixed if fixed else 500, history=600)
    if S0 is not None:
        kw["S0"] = to_dev(S0.astype(np.float32))
    if Y0 is not None:
        kw["Y0"] = to_dev(Y0.astype(np.float32))
    Q = w.Q if masked is None else masked
    if Q is None:
        res = mlp.pcp_solve(D, w.lam, w.mu0, **kw)
    else:
        res = mlp.cpcp_solve(D, to_dev(Q.astype(np.uint8)), w.lam, w.mu0, **kw)
    torch.cuda.synchronize()
    return res


def _check(res, ref, tol=TOL32, rank=True):
    eL = rel(to_np(res.L), ref.L)
    eS = rel(to_np(res.S), ref.S)
    say(f"   errL {eL:.2e} errS {eS:.2e} rank {res.rank}/{ref.rank} iters {res.iters}/{ref.iters}")
    assert eL <= tol and eS <= tol
    if rank:
        assert res.rank == ref.rank


@pytest.mark.parametrize("levels", [0, 2])
def test_c1_fixed_iterations(levels):
    w = synth.config("c1")
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, tol=1e-6)
    say("c1 fixed", levels, ref.iters)
    res = _run_gpu(w, levels, fixed=ref.iters)
    assert res.iters == ref.iters
    _check(res, ref)
    Y = to_np(res.Y)
    assert rel(Y, ref.Y) <= 1e-4


@pytest.mark.parametrize("levels", [0, 2])
def test_c1_to_tolerance(levels):
    w = synth.config("c1")
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, tol=1e-6, record=True)
    say("c1 tol", levels)
    res = _run_gpu(w, levels, tol=1e-6)
    assert res.status == mlp.MLPCP_OK and res.fg <= 1e-6
    assert abs(res.iters - ref.iters) <= 1
    _check(res, ref)
    # per-iteration ranks and gaps track the oracle
    assert res.rank_history[: len(ref.history)] == [h["rank"] for h in ref.history][: len(res.rank_history)]
    fg_ref = np.array([h["fg"] for h in ref.history])
    k = min(len(fg_ref), len(res.fg_history))
    assert np.allclose(res.fg_history[:k], fg_ref[:k], rtol=1e-3, atol=1e-8)


@pytest.mark.parametrize("levels,observed", [(0, 0.6), (2, 0.6), (3, 0.7)])
def test_masked_small(levels, observed):
    w = synth.gaussian_lowrank_plus_sparse(240, 200, 6, seed=21, sparse_frac=0.08, sparse_kind="uniform",
                                           sparse_amp=5.0, observed_frac=observed, levels=levels)
    ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=levels, tol=1e-6)
    say("masked", levels, observed, ref.iters)
    res = _run_gpu(w, levels, fixed=ref.iters)
    _check(res, ref)
    S = to_np(res.S)
    Y = to_np(res.Y)
    assert not S[~w.Q].any() and not Y[~w.Q].any()


def test_full_mask_equals_pcp():
    w = synth.gaussian_lowrank_plus_sparse(150, 120, 5, seed=4, sparse_frac=0.05, levels=2)
    say("full mask")
    a = _run_gpu(w, 2, fixed=12)
    b = _run_gpu(w, 2, fixed=12, masked=np.ones(w.D.shape, bool))
    assert np.array_equal(to_np(a.L), to_np(b.L)) and np.array_equal(to_np(a.S), to_np(b.S))


def test_ragged_rows_and_odd_width():
    # m not a multiple of the row tile, odd n (vertex-centred restriction)
    w = synth.gaussian_lowrank_plus_sparse(333, 101, 4, seed=8, sparse_frac=0.05, levels=1)
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=1, tol=1e-6)
    say("ragged", ref.iters)
    res = _run_gpu(w, 1, fixed=ref.iters)
    _check(res, ref)


def test_warm_start_inputs():
    w = synth.gaussian_lowrank_plus_sparse(160, 128, 5, seed=9, sparse_frac=0.05, levels=2)
    rng = np.random.default_rng(1)
    S0 = 0.01 * rng.normal(size=w.D.shape).astype(np.float32)
    Y0 = np.clip(0.1 * rng.normal(size=w.D.shape), -w.lam, w.lam).astype(np.float32)
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=2, fixed_iters=10, S0=S0.astype(np.float64),
                      Y0=Y0.astype(np.float64))
    say("warm start")
    res = _run_gpu(w, 2, fixed=10, S0=S0, Y0=Y0)
    _check(res, ref)


def test_determinism():
    w = synth.gaussian_lowrank_plus_sparse(300, 256, 6, seed=10, sparse_frac=0.05, observed_frac=0.8, levels=2)
    say("determinism")
    a = _run_gpu(w, 2, fixed=15)
    b = _run_gpu(w, 2, fixed=15)
    assert np.array_equal(to_np(a.L), to_np(b.L)) and np.array_equal(to_np(a.S), to_np(b.S))
