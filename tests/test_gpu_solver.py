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
    say(f"   errL {eL:.2e} errS {eS:.2e} rank {res.rank}/{ref.rank} iters {res.iters}/{ref.iters} "
        f"partial eigensolve iters {res.partial_eig_iters}")
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


@pytest.mark.parametrize("masked", [False, True])
def test_default_mu0_on_device(masked):
    """mu0 <= 0 selects 1.25 / ||P_Q D||_2, computed by the library on the device; it
    matches the oracle's LAPACK spectral norm to 1e-6 and the solve then matches the
    oracle run with that penalty."""
    w = synth.gaussian_lowrank_plus_sparse(400, 300, 8, seed=23, sparse_frac=0.08, levels=2,
                                           observed_frac=0.7 if masked else None)
    torch, dev = torch_dev()
    mu_ref = 1.25 / oracle.spectral_norm(w.D, w.Q)
    say("default mu0", masked)
    kw = dict(levels=2, tol=1e-6, history=600)
    D = to_dev(w.D)
    if masked:
        res = mlp.cpcp_solve(D, to_dev(w.Q.astype(np.uint8)), w.lam, 0.0, **kw)
    else:
        res = mlp.pcp_solve(D, w.lam, None, **kw)
    torch.cuda.synchronize()
    say(f"   mu0 {res.mu0:.12e} oracle {mu_ref:.12e}")
    assert abs(res.mu0 - mu_ref) <= 1e-6 * mu_ref
    ref = oracle.ialm(w.D, w.lam, res.mu0, Q=w.Q, levels=2, tol=1e-6)
    assert res.status == mlp.MLPCP_OK and res.iters == ref.iters
    _check(res, ref)


@pytest.mark.parametrize("where", ["D", "S0", "Y0"])
@pytest.mark.parametrize("value", [float("nan"), float("inf")])
def test_nonfinite_input_is_reported(where, value):
    """A NaN or Inf in an observed entry of D, S0 or Y0 gives MLPCP_E_NONFINITE before
    any iteration (the initial pass over the data detects it)."""
    w = synth.config("c1")
    torch, dev = torch_dev()
    D = w.D.copy()
    S0 = np.zeros_like(D)
    Y0 = np.zeros_like(D)
    {"D": D, "S0": S0, "Y0": Y0}[where][17, 5] = value
    say("nonfinite", where, value)
    with pytest.raises(mlp.MLPCPError) as e:
        mlp.pcp_solve(to_dev(D), w.lam, w.mu0, levels=2, S0=to_dev(S0), Y0=to_dev(Y0))
    torch.cuda.synchronize()
    assert e.value.status == mlp.MLPCP_E_NONFINITE


def test_nonfinite_off_mask_is_ignored():
    """D off Q never reaches the result: NaN there gives the same bits as zeros there."""
    w = synth.gaussian_lowrank_plus_sparse(240, 200, 5, seed=29, sparse_frac=0.05, levels=2, observed_frac=0.6)
    torch, dev = torch_dev()
    Dz = np.where(w.Q, w.D, 0.0).astype(np.float32)
    Dn = np.where(w.Q, w.D, np.nan).astype(np.float32)
    Q = to_dev(w.Q.astype(np.uint8))
    say("nan off mask")
    a = mlp.cpcp_solve(to_dev(Dz), Q, w.lam, w.mu0, levels=2, tol=1e-6)
    b = mlp.cpcp_solve(to_dev(Dn), Q, w.lam, w.mu0, levels=2, tol=1e-6)
    torch.cuda.synchronize()
    assert a.status == b.status == mlp.MLPCP_OK and a.iters == b.iters
    assert np.array_equal(to_np(a.L), to_np(b.L)) and np.array_equal(to_np(a.S), to_np(b.S))


@pytest.mark.parametrize("levels", [0, 2])
@pytest.mark.parametrize("masked", [False, True])
def test_max_iter_exhaustion(levels, masked):
    """max_iter reached before the tolerance: MLPCP_NOT_CONVERGED with valid outputs,
    equal to the oracle's iterate after max_iter iterations."""
    w = synth.gaussian_lowrank_plus_sparse(300, 240, 6, seed=37, sparse_frac=0.05, levels=levels,
                                           observed_frac=0.7 if masked else None)
    K = 5
    ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=levels, fixed_iters=K)
    say("max_iter", levels, masked)
    res = _run_gpu(w, levels, tol=1e-6, fixed=K)
    assert res.status == mlp.MLPCP_NOT_CONVERGED and res.iters == K and res.fg > 1e-6
    _check(res, ref)


@pytest.mark.parametrize("masked", [False, True])
def test_zero_data(masked):
    """P_Q D = 0: L = S = Y = 0 with no iteration, status OK (also with the default mu0)."""
    torch, dev = torch_dev()
    m, n = 256, 200
    D = torch.zeros((m, n), dtype=torch.float32, device=dev)
    say("zero data", masked)
    for mu0 in (1.0, None):
        if masked:
            Q = torch.ones((m, n), dtype=torch.uint8, device=dev)
            r = mlp.cpcp_solve(D, Q, 0.05, mu0, levels=2)
        else:
            r = mlp.pcp_solve(D, 0.05, mu0, levels=2)
        torch.cuda.synchronize()
        assert r.status == mlp.MLPCP_OK and r.iters == 0 and r.rank == 0
        assert not to_np(r.L).any() and not to_np(r.S).any() and not to_np(r.Y).any()


@pytest.mark.parametrize("masked", [False, True])
def test_partial_eigensolve_matches_oracle(masked):
    """A 1024-wide plain solve at rank 8, where every SVT after the first ones at that
    rank comes from the rank-predicted partial eigensolve (64-column subspace iteration,
    Rayleigh-Ritz, Cholesky certificate): L and S within 1e-5 of the oracle's full-SVD
    solve, the same rank in every iteration, and the partial path taken."""
    w = synth.gaussian_lowrank_plus_sparse(1100, 1024, 8, seed=33, sparse_frac=0.05,
                                           observed_frac=0.7 if masked else None, levels=0)
    ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=0, tol=1e-6, record=True)
    say("partial eigensolve", masked, ref.iters, ref.rank)
    res = _run_gpu(w, 0, tol=1e-6)
    assert res.status == mlp.MLPCP_OK and res.fg <= 1e-6
    assert res.iters == ref.iters
    _check(res, ref)
    assert res.rank_history == [h["rank"] for h in ref.history]
    assert res.partial_eig_iters >= 1


@pytest.mark.parametrize("levels,masked,shape", [(2, False, (300, 300)), (0, False, (300, 300)),
                                                 (3, True, (700, 520)), (1, True, (900, 500))])
def test_matrix_function_svt_matches_oracle(levels, masked, shape):
    """The matrix-function coarse SVT (f(G) from scaled Newton-Schulz products, no
    eigenvectors) against the oracle's full-SVD solve and against the Jacobi path of the
    same library: L and S within 1e-5 of the oracle, the same rank in every iteration,
    the path taken in every iteration that follows a nonzero rank, and its norm bounds
    within the growth its step counts assume.  Padded widths 128 (n_H = 75), 320 (the
    plain 300-wide Gram), 128 (n_H = 65, one past the one-workgroup path) and 256
    (n_H = 250)."""
    m, n = shape
    w = synth.gaussian_lowrank_plus_sparse(m, n, 10, seed=41 + levels, sparse_frac=0.06, sparse_kind="uniform",
                                           sparse_amp=6.0, observed_frac=0.65 if masked else None, levels=levels)
    ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=levels, tol=1e-6, record=True)
    say("matrix-function svt", levels, masked, shape, ref.iters, ref.rank)
    res = _run_gpu(w, levels, tol=1e-6)
    assert res.status == mlp.MLPCP_OK and res.fg <= 1e-6
    assert res.iters == ref.iters
    _check(res, ref)
    ranks = [h["rank"] for h in ref.history]
    assert res.rank_history == ranks
    # the path is taken in every iteration that follows a nonzero rank, and in those after
    # a zero rank whose Gershgorin discs do not settle it
    expect = sum(1 for i in range(1, len(ranks)) if ranks[i - 1] > 0)
    say(f"   matrix-function iters {res.msvt_iters} (at least {expect}) products {res.msvt_products} "
        f"flags {res.msvt_flags}")
    assert expect <= res.msvt_iters <= res.iters and res.msvt_flags == 0
    # the eigensolver path of the same solve
    torch, dev = torch_dev()
    D = to_dev(w.D)
    kw = dict(levels=levels, tol=1e-6, history=600, svt_method=1)
    if w.Q is None:
        eig = mlp.pcp_solve(D, w.lam, w.mu0, **kw)
    else:
        eig = mlp.cpcp_solve(D, to_dev(w.Q.astype(np.uint8)), w.lam, w.mu0, **kw)
    torch.cuda.synchronize()
    assert eig.msvt_iters == 0 and eig.rank_history == ranks
    assert rel(to_np(res.L), to_np(eig.L)) <= TOL32 and rel(to_np(res.S), to_np(eig.S)) <= TOL32


@pytest.mark.parametrize("levels", [2, 0])
def test_matrix_function_svt_ill_conditioned(levels):
    """A long fixed-iteration solve (mu grows by 1.5 per iteration, so the Gram's largest
    eigenvalue ends about 1e10 times tau^2): the coupled inverse square root iteration
    stays stable (its products are not symmetrised) and the result tracks the oracle's
    full SVD, with the same rank in every iteration."""
    w = synth.config("c1")
    K = 36
    ref = oracle.ialm(w.D, w.lam, w.mu0, levels=levels, fixed_iters=K, record=True)
    say("ill-conditioned matrix-function svt", levels, K)
    res = _run_gpu(w, levels, fixed=K)
    assert res.iters == K
    _check(res, ref)
    ranks = [h["rank"] for h in ref.history]
    assert res.rank_history == ranks
    expect = sum(1 for i in range(1, K) if ranks[i - 1] > 0)
    say(f"   matrix-function iters {res.msvt_iters} (at least {expect}) flags {res.msvt_flags}")
    assert res.msvt_iters >= expect and res.msvt_flags == 0


def test_concurrent_solves_from_host_threads():
    """Three solves at once from three host threads, each on a stream of its own: a tall
    PCP (one-workgroup coarse SVT), a wide CPCP (matrix-function SVT with its Gershgorin
    probe) and an ML-FWT solve.  Each thread's stop tests read the records its own
    pinned page receives, so the results equal, bit for bit, those of the same solves
    run one after the other."""
    import threading

    torch, dev = torch_dev()
    wa = synth.gaussian_lowrank_plus_sparse(300, 256, 6, seed=51, sparse_frac=0.05, levels=2)
    wb = synth.gaussian_lowrank_plus_sparse(600, 512, 8, seed=52, sparse_frac=0.05, levels=1, observed_frac=0.7)
    wc = synth.fw_cpcp(1200, 400, 2, seed=53, levels=3, observed_frac=0.8)
    Da, Db, Dc = to_dev(wa.D), to_dev(wb.D), to_dev(wc.D)
    Qb, Qc = to_dev(wb.Q.astype(np.uint8)), to_dev(wc.Q.astype(np.uint8))
    torch.cuda.synchronize()

    def run(k):
        if k == 0:
            r = mlp.pcp_solve(Da, wa.lam, wa.mu0, levels=2, tol=1e-6, history=600)
            return r.iters, to_np(r.L), to_np(r.S)
        if k == 1:
            r = mlp.cpcp_solve(Db, Qb, wb.lam, wb.mu0, levels=1, tol=1e-6, history=600)
            return r.iters, to_np(r.L), to_np(r.S)
        r = mlp.cpcp_fwt(Dc, Qc, wc.lam_L, wc.lam, levels=3, tol=1e-3, history=64)
        return r.iters, to_np(r.L), to_np(r.S)

    ref = [run(k) for k in range(3)]
    say("concurrent: sequential iterations", [x[0] for x in ref])
    out, errs = [None] * 3, []

    def worker(k):
        try:
            st = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(st):
                out[k] = run(k)
            st.synchronize()
        except Exception as e:   # reported below, in the main thread
            errs.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(3)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=90)
    assert not any(t.is_alive() for t in threads), "a solve did not finish"
    assert not errs, errs
    for k in range(3):
        assert out[k][0] == ref[k][0]
        assert np.array_equal(out[k][1], ref[k][1]) and np.array_equal(out[k][2], ref[k][2])
