"""GPU parity of FW-T and ML-FWT (Alg. 3, Alg. 6) for the unconstrained CPCP problem,
through the C ABI, against the FP64 oracle on the same seeded inputs.

Bar (float32 arithmetic on the GPU, float32-representable lam_L, lam_S on both sides):
relative Frobenius error of L and S <= 1e-5, objective history within 1e-6 relative,
step sizes alpha within 1e-4 absolute of the oracle's, and the same iteration count
when stopping on the tolerance.  The plain path finds its top singular pair by power
iteration (stopping at ||x_new - x_old|| <= 1e-6), the oracle by LAPACK SVD; its
fixed-iteration cases stay where the spectral gap of the gradient is clear.

Cases: small problems that span several row batches with ragged tails (including a
width that is not a multiple of 4, which takes the scalar path), masked and fully
observed, multilevel and plain; the reduced and full-size Table 2 workloads at a
fixed iteration count and to the 1e-3 tolerance; and the degenerate inputs (zero
data, an empty mask)."""
import functools

import numpy as np
import pytest

import oracle.fwt as ofw
import paper_2206_13369_amd as mlp
import synth
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


def _small(m, n, rank, levels, obs, seed):
    return synth.fw_cpcp(m, n, rank, seed=seed, levels=levels, observed_frac=obs)


@functools.lru_cache(maxsize=None)
def _fw(name, scale):
    return synth.fw_config(name, scale)


def _gpu(w, levels, *, tol=1e-3, max_iter=1000, masked=True, history=64):
    torch, dev = torch_dev()
    Q = to_dev(w.Q.astype(np.uint8)) if masked else None
    r = mlp.cpcp_fwt(to_dev(w.D), Q, w.lam_L, w.lam, levels=levels, tol=tol, max_iter=max_iter, history=history)
    torch.cuda.synchronize()
    return r


def _ora(w, levels, *, fixed=None, tol=1e-3, masked=True):
    return ofw.fwt(w.D, w.lam_L, w.lam, Q=w.Q if masked else None, levels=levels, tol=tol, fixed_iters=fixed)


def _compare(r, ref, tol=1e-5, check_alpha=True):
    eL, eS = rel(to_np(r.L), ref.L), rel(to_np(r.S), ref.S)
    fh = np.array([h["f"] for h in ref.history])
    ah = np.array([h["alpha"] for h in ref.history])
    k = min(len(r.f_history), len(fh))
    ef = float(np.max(np.abs(np.array(r.f_history[:k]) - fh[:k]) / fh[:k])) if k else 0.0
    ea = float(np.max(np.abs(np.array(r.alpha_history[:k]) - ah[:k]))) if k else 0.0
    say(f"   iters {r.iters}/{ref.iters} errL {eL:.2e} errS {eS:.2e} f {r.f:.6e}/{ref.f:.6e} "
        f"max rel f err {ef:.1e} max alpha err {ea:.1e} power steps {r.power_steps}")
    assert r.iters == ref.iters
    assert eL <= tol and eS <= tol
    assert ef <= 1e-6
    if check_alpha:
        assert ea <= 1e-4
    assert abs(r.f - ref.f) <= 1e-6 * abs(ref.f)


@pytest.mark.parametrize("m,n,rank,levels,obs,masked", [
    (700, 96, 3, 2, 0.8, True),      # several row batches, ragged tail
    (530, 70, 2, 3, 0.6, True),      # n % 4 != 0: scalar path; odd coarse widths
    (640, 128, 3, 2, 1.0, False),    # fully observed (Q = NULL)
    (300, 300, 4, 3, 0.7, True),     # square
    (1030, 128, 3, 1, 0.8, True),    # one level: two-column intervals, n_H = 64
    (512, 255, 3, 2, 0.8, True),     # odd width on the scalar path, n_H = 64
])
def test_ml_fixed_iterations(m, n, rank, levels, obs, masked):
    w = _small(m, n, rank, levels, obs, seed=m + n)
    K = 25
    say("ML-FWT", (m, n), "levels", levels, "masked", masked, "K", K)
    r = _gpu(w, levels, tol=1e-30, max_iter=K, masked=masked)
    ref = _ora(w, levels, fixed=K, masked=masked)
    assert r.status == mlp.MLPCP_NOT_CONVERGED
    _compare(r, ref)


@pytest.mark.parametrize("m,n,rank,obs,masked", [
    (600, 96, 3, 0.8, True),
    (410, 70, 2, 0.6, True),         # scalar path
    (500, 128, 3, 1.0, False),
    (1100, 1002, 3, 0.8, True),      # wide, scalar path
])
def test_plain_fixed_iterations(m, n, rank, obs, masked):
    w = _small(m, n, rank, 0, obs, seed=m + 2 * n)
    K = 8
    say("FW-T", (m, n), "masked", masked, "K", K)
    r = _gpu(w, 0, tol=1e-30, max_iter=K, masked=masked)
    ref = _ora(w, 0, fixed=K, masked=masked)
    _compare(r, ref)


@pytest.mark.parametrize("name,scale,levels", [("fw1", 0.1, None), ("fw3", 0.1, None), ("fw1", 0.1, 0),
                                               ("fw3", 0.1, 0)])
def test_reduced_workloads_to_tolerance(name, scale, levels):
    w = _fw(name, scale)
    lv = w.levels if levels is None else levels
    say(name, scale, w.D.shape, "levels", lv, "to 1e-3")
    r = _gpu(w, lv)
    ref = _ora(w, lv)
    assert r.status == mlp.MLPCP_OK and r.converged
    _compare(r, ref)
    # deterministic: a second run gives the same bits
    r2 = _gpu(w, lv)
    assert r2.iters == r.iters and np.array_equal(to_np(r2.L), to_np(r.L)) and np.array_equal(to_np(r2.S), to_np(r.S))


def test_full_fw1_multilevel_to_tolerance():
    w = _fw("fw1", 1.0)
    say("fw1 full", w.D.shape, "levels", w.levels, "to 1e-3")
    r = _gpu(w, w.levels)
    ref = _ora(w, w.levels)
    _compare(r, ref)


def test_wide_rows_longest_chunks():
    # n = 8000 at 7 levels: 127-column intervals cut into chunks of 32, the most per row
    w = _small(8000, 8000, 2, 7, 0.8, seed=23)
    K = 3
    say("ML-FWT 8000x8000 levels 7, K", K)
    r = _gpu(w, 7, tol=1e-30, max_iter=K)
    ref = _ora(w, 7, fixed=K)
    _compare(r, ref)


@pytest.mark.slow
def test_full_fw2_multilevel_fixed():
    w = _fw("fw2", 1.0)
    K = 3
    say("fw2 full", w.D.shape, "levels", w.levels, "K", K)
    r = _gpu(w, w.levels, tol=1e-30, max_iter=K)
    ref = _ora(w, w.levels, fixed=K)
    _compare(r, ref)


def test_zero_data_and_empty_mask():
    torch, dev = torch_dev()
    D = torch.zeros((256, 64), dtype=torch.float32, device=dev)
    for Q in (None, torch.ones((256, 64), dtype=torch.uint8, device=dev)):
        for lv in (0, 2):
            r = mlp.cpcp_fwt(D, Q, 1.0, 0.1, levels=lv)
            assert r.status == mlp.MLPCP_OK and r.iters == 0 and r.f == 0.0
            assert float(r.L.abs().max()) == 0.0 and float(r.S.abs().max()) == 0.0
    w = _small(256, 64, 2, 2, 0.8, seed=5)
    Q0 = torch.zeros((256, 64), dtype=torch.uint8, device=dev)
    r = mlp.cpcp_fwt(to_dev(w.D), Q0, w.lam_L, w.lam, levels=2)
    assert r.status == mlp.MLPCP_OK and r.iters == 0
    assert float(r.L.abs().max()) == 0.0 and float(r.S.abs().max()) == 0.0


def test_unsupported_shapes_rejected():
    torch, dev = torch_dev()
    D = torch.zeros((512, 200), dtype=torch.float32, device=dev)
    with pytest.raises(mlp.MLPCPError):
        mlp.cpcp_fwt(D, None, 1.0, 0.1, levels=1)        # n_H = 100 > 64
    with pytest.raises(mlp.MLPCPError):
        mlp.cpcp_fwt(D, None, 0.0, 0.1, levels=2)
