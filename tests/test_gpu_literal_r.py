"""GPU parity of the multilevel solver with the literal interpolation operator
(mlpcp_opts.r_norm = 1: R = P / ||P||_2; 2: R = P) against the FP64 oracle with the same
explicit R, at a fixed iteration count (these variants need not converge to the
tolerance: the ablation of the orthonormalisation reading).  Bar: relative Frobenius
error of L and S <= 1e-5 and identical ranks."""
import numpy as np
import pytest

import oracle
import paper_2206_13369_amd as mlp
import synth
from oracle import diagnostics as dg
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r_norm", [1, 2])
@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_literal_restriction_fixed_iterations(name, r_norm):
    torch, dev = torch_dev()
    if name == "c1":
        w = synth.config("c1")
    else:   # a reduced compressive case: 600 x 400, 3 levels, masked
        w = synth.gaussian_lowrank_plus_sparse(600, 400, 12, seed=21, sparse_frac=0.1, sparse_kind="uniform",
                                               sparse_amp=10.0, observed_frac=0.6, levels=3, name="c2s")
    K = 8
    R = dg.literal_restriction(w.n, w.levels, scaled=(r_norm == 1))
    say(name, w.D.shape, "levels", w.levels, "r_norm", r_norm, "K", K)
    ref = oracle.ialm(w.D, w.lam, w.mu0, Q=w.Q, levels=w.levels, fixed_iters=K, R=R, record=True)
    kw = dict(levels=w.levels, tol=1e-30, max_iter=K, r_norm=r_norm, history=K)
    if w.Q is None:
        r = mlp.pcp_solve(to_dev(w.D), w.lam, w.mu0, **kw)
    else:
        r = mlp.cpcp_solve(to_dev(w.D), to_dev(w.Q.astype(np.uint8)), w.lam, w.mu0, **kw)
    torch.cuda.synchronize()
    eL, eS = rel(to_np(r.L), ref.L), rel(to_np(r.S), ref.S)
    say(f"   errL {eL:.2e} errS {eS:.2e} ranks {r.rank_history} / {[h['rank'] for h in ref.history]} "
        f"fg {r.fg:.3e} / {ref.fg:.3e}")
    assert r.rank_history == [h["rank"] for h in ref.history]
    assert eL <= 1e-5 and eS <= 1e-5


def test_restriction_ablation_recovery():
    """The three normalisations solved to FG <= 1e-6 on c1, c2 and the video workload:
    all reach the feasibility tolerance (the S and Y steps absorb what L misses), but only
    the orthonormal R recovers L0; P / ||P||_2 under-fits (ranks too low) and the raw P
    over-fits.  Thm. 3's epsilon at the final coarse iterate and delta = max_k Delta_k
    (Lemma 3, with the final iterate for L_H*) come from the FP64 oracle on c1.  The
    numbers are printed for the design notes; the assertion is the reading's claim: the
    orthonormal operator recovers L0 best on every workload."""
    torch, dev = torch_dev()
    cases = [("c1", synth.config("c1")), ("c2", synth.config("c2")), ("c3", synth.config("c3", 0.25))]
    for name, w in cases:
        errs = {}
        for rn in (0, 1, 2):
            kw = dict(levels=w.levels, tol=1e-6, max_iter=500, r_norm=rn)
            if w.Q is None:
                r = mlp.pcp_solve(to_dev(w.D), w.lam, w.mu0, **kw)
            else:
                r = mlp.cpcp_solve(to_dev(w.D), to_dev(w.Q.astype(np.uint8)), w.lam, w.mu0, **kw)
            torch.cuda.synchronize()
            S0 = w.S0 if w.Q is None else np.where(w.Q, w.S0, 0.0)
            eL, eS = rel(to_np(r.L), w.L0), rel(to_np(r.S), S0)
            errs[rn] = eL
            say(f"ablation {name} r_norm {rn}: iters {r.iters} fg {r.fg:.2e} rank {r.rank} "
                f"err(L0) {eL:.3e} err(S0) {eS:.3e}")
        assert errs[0] < errs[1] and errs[0] < errs[2]
    w = synth.config("c1")
    for rn in (1, 2):
        R = dg.literal_restriction(w.n, w.levels, scaled=(rn == 1))
        ref = oracle.ialm(w.D, w.lam, w.mu0, levels=w.levels, tol=1e-6, max_iter=300, R=R, keep_iterates=True)
        LHs = ref.history[-1]["LH"]
        eps = dg.epsilon(LHs, R)
        dl = max(dg.delta(h["LH"], LHs, R) for h in ref.history)
        say(f"diagnostics c1 r_norm {rn}: eps {eps:.3e} (||L_H||_* {float(np.linalg.svd(LHs, compute_uv=False).sum()):.3e}), "
            f"delta {dl:.3e}, oracle iters {ref.iters}")
