"""GPU parity of the differentiation form: the explicit iteration, and gradients of
the recovery loss ||L_K - L0||_F^2 of K unrolled (multilevel) iterations with respect
to D and lambda, through the hand-written adjoint, against the FP64 reference
gradient (PyTorch autograd on the CPU, itself pinned to finite differences) and
against FP64 central differences computed by the oracle.  Tolerance 1e-4 relative."""
import numpy as np
import pytest

import oracle
from oracle import unrolled as OU
import paper_2206_13369_amd as mlp
import synth
from gpu_util import rel, say, to_dev, to_np, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("levels", [0, 2])
def test_step_matches_oracle_iteration(levels):
    torch, dev = torch_dev()
    w = synth.gaussian_lowrank_plus_sparse(150, 128, 5, seed=31, sparse_frac=0.05, levels=levels)
    rng = np.random.default_rng(2)
    S0 = (0.05 * rng.normal(size=w.D.shape)).astype(np.float32)
    Y0 = np.clip(0.2 * rng.normal(size=w.D.shape), -w.lam, w.lam).astype(np.float32)
    mu = 3.0 * w.mu0
    say("step", levels)
    ref = oracle.ialm(w.D, w.lam, mu, levels=levels, fixed_iters=1, S0=S0.astype(np.float64),
                      Y0=Y0.astype(np.float64))
    L, S, Y, r = mlp.ialm_step(to_dev(w.D), to_dev(S0), to_dev(Y0), w.lam, mu, levels)
    torch.cuda.synchronize()
    assert r == ref.rank
    assert rel(to_np(L), ref.L) <= 1e-5 and rel(to_np(S), ref.S) <= 1e-5 and rel(to_np(Y), ref.Y) <= 1e-5


def _gpu_grad(w, mus, levels):
    torch, dev = torch_dev()
    from paper_2206_13369_amd.autograd import unrolled
    D = to_dev(w.D).requires_grad_(True)
    lam = torch.tensor(w.lam, dtype=torch.float32, device=dev, requires_grad=True)
    L, _ = unrolled(D, lam, mus, levels)
    L0 = to_dev(w.L0.astype(np.float32))
    loss = ((L - L0) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return float(loss), to_np(D.grad).astype(np.float64), float(lam.grad)


@pytest.mark.parametrize("levels,m,n,K", [(0, 120, 96, 6), (2, 160, 128, 8), (1, 97, 64, 5)])
def test_unrolled_gradient_matches_fp64_reference(levels, m, n, K):
    w = synth.gaussian_lowrank_plus_sparse(m, n, 4, seed=40 + levels, sparse_frac=0.05, levels=levels)
    mus = oracle.default_schedule(w.mu0, K)
    say("grad", levels, m, n, K)
    lref, gD_ref, gl_ref, _ = OU.loss_and_grad(w.D, w.L0, w.lam, mus, levels)
    loss, gD, gl = _gpu_grad(w, mus, levels)
    say(f"   loss {loss:.6e}/{lref:.6e} errD {rel(gD, gD_ref):.2e} lam {gl:.6e}/{gl_ref:.6e}")
    assert abs(loss - lref) <= 1e-5 * lref
    assert rel(gD, gD_ref) <= 1e-4
    assert abs(gl - gl_ref) <= 1e-4 * abs(gl_ref)


@pytest.mark.slow
def test_c4_unrolled_gradient():
    # 1000 x 1000, rank 20, 5% +-1, K = 20 unrolled iterations, 2 levels (n_H = 250)
    w = synth.config("c4")
    K = 20
    mus = oracle.default_schedule(w.mu0, K)
    say("c4 reference gradient")
    lref, gD_ref, gl_ref, _ = OU.loss_and_grad(w.D, w.L0, w.lam, mus, w.levels)
    say("c4 gpu gradient")
    loss, gD, gl = _gpu_grad(w, mus, w.levels)
    eD = rel(gD, gD_ref)
    say(f"   loss {loss:.6e}/{lref:.6e} errD {eD:.2e} lam {gl:.6e}/{gl_ref:.6e}")
    assert abs(loss - lref) <= 1e-5 * lref
    assert eD <= 1e-4
    assert abs(gl - gl_ref) <= 1e-4 * abs(gl_ref)
    # FP64 central differences (oracle forward) along seeded unit directions,
    # rejecting directions that change an active set; with 10^6 entries over 20
    # iterations a step of 1e-6 flips some shrinkage support, so h = 1e-8 (FP64
    # rounding of the difference quotient ~ 1e-16 * loss / h, far below 1e-4)
    D = w.D.astype(np.float64)
    h = 1e-8
    rng = np.random.default_rng(7)
    f0, S0_, r0 = OU.loss_only(D, w.L0, w.lam, mus, w.levels)
    supp0 = S0_ != 0
    used = 0
    for _ in range(6):
        E = rng.normal(size=D.shape)
        E /= np.linalg.norm(E)
        fp, Sp, rp = OU.loss_only(D + h * E, w.L0, w.lam, mus, w.levels)
        fm, Sm, rm = OU.loss_only(D - h * E, w.L0, w.lam, mus, w.levels)
        if not (np.array_equal(Sp != 0, supp0) and np.array_equal(Sm != 0, supp0) and rp == r0 and rm == r0):
            say("   direction rejected (active set changed)")
            continue
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(gD * E))
        say(f"   fd {fd:.6e} gpu {an:.6e}")
        assert abs(fd - an) <= 1e-4 * np.linalg.norm(gD)
        used += 1
        if used == 3:
            break
    assert used >= 2
