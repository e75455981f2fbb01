"""GPU parity of the differentiation form: the explicit iteration, and gradients of
the recovery loss ||L_K - L0||_F^2 of K unrolled (multilevel) iterations with respect
to D and lambda, through the hand-written adjoint, against the FP64 reference
gradient (PyTorch autograd on the CPU, itself pinned to FP64 central differences at
the full 1000 x 1000 size in the CPU tests).  Tolerance 1e-4 relative.  The adjoint of
one iteration is also checked as the transpose of the FP64 forward-mode derivative:
<J v, w> = <v, J^T w>."""
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


@pytest.mark.parametrize("levels", [0, 2])
def test_step_vjp_dot_product(levels):
    """<J v, w> with J v the FP64 forward-mode derivative of one iteration (CPU) equals
    <v, J^T w> with J^T w from mlpcp_ialm_step_vjp on the GPU, for a tangent v of all
    four inputs (D, S, Y, lambda) and a cotangent w of all three outputs."""
    import torch as T
    from torch.func import jvp
    torch, dev = torch_dev()
    w = synth.gaussian_lowrank_plus_sparse(150, 128, 5, seed=33, sparse_frac=0.05, levels=levels)
    rng = np.random.default_rng(4)
    m, n = w.D.shape
    S0 = (0.05 * rng.normal(size=(m, n))).astype(np.float32)
    Y0 = np.clip(0.2 * rng.normal(size=(m, n)), -w.lam, w.lam).astype(np.float32)
    lam32 = float(np.float32(w.lam))
    mu = 3.0 * w.mu0
    v = [rng.normal(size=(m, n)) for _ in range(3)] + [0.7]
    c = [rng.normal(size=(m, n)).astype(np.float32) for _ in range(3)]
    say("step dot product", levels)
    R = OU.restriction(n, levels)
    f64 = lambda a: T.tensor(np.asarray(a, dtype=np.float64))
    _, Jv = jvp(lambda D_, S_, Y_, l_: OU.step(D_, S_, Y_, l_, mu, R),
                (f64(w.D), f64(S0), f64(Y0), T.tensor(lam32, dtype=T.float64)),
                (f64(v[0]), f64(v[1]), f64(v[2]), T.tensor(v[3], dtype=T.float64)))
    lhs = sum(float((a * f64(b)).sum()) for a, b in zip(Jv, c))
    Db = torch.zeros((m, n), dtype=torch.float32, device=dev)
    Sb, Yb, lb = mlp.ialm_step_vjp(to_dev(w.D), to_dev(S0), to_dev(Y0), lam32, mu, levels,
                                   to_dev(c[0]), to_dev(c[1]), to_dev(c[2]), Db)
    torch.cuda.synchronize()
    rhs = (float(np.sum(v[0] * to_np(Db))) + float(np.sum(v[1] * to_np(Sb))) + float(np.sum(v[2] * to_np(Yb)))
           + v[3] * lb)
    say(f"   <Jv, w> {lhs:.9e}  <v, J^T w> {rhs:.9e}")
    assert abs(lhs - rhs) <= 1e-4 * max(abs(lhs), abs(rhs))


def test_unrolled_gradient_row_padded_D():
    """D passed as a row-padded view (leading dimension > n): the gradient lands in the
    view's entries only and equals the gradient for a contiguous D."""
    torch, dev = torch_dev()
    from paper_2206_13369_amd.autograd import unrolled
    w = synth.gaussian_lowrank_plus_sparse(120, 96, 4, seed=45, sparse_frac=0.05, levels=1)
    mus = oracle.default_schedule(w.mu0, 5)
    say("padded D gradient")
    _, gD_ref, gl_ref = _gpu_grad(w, mus, 1)
    X = torch.full((120, 104), 7.0, dtype=torch.float32, device=dev)
    X[:, :96] = to_dev(w.D)
    X.requires_grad_(True)
    lam = torch.tensor(w.lam, dtype=torch.float32, device=dev, requires_grad=True)
    L, _ = unrolled(X[:, :96], lam, mus, 1)
    loss = ((L - to_dev(w.L0.astype(np.float32))) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g = to_np(X.grad).astype(np.float64)
    assert not g[:, 96:].any()
    assert rel(g[:, :96], gD_ref) <= 1e-6
    assert abs(float(lam.grad) - gl_ref) <= 1e-6 * abs(gl_ref)
