"""Seeded synthetic workloads for multilevel PCP / CPCP.

This module only draws random inputs.  It holds none of the solver's
arithmetic, so both the FP64 oracle tests and the GPU path may consume it.

Every workload is an observation matrix ``D = L0 + S0`` (frames or bands
stacked as columns, so ``m`` = pixels and ``n`` = frames/bands, ``m >= n``),
an optional observation mask ``Q`` (True = observed, the subset of entries of
the compressive problem), the weight ``lam`` of the l1 term and the number of
restriction levels.  ``mu0`` is the initial penalty of the augmented
Lagrangian; it is a parameter of the workload, chosen as 1.25 / ||P_Q D||_2
(the customary inexact-ALM start), and is passed to both solvers.

Randomness: NumPy PCG64 with a fixed seed per workload.  Values are drawn in
FP64 and D is rounded to FP32 once; both solvers consume that rounded D
(the oracle promotes it back to FP64).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Workload",
    "gaussian_lowrank_plus_sparse",
    "range_conforming_lowrank_plus_sparse",
    "video_like",
    "hyperspectral_like",
    "config",
    "CONFIG_NAMES",
    "mu0_for",
    "fw_cpcp",
    "fw_config",
    "FW_CONFIG_NAMES",
]


@dataclasses.dataclass
class Workload:
    name: str
    D: np.ndarray                 # float32, m x n, C-contiguous
    Q: Optional[np.ndarray]       # bool m x n (True = observed) or None = fully observed
    L0: np.ndarray                # float64 ground-truth low-rank part
    S0: np.ndarray                # float64 ground-truth sparse part
    lam: float
    levels: int
    rank: int
    mu0: float
    tol: float = 1e-6
    recipe: str = ""
    lam_L: Optional[float] = None  # weight of the nuclear term (unconstrained CPCP only;
                                   # ``lam`` then weighs the l1 term)

    @property
    def m(self) -> int:
        return self.D.shape[0]

    @property
    def n(self) -> int:
        return self.D.shape[1]

    def mask_u8(self) -> Optional[np.ndarray]:
        return None if self.Q is None else self.Q.astype(np.uint8)


def mu0_for(D32: np.ndarray, Q: Optional[np.ndarray]) -> float:
    """Initial penalty 1.25 / ||P_Q D||_2 (spectral norm of the observed data)."""
    X = D32.astype(np.float64)
    if Q is not None:
        X = np.where(Q, X, 0.0)
    return 1.25 / float(np.linalg.norm(X, 2))


def _exact_support(rng, total: int, frac: float) -> np.ndarray:
    k = int(round(frac * total))
    return rng.choice(total, size=k, replace=False)


def _mask(rng, m: int, n: int, frac: float) -> np.ndarray:
    Q = np.zeros(m * n, dtype=bool)
    Q[_exact_support(rng, m * n, frac)] = True
    return Q.reshape(m, n)


def gaussian_lowrank_plus_sparse(m: int, n: int, rank: int, *, seed: int,
                                 sparse_frac: float, sparse_kind: str = "pm1",
                                 sparse_amp: float = 1.0,
                                 observed_frac: Optional[float] = None,
                                 levels: int = 2, lam: Optional[float] = None,
                                 name: str = "gaussian") -> Workload:
    """L0 = X Y^T with X (m x r), Y (n x r) i.i.d. N(0, 1/n); S0 on an exact
    uniform random support: values +-amp ("pm1") or U[-amp, amp] ("uniform")."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sd = 1.0 / math.sqrt(n)
    X = rng.normal(0.0, sd, size=(m, rank))
    Y = rng.normal(0.0, sd, size=(n, rank))
    L0 = X @ Y.T
    S0 = np.zeros(m * n)
    idx = _exact_support(rng, m * n, sparse_frac)
    if sparse_kind == "pm1":
        S0[idx] = sparse_amp * rng.choice([-1.0, 1.0], size=idx.size)
    elif sparse_kind == "uniform":
        S0[idx] = rng.uniform(-sparse_amp, sparse_amp, size=idx.size)
    else:
        raise ValueError(sparse_kind)
    S0 = S0.reshape(m, n)
    Q = None if observed_frac is None else _mask(rng, m, n, observed_frac)
    D = np.ascontiguousarray((L0 + S0).astype(np.float32))
    lam = (1.0 / math.sqrt(max(m, n))) if lam is None else lam
    return Workload(name, D, Q, L0, S0, lam, levels, rank, mu0_for(D, Q),
                    recipe=f"X,Y ~ N(0,1/{n}) rank {rank}; S0 {sparse_frac:.0%} {sparse_kind} amp {sparse_amp}; "
                           f"observed {observed_frac}; seed {seed}")


def range_conforming_lowrank_plus_sparse(m: int, n: int, rank: int, basis: np.ndarray, *, seed: int,
                                         sparse_frac: float = 0.05, levels: int = 2,
                                         observed_frac: Optional[float] = None,
                                         name: str = "conforming") -> Workload:
    """L0 = X (B W)^T whose rows lie in the column range of the given n x n_H
    matrix ``basis`` (used to build inputs where the coarse-model assumption
    L0 = L_H R^T holds exactly).  ``basis`` is supplied by the caller."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nH = basis.shape[1]
    X = rng.normal(0.0, 1.0 / math.sqrt(n), size=(m, rank))
    W = rng.normal(0.0, 1.0, size=(nH, rank))
    Yf = basis @ W
    Yf /= np.linalg.norm(Yf, axis=0, keepdims=True)
    L0 = X @ Yf.T
    S0 = np.zeros(m * n)
    idx = _exact_support(rng, m * n, sparse_frac)
    S0[idx] = rng.choice([-1.0, 1.0], size=idx.size)
    S0 = S0.reshape(m, n)
    Q = None if observed_frac is None else _mask(rng, m, n, observed_frac)
    D = np.ascontiguousarray((L0 + S0).astype(np.float32))
    return Workload(name, D, Q, L0, S0, 1.0 / math.sqrt(max(m, n)), levels, rank, mu0_for(D, Q),
                    recipe=f"rows of L0 in range(basis); rank {rank}; S0 {sparse_frac:.0%} +-1; seed {seed}")


def video_like(height: int = 240, width: int = 320, frames: int = 400, rank: int = 5, *,
               seed: int = 3, blur_px: float = 16.0, blobs_per_frame: int = 16, blob: int = 20,
               noise_var: float = 1e-3, levels: int = 3, name: str = "video") -> Workload:
    """Surveillance-video stand-in: frames stacked as columns (m = height*width).

    Background L0 = B W^T: B holds ``rank`` smooth spatial bases (Gaussian-blurred
    white noise), W slowly varying temporal weights 1 + 0.2 sin(2 pi f t / frames + phi)
    with distinct f <= 4 cycles per clip; L0 is scaled so max|L0| = 1.
    Foreground S0: moving blob x blob squares (constant velocity 1-4 px/frame,
    reflecting at the borders), pixel values U[0.3, 1] added to the background.
    Dense N(0, noise_var) noise on every entry (noise_var is a variance)."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.Generator(np.random.PCG64(seed))
    m = height * width
    B = np.empty((m, rank))
    for k in range(rank):
        img = gaussian_filter(rng.normal(size=(height, width)), blur_px, mode="wrap")
        img -= img.mean()
        img /= np.abs(img).max()
        B[:, k] = img.ravel() + (1.0 if k == 0 else 0.0)
    t = np.arange(frames)
    freqs = rng.permutation(np.arange(0, 5))[:rank].astype(float)
    if rank > 5:
        freqs = np.concatenate([freqs, rng.uniform(0.5, 4.0, size=rank - 5)])
    W = np.empty((frames, rank))
    for k in range(rank):
        W[:, k] = 1.0 + 0.2 * np.sin(2 * np.pi * freqs[k] * t / frames + rng.uniform(0, 2 * np.pi))
    L0 = B @ W.T
    L0 /= np.abs(L0).max()
    S0 = np.zeros((frames, height, width))
    pos = np.stack([rng.uniform(0, height - blob, blobs_per_frame),
                    rng.uniform(0, width - blob, blobs_per_frame)], axis=1)
    speed = rng.uniform(1.0, 4.0, blobs_per_frame)
    ang = rng.uniform(0, 2 * np.pi, blobs_per_frame)
    vel = np.stack([speed * np.sin(ang), speed * np.cos(ang)], axis=1)
    lim = np.array([height - blob, width - blob], dtype=float)
    for f in range(frames):
        for b in range(blobs_per_frame):
            y0, x0 = int(pos[b, 0]), int(pos[b, 1])
            S0[f, y0:y0 + blob, x0:x0 + blob] = rng.uniform(0.3, 1.0, size=(blob, blob))
        pos += vel
        for d in range(2):
            lo = pos[:, d] < 0
            hi = pos[:, d] > lim[d]
            pos[lo, d] = -pos[lo, d]
            pos[hi, d] = 2 * lim[d] - pos[hi, d]
            vel[lo | hi, d] = -vel[lo | hi, d]
    S0 = S0.reshape(frames, m).T.copy()
    noise = rng.normal(0.0, math.sqrt(noise_var), size=(m, frames))
    D = np.ascontiguousarray((L0 + S0 + noise).astype(np.float32))
    return Workload(name, D, None, L0, S0, 1.0 / math.sqrt(m), levels, rank, mu0_for(D, None),
                    recipe=f"{height}x{width}x{frames} video stand-in; rank {rank} smooth bases (blur {blur_px}px); "
                           f"{blobs_per_frame} moving {blob}x{blob} blobs U[0.3,1]; N(0,{noise_var}) noise; seed {seed}")


def hyperspectral_like(side: int = 512, bands: int = 200, endmembers: int = 8, *, seed: int = 5,
                       impulse_frac: float = 0.05, observed_frac: float = 0.30, levels: int = 4,
                       name: str = "hyperspectral") -> Workload:
    """Hyperspectral-cube stand-in: pixels as rows (m = side^2), bands as columns.

    L0 = A E^T with E (bands x endmembers): each spectrum a sum of 2-4 Gaussian
    bumps of width >= 20 bands, scaled to [0, 1]; abundance rows A ~ Dirichlet(0.5).
    S0: impulse_frac of entries, additive U[0, 1]; Q keeps observed_frac of entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = side * side
    b = np.arange(bands, dtype=float)
    E = np.zeros((bands, endmembers))
    for k in range(endmembers):
        for _ in range(int(rng.integers(2, 5))):
            c = rng.uniform(0, bands)
            w = rng.uniform(20.0, 60.0)
            E[:, k] += rng.uniform(0.3, 1.0) * np.exp(-0.5 * ((b - c) / w) ** 2)
        E[:, k] -= E[:, k].min()
        E[:, k] /= E[:, k].max()
    A = rng.dirichlet(0.5 * np.ones(endmembers), size=m)
    L0 = A @ E.T
    S0 = np.zeros(m * bands)
    idx = _exact_support(rng, m * bands, impulse_frac)
    S0[idx] = rng.uniform(0.0, 1.0, size=idx.size)
    S0 = S0.reshape(m, bands)
    Q = _mask(rng, m, bands, observed_frac)
    D = np.ascontiguousarray((L0 + S0).astype(np.float32))
    return Workload(name, D, Q, L0, S0, 1.0 / math.sqrt(m), levels, endmembers, mu0_for(D, Q),
                    recipe=f"{side}x{side}x{bands} cube stand-in; {endmembers} smooth endmembers x Dirichlet(0.5); "
                           f"{impulse_frac:.0%} U[0,1] impulses; {observed_frac:.0%} observed; seed {seed}")


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def config(name: str, scale: float = 1.0) -> Workload:
    """The five workloads.  ``scale`` < 1 shrinks the tall dimension (for quick
    tests); 1.0 gives the full sizes.

    c1  PCP 300x300, rank 10, 5% +-1, 2 levels
    c2  CPCP 2000x2000, rank 50, 10% U[-10,10], 60% observed, 3 levels
    c3  video PCP 76800x400 (240x320 frames), rank 5, 3 levels
    c4  PCP 1000x1000, rank 20, 5% +-1, 2 levels (unrolled / differentiated)
    c5  hyperspectral CPCP 262144x200 (512x512 pixels), rank 8, 30% observed, 4 levels
    """
    if name == "c1":
        w = gaussian_lowrank_plus_sparse(300, 300, 10, seed=1, sparse_frac=0.05, levels=2, name="c1")
        w.tol = 1e-7
        return w
    if name == "c2":
        return gaussian_lowrank_plus_sparse(2000, 2000, 50, seed=2, sparse_frac=0.10, sparse_kind="uniform",
                                            sparse_amp=10.0, observed_frac=0.60, levels=3, name="c2")
    if name == "c3":
        h = max(8, int(round(240 * scale)))
        return video_like(height=h, width=320, frames=400, levels=3, name="c3")
    if name == "c4":
        return gaussian_lowrank_plus_sparse(1000, 1000, 20, seed=4, sparse_frac=0.05, levels=2, name="c4")
    if name == "c5":
        side = max(16, int(round(512 * math.sqrt(scale))))
        return hyperspectral_like(side=side, bands=200, levels=4, name="c5")
    raise KeyError(name)


def fw_cpcp(m: int, n: int, rank: int, *, seed: int, levels: int, sparse_frac: float = 0.05,
            sparse_amp: float = 5.0, observed_frac: float = 0.8, delta: float = 0.02,
            name: str = "fw") -> Workload:
    """Synthetic unconstrained-CPCP data after the synthetic experiments of Sec. 4.1
    (D = L^ + S^ with rank-r L^ whose singular values decay as 1/k^2, sparse S^, part
    of the entries observed).  Sizes the paper leaves open are fixed here:

    L0 = U diag(s0 / k^2) V^T, U (m x r) orthonormal from a Gaussian, V (n x r)
    orthonormalised smooth curves cos(pi k t + phi_k), t in [0, 1], k = 0..r-1 (rows of
    L0 vary slowly along n, as the coarse model presumes); s0 gives L0 unit RMS.
    S0: ``sparse_frac`` of the entries, exact uniform support, values U[-amp, amp].
    Q: ``observed_frac`` of the entries, exact uniform support.
    lam_L = delta * observed_frac * s0 (a fraction of the top singular value of the
    observed low-rank part), lam_S = lam_L / sqrt(max(m, n)); both rounded to float32
    so that every solver sees the same values.  ``lam`` holds lam_S."""
    rng = np.random.Generator(np.random.PCG64(seed))
    U, _ = np.linalg.qr(rng.normal(size=(m, rank)))
    t = np.linspace(0.0, 1.0, n)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=rank)
    V = np.stack([np.cos(math.pi * k * t + phases[k]) for k in range(rank)], axis=1)
    V, _ = np.linalg.qr(V)
    decay = 1.0 / np.arange(1, rank + 1, dtype=np.float64) ** 2
    s0 = math.sqrt(m * n / float(np.sum(decay ** 2)))
    L0 = (U * (s0 * decay)) @ V.T
    S0 = np.zeros(m * n)
    idx = _exact_support(rng, m * n, sparse_frac)
    S0[idx] = rng.uniform(-sparse_amp, sparse_amp, size=idx.size)
    S0 = S0.reshape(m, n)
    Q = _mask(rng, m, n, observed_frac)
    D = np.ascontiguousarray((L0 + S0).astype(np.float32))
    lam_L = float(np.float32(delta * observed_frac * s0))
    lam_S = float(np.float32(lam_L / math.sqrt(max(m, n))))
    return Workload(name, D, Q, L0, S0, lam_S, levels, rank, 0.0, tol=1e-3, lam_L=lam_L,
                    recipe=f"L0 rank {rank}, sigma_k = s0/k^2, smooth right factors; S0 {sparse_frac:.0%} "
                           f"U[-{sparse_amp},{sparse_amp}]; observed {observed_frac:.0%}; lam_L {lam_L:.4g} "
                           f"lam_S {lam_S:.4g}; seed {seed}")


FW_CONFIG_NAMES = ("fw1", "fw2", "fw3", "fw4")


def fw_config(name: str, scale: float = 1.0) -> Workload:
    """The four synthetic CPCP problems of the Frank-Wolfe comparison (Table 2 sizes):

    fw1  10000 x 500,  rank 2, 3 levels (n_H = 63)
    fw2  10000 x 5000, rank 2, 7 levels (n_H = 40)
    fw3  10000 x 500,  rank 5, 3 levels
    fw4  10000 x 5000, rank 5, 7 levels

    ``scale`` < 1 shrinks m (for quick tests)."""
    sizes = {"fw1": (500, 2, 3, 11), "fw2": (5000, 2, 7, 12), "fw3": (500, 5, 3, 13), "fw4": (5000, 5, 7, 14)}
    n, rank, levels, seed = sizes[name]
    m = max(n, int(round(10000 * scale)))
    return fw_cpcp(m, n, rank, seed=seed, levels=levels, name=name)
