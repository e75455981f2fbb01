"""FP64 CPU oracle for multilevel PCP / CPCP (Hovhannisyan, Panagakis, Parpas,
Zafeiriou, "Fast Multilevel Algorithms for Compressive Principle Component
Pursuit", arXiv 2206.13369).

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library, its C ABI
or its Python binding) may import, call, link or execute anything here; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark do.
The oracle shares no code with the GPU path.

It is a plain, slow, obviously-correct transcription of the method's steps in
NumPy float64 (LAPACK SVD as the one library primitive), plus a PyTorch-CPU
float64 copy of the unrolled solver for reference gradients:

* ``restriction``  interpolation restriction operator of Sec. 3.1, eq. (Rx),
                   its multi-level composite and the orthonormalised form
                   used by the coarse model.
* ``prox``         elementwise soft threshold and singular value thresholding
                   (the two closed-form subproblem solutions of Alg. 1).
* ``ialm``         inexact ALM (Alg. 1), multilevel inexact ALM (Alg. 4) and
                   their masked (compressive) form.
* ``unrolled``     K unrolled multilevel iterations with a fixed penalty
                   schedule, differentiated by torch.autograd in float64.
* ``fwt``          Frank-Wolfe Thresholding (Alg. 3) and its multilevel form
                   (Alg. 6) for the unconstrained CPCP problem, eq. (cpcp).

Every reading of a passage that is silent, garbled or ambiguous is listed in
the module where it is taken.
"""
from .restriction import (interp_level, composite_interp, coarse_dim, orthonormal_restriction,
                          restrict, prolong)
from .prox import shrink, svt, svt_prox
from .ialm import IALMResult, ialm, default_schedule
from .power import spectral_norm
from . import fwt

__all__ = [
    "interp_level", "composite_interp", "coarse_dim", "orthonormal_restriction", "restrict", "prolong",
    "shrink", "svt", "svt_prox", "IALMResult", "ialm", "default_schedule", "spectral_norm",
    "fwt",
]
