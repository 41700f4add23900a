"""Plain FP64 CPU oracle for tensor-train multiplication (test infrastructure).

This package is test infrastructure, not product code.  It is a slow,
deliberately plain NumPy/LAPACK implementation of what the GPU library
computes, written from the paper (Michailidis, Fenton, Kiffner, "Tensor Train
Multiplication", arXiv 2410.19747).  Only the test suite, the package's smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library
never does, and the oracle imports nothing from the GPU library.

Contents
--------
tt            TT basics: dense decompression, inner products, QR gauge sweeps,
              the truncation rule of Eq. (eps), TT rounding, gauge-free errors.
ttm           The TTM algorithm of Sec. II.B: concatenation (Eq. tensor),
              Contract (Eq. contract), Swap with truncated SVD, QR gauge moves.
conventional  The conventional product of Sec. II.A: Kronecker cores
              (Eq. carriageXi) with rounding, and the single-site variational
              fit of A*B.
adjoint       Gradient of <W, A*B> with respect to the cores of A and B by
              three-train environments (the paper has no gradients).
"""
from .tt import (  # noqa: F401
    dense,
    brute_force,
    inner,
    inner3,
    tt_norm,
    tt_sub,
    rel_frob,
    left_orthogonalize,
    right_orthogonalize,
    rank_rule,
    svd,
    tt_round,
    bonds_of,
    is_left_orthonormal,
    is_right_orthonormal,
)
from .ttm import contract, swap, swap_centre_right, ttm, TTMResult, model_flops  # noqa: F401
from .conventional import (  # noqa: F401
    kron_cores,
    conventional_exact,
    conventional_variational,
    splitmix64_uniform,
    initial_guess,
)
from .adjoint import inner3_grad, left_envs, right_envs  # noqa: F401,E402
from .ttm_grad import ttm_vjp, qr_vjp, trunc_svd_vjp  # noqa: F401,E402
