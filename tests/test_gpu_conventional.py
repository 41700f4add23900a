"""GPU parity of conventional_multiply (the variational baseline of Sec. II.A)
against the oracle's conventional_variational with the same seed, tolerance
and sweep limit, and against brute force where the bond allows exactness."""
import sys

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _conv(A, B, chi, tol, **kw):
    import torch
    import paper_2410_19747_amd as T
    assert torch.cuda.is_available()
    C, st = T.conventional(A, B, chi, tol, **kw)
    return [c.detach().cpu().numpy() for c in C.cores()], st


def test_gpu_conventional_exact_r10():
    _say("case: conventional R10 chi_out=64")
    A, B = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)
    C, st = _conv(A, B, 64, 1e-13, max_sweeps=6)
    assert O.rel_frob(C, O.brute_force(A, B)) <= 1e-12
    ref, sweeps, _ = O.conventional_variational(A, B, 64, 1e-13, max_sweeps=6)
    assert st["sweeps"] == sweeps


def test_gpu_conventional_truncated_r10_vs_oracle():
    _say("case: conventional R10 chi_out=8")
    A, B = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)
    ref, sweeps, hist = O.conventional_variational(A, B, 8, 1e-13, max_sweeps=10, seed=12345)
    C, st = _conv(A, B, 8, 1e-13, max_sweeps=10, seed=12345)
    assert st["sweeps"] == sweeps
    # Same seed, same sweeps: the fits differ by rounding only.  The sweep map
    # does not amplify it (perturbing the oracle's input by 1e-15 moves its
    # output by 3e-15 here, and by 5e-15 on the 256^3 case below), so the FP64
    # bar of 1e-12 applies to these unconverged fits too.
    assert O.rel_frob(C, ref) <= 1e-12
    # both are (near-)optimal rank-8 approximations of the same tensor
    ex = O.brute_force(A, B)
    assert abs(O.rel_frob(C, ex) - O.rel_frob(ref, ex)) <= 1e-12


def test_gpu_conventional_t16():
    _say("case: conventional T16")
    A, B = I.turbulence_qtt(16, 201, 0), I.turbulence_qtt(16, 202, 0)
    ref, sweeps, _ = O.conventional_variational(A, B, 64, 1e-13, max_sweeps=8)
    C, st = _conv(A, B, 64, 1e-13, max_sweeps=8)
    assert O.rel_frob(C, O.brute_force(A, B)) <= 1e-12
    assert O.rel_frob(C, ref) <= 1e-12


def test_gpu_conventional_turbulence_chi64_vs_oracle():
    _say("case: conventional 256^3 chi=64")
    A = I.turbulence_qtt(256, 101, 64)
    ref, sweeps, _ = O.conventional_variational(A, A, 64, 1e-12, max_sweeps=4)
    C, st = _conv(A, A, 64, 1e-12, max_sweeps=4)
    assert st["sweeps"] == sweeps
    assert O.rel_frob(C, ref) <= 1e-12
    assert max(O.bonds_of(C)) <= 64


def test_gpu_conventional_zero_factor():
    """A zero factor: the fit is exactly zero, and the stop rule (a relative
    change of the centre's norm of at most tol) holds at once on the second
    sweep, as in the oracle."""
    _say("case: conventional zero factor")
    A = I.random_tt(6, 3, 4, 31)
    Z = [np.zeros_like(c) for c in A]
    C, st = _conv(Z, A, 8, 1e-13, max_sweeps=6)
    assert np.abs(O.dense(C)).max() == 0.0
    _, sweeps, _ = O.conventional_variational(Z, A, 8, 1e-13, max_sweeps=6)
    assert st["sweeps"] == sweeps == 2
