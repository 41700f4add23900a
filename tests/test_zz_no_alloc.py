"""GPU test of ttm_multiply_static, the entry point that allocates nothing.

Two calls in a row through the C ABI, the second on a smaller input, each
compared with ttm_multiply_ex on the same inputs (same kernels: the results
must be bitwise equal, and within the FP64 parity bar of 1e-12 in any case);
the small product is also checked against the oracle.  The second call runs
on a static array that still holds the first call's data.
"""
import ctypes

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _run_both(T, A, B, chi, tol):
    Cs, ss = T.multiply_static(A, B, chi, tol)
    Cw, sw = T.multiply(A, B, chi, tol)
    torch.cuda.synchronize()
    return (Cs, ss), (Cw, sw)


def _packed_equal(C1, C2):
    n1 = sum(C1.bonds[i] * C1.phys[i] * C1.bonds[i + 1] for i in range(C1.n_sites))
    n2 = sum(C2.bonds[i] * C2.phys[i] * C2.bonds[i + 1] for i in range(C2.n_sites))
    return C1.bonds == C2.bonds and n1 == n2 and torch.equal(C1.data[:n1], C2.data[:n2])


def test_static_workspace_matches_workspace_entry():
    import paper_2410_19747_amd as T

    torch.cuda.set_device(0)
    L = T.lib()
    # first call: the 256^3 turbulence square at chi = 64 (19 MiB of workspace)
    ux = I.turbulence_qtt(256, 101, 64)
    print("static entry: 256^3 u_x*u_x chi=64", flush=True)
    A = T.pack(ux)
    (Cs, ss), (Cw, sw) = _run_both(T, A, A, 64, 1e-14)
    assert ss["ranks"] == sw["ranks"]
    big_s = [c.cpu().numpy() for c in Cs.cores()]
    big_w = [c.cpu().numpy() for c in Cw.cores()]
    assert O.rel_frob(big_s, big_w) <= 1e-12
    assert _packed_equal(Cs, Cw)
    # second call: smaller input (10 sites, d = 2, chi 8) on the same array
    print("static entry: R10 chi_out=8", flush=True)
    Ar, Br = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)
    (Cs2, ss2), (Cw2, sw2) = _run_both(T, Ar, Br, 8, 1e-14)
    assert ss2["ranks"] == sw2["ranks"]
    small_s = [c.cpu().numpy() for c in Cs2.cores()]
    assert O.rel_frob(small_s, [c.cpu().numpy() for c in Cw2.cores()]) <= 1e-12
    assert _packed_equal(Cs2, Cw2)
    ref = O.ttm(Ar, Br, 8, 1e-14)
    assert O.rel_frob(small_s, ref.cores) <= 1e-12
    assert ss2["ranks"] == ref.ranks
    # and the first product once more after the small one: unchanged
    print("static entry: 256^3 again", flush=True)
    Cs3, _ = T.multiply_static(A, A, 64, 1e-14)
    torch.cuda.synchronize()
    assert _packed_equal(Cs3, Cw)
    # a product beyond the static size is refused before any GPU work
    Abig = T.pack(I.random_tt(8, 8, 128, 3))
    with pytest.raises(T.TTMError) as ei:
        T.multiply_static(Abig, Abig, 128, 1e-14)
    assert ei.value.code == T.TTM_EWORKSPACE
    assert str(T._abi.TTM_STATIC_WS_BYTES) in str(ei.value)
    assert L.ttm_last_error() != b""
