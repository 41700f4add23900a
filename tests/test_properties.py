"""Property-based checks over random small shapes (no GPU).

The oracle on random trains of 1-5 sites, mixed physical dimensions and
bonds that may exceed the structural bound:
* untruncated, it reproduces the brute-force product A(x) B(x) (Sec. II);
* the product commutes (up to rounding) where nothing is truncated;
* truncated, its error lies between the Eckart-Young bound at every cut and
  the sum of the discarded norms of Eq. (eps).
The gradient of <W, A*B> equals the dense sum and satisfies Euler's identity
at every core.  The conventional product is exact before rounding, and its
rounding error lies between the Eckart-Young bound and the TT-SVD bound.
The library's size query, on random shapes and options, gives the output
capacity its header states, and that capacity holds the oracle's product.
"""
import ctypes

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle as O
from paper_2410_19747_amd import _abi

SETTINGS = settings(max_examples=40, deadline=None, derandomize=True)


@st.composite
def train_pair(draw, max_sites=5, max_d=3, max_bond=4):
    n = draw(st.integers(1, max_sites))
    d = [draw(st.integers(1, max_d)) for _ in range(n)]
    seed = draw(st.integers(0, 2 ** 31))
    rng = np.random.default_rng(seed)

    def train():
        b = [1] + [draw(st.integers(1, max_bond)) for _ in range(n - 1)] + [1]
        return [rng.standard_normal((b[i], d[i], b[i + 1])) for i in range(n)]

    return train(), train()


def _exact(A, B):
    return O.dense(A) * O.dense(B)


@SETTINGS
@given(train_pair())
def test_untruncated_product_is_the_brute_force_product(pair):
    A, B = pair
    res = O.ttm(A, B, 10 ** 6, 0.0, chi_mid=0)
    ref = _exact(A, B)
    if np.linalg.norm(ref) == 0.0:
        assert np.abs(O.dense(res.cores)).max() == 0.0
    else:
        assert O.rel_frob(res.cores, ref) <= 1e-12
    n = len(A)
    assert res.n_contract == n and res.n_swap == n * (n - 1) // 2


@SETTINGS
@given(train_pair())
def test_untruncated_product_commutes(pair):
    A, B = pair
    ab = O.ttm(A, B, 10 ** 6, 0.0, chi_mid=0).cores
    ba = O.ttm(B, A, 10 ** 6, 0.0, chi_mid=0).cores
    scale = np.linalg.norm(_exact(A, B))
    assert np.linalg.norm(O.dense(ab) - O.dense(ba)) <= 1e-12 * max(scale, 1e-300)


@SETTINGS
@given(train_pair(max_sites=5, max_d=3, max_bond=4), st.integers(1, 4))
def test_truncated_error_between_eckart_young_and_discarded_sum(pair, chi):
    A, B = pair
    res = O.ttm(A, B, chi, 1e-14)
    ref = _exact(A, B)
    err = np.linalg.norm(O.dense(res.cores) - ref)
    nrm = np.linalg.norm(ref)
    assert max(O.bonds_of(res.cores)) <= chi
    assert err <= res.error_bound * (1 + 1e-9) + 1e-12 * nrm
    shape = ref.shape
    for k in range(1, len(shape)):
        s = np.linalg.svd(ref.reshape(int(np.prod(shape[:k])), -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[chi:] ** 2)) * (1 - 1e-9) - 1e-12 * nrm


class _Train:
    def __init__(self, phys, bonds):
        n = len(phys)
        self.p = (ctypes.c_int32 * n)(*phys)
        self.b = (ctypes.c_int32 * (n + 1))(*bonds)
        self.o = (ctypes.c_int64 * n)(*([0] * n))
        self.view = _abi.TtmTT(n, ctypes.cast(self.p, _abi.I32P), ctypes.cast(self.b, _abi.I32P),
                               ctypes.cast(self.o, _abi.I64P), ctypes.c_void_p(0x1000), 0)


_LIB = []


def _lib():
    if not _LIB:
        _LIB.append(_abi.load_library())
    return _LIB[0]


@settings(max_examples=300, deadline=None, derandomize=True)
@given(st.data())
def test_query_capacity(data):
    """With the final sweep, out_capacity = sum_i c_i d_i c_{i+1} with
    c_i = min(prod_{k<i} d_k, prod_{k>=i} d_k, chi_out, chi_mid if > 0), as
    the header states.  With or without it, the capacity holds what the product writes:
    the oracle's cores at eps = 0 (every nonzero value kept up to the caps)."""
    L = _lib()
    n = data.draw(st.integers(1, 6))
    d = [data.draw(st.integers(1, 4)) for _ in range(n)]
    ba = [1] + [data.draw(st.integers(1, 5)) for _ in range(n - 1)] + [1]
    bb = [1] + [data.draw(st.integers(1, 5)) for _ in range(n - 1)] + [1]
    chi = data.draw(st.integers(1, 24))
    chi_mid = data.draw(st.sampled_from([-1, 0, 3, 17]))
    final_round = data.draw(st.booleans())
    opt = _abi.TtmOptions()
    L.ttm_default_options(ctypes.byref(opt))
    opt.chi_mid = chi_mid
    opt.final_round = 1 if final_round else 0
    ws, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    A, B = _Train(d, ba), _Train(d, bb)
    rc = L.ttm_query(ctypes.byref(A.view), ctypes.byref(B.view), chi, ctypes.byref(opt), ctypes.byref(ws),
                     ctypes.byref(cap))
    assert rc == 0 and ws.value > 0
    if final_round:
        bound = chi if chi_mid <= 0 else min(chi, chi_mid)
        c = [1] * (n + 1)
        for i in range(1, n):
            c[i] = min(int(np.prod(d[:i])), int(np.prod(d[i:])), bound)
        assert cap.value == sum(c[i] * d[i] * c[i + 1] for i in range(n))
    rng = np.random.default_rng(data.draw(st.integers(0, 2 ** 31)))
    At = [rng.standard_normal((ba[i], d[i], ba[i + 1])) for i in range(n)]
    Bt = [rng.standard_normal((bb[i], d[i], bb[i + 1])) for i in range(n)]
    res = O.ttm(At, Bt, chi, 0.0, chi_mid=None if chi_mid == -1 else chi_mid, final_round=final_round)
    assert sum(c.size for c in res.cores) <= cap.value


@settings(max_examples=200, deadline=None, derandomize=True)
@given(st.data())
def test_conventional_query_capacity(data):
    """The variational fit keeps the structural bonds capped at chi_out:
    out_capacity = sum_i c_i d_i c_{i+1}, c_i = min(prod_{k<i} d_k,
    prod_{k>=i} d_k, chi_out), whatever the input bonds."""
    L = _lib()
    n = data.draw(st.integers(1, 7))
    d = [data.draw(st.integers(1, 5)) for _ in range(n)]
    ba = [1] + [data.draw(st.integers(1, 9)) for _ in range(n - 1)] + [1]
    bb = [1] + [data.draw(st.integers(1, 9)) for _ in range(n - 1)] + [1]
    chi = data.draw(st.integers(1, 40))
    ws, cap = ctypes.c_size_t(0), ctypes.c_int64(0)
    A, B = _Train(d, ba), _Train(d, bb)
    rc = L.conventional_query(ctypes.byref(A.view), ctypes.byref(B.view), chi, None, ctypes.byref(ws),
                              ctypes.byref(cap))
    assert rc == 0 and ws.value > 0
    c = [1] * (n + 1)
    for i in range(1, n):
        c[i] = min(int(np.prod(d[:i])), int(np.prod(d[i:])), chi)
    assert cap.value == sum(c[i] * d[i] * c[i + 1] for i in range(n))


@SETTINGS
@given(st.data())
def test_gradient_value_and_euler_identity(data):
    """<W, A*B> equals the dense sum, and L is linear in every core, so
    <dL/dA_k, A_k> = <dL/dB_k, B_k> = L at every site."""
    n = data.draw(st.integers(1, 5))
    d = [data.draw(st.integers(1, 3)) for _ in range(n)]
    rng = np.random.default_rng(data.draw(st.integers(0, 2 ** 31)))

    def train():
        b = [1] + [data.draw(st.integers(1, 4)) for _ in range(n - 1)] + [1]
        return [rng.standard_normal((b[i], d[i], b[i + 1])) for i in range(n)]

    W, A, B = train(), train(), train()
    val, dA, dB = O.inner3_grad(W, A, B)
    ref = float(np.sum(O.dense(W) * O.dense(A) * O.dense(B)))
    scale = float(np.sum(np.abs(O.dense(W) * O.dense(A) * O.dense(B))))
    assert abs(val - ref) <= 1e-12 * max(scale, 1e-300)
    for k in range(n):
        assert dA[k].shape == A[k].shape and dB[k].shape == B[k].shape
        assert abs(float(np.sum(dA[k] * A[k])) - val) <= 1e-12 * max(scale, 1e-300)
        assert abs(float(np.sum(dB[k] * B[k])) - val) <= 1e-12 * max(scale, 1e-300)


@SETTINGS
@given(train_pair(), st.integers(1, 4))
def test_conventional_products(pair, chi):
    """Eq. (carriageXi): the Kronecker carriages give A*B exactly; rounded
    at cap chi, the error is at least the Eckart-Young bound at every cut and
    at most the root of the summed squared tails (one per cut, N - 1 of
    them)."""
    A, B = pair
    ref = _exact(A, B)
    nrm = np.linalg.norm(ref)
    K = O.kron_cores(A, B)
    assert np.linalg.norm(O.dense(K) - ref) <= 1e-12 * max(nrm, 1e-300)
    R = O.conventional_exact(A, B, chi, 0.0)
    assert max(O.bonds_of(R)) <= chi
    err = np.linalg.norm(O.dense(R) - ref)
    shape = ref.shape
    tails = []
    for k in range(1, len(shape)):
        s = np.linalg.svd(ref.reshape(int(np.prod(shape[:k])), -1), compute_uv=False)
        tail = float(np.sum(s[chi:] ** 2))
        tails.append(tail)
        assert err >= np.sqrt(tail) * (1 - 1e-9) - 1e-12 * nrm
    assert err <= np.sqrt(sum(tails)) * (1 + 1e-9) + 1e-12 * nrm
