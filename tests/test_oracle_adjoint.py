"""Pins of the oracle's gradient of <W, A*B> (no GPU).

Each check comes from outside the environment formula: the dense sum over
all indices, the loss's linearity in each core (so a gradient entry is the
loss with that core replaced by a unit tensor), Euler's identity for a
function linear in a core, and central finite differences of the loss
<W, TTM(A, B)> computed by the oracle's TTM product where no truncation
drops anything.
"""
import itertools

import numpy as np

import oracle as O
import ttm_inputs as I


def _dense_loss(W, A, B):
    return float(np.sum(O.dense(W) * O.dense(A) * O.dense(B)))


def _trains(seed, n=4, d=(2, 3, 2, 3), chis=(3, 2, 2)):
    W = I.random_tt(n, list(d), chis[0], seed)
    A = I.random_tt(n, list(d), chis[1], seed + 1)
    B = I.random_tt(n, list(d), chis[2], seed + 2)
    return W, A, B


def test_value_is_dense_sum_and_inner3():
    W, A, B = _trains(10)
    v, dA, dB = O.inner3_grad(W, A, B)
    assert abs(v - _dense_loss(W, A, B)) <= 1e-13 * max(1.0, abs(v))
    assert abs(v - O.inner3(W, A, B)) <= 1e-13 * max(1.0, abs(v))
    assert [g.shape for g in dA] == [a.shape for a in A]
    assert [g.shape for g in dB] == [b.shape for b in B]


def test_gradient_entries_by_linearity_brute_force():
    """dL/dA_k[idx] is the loss with core k of A replaced by the unit tensor
    at idx (L is linear in that core), evaluated on the dense tensors."""
    W, A, B = _trains(20)
    _, dA, dB = O.inner3_grad(W, A, B)
    for X, dX, other, first in ((A, dA, B, True), (B, dB, A, False)):
        for k, core in enumerate(X):
            for idx in itertools.product(*[range(s) for s in core.shape]):
                unit = np.zeros_like(core)
                unit[idx] = 1.0
                Xk = list(X)
                Xk[k] = unit
                ref = _dense_loss(W, Xk, other) if first else _dense_loss(W, other, Xk)
                assert abs(dX[k][idx] - ref) <= 1e-13 * (1.0 + abs(ref)), (k, idx)


def test_euler_identity_every_core():
    """For L linear in core k: <dL/dA_k, A_k> = L, for every k and both trains."""
    W, A, B = _trains(30, n=6, d=(2, 2, 3, 2, 2, 3), chis=(4, 3, 5))
    v, dA, dB = O.inner3_grad(W, A, B)
    for g, a in zip(dA, A):
        assert abs(np.sum(g * a) - v) <= 1e-12 * max(1.0, abs(v))
    for g, b in zip(dB, B):
        assert abs(np.sum(g * b) - v) <= 1e-12 * max(1.0, abs(v))


def test_symmetry_in_the_two_factors():
    W, A, B = _trains(40)
    v1, dA1, dB1 = O.inner3_grad(W, A, B)
    v2, dA2, dB2 = O.inner3_grad(W, B, A)
    assert abs(v1 - v2) <= 1e-13 * max(1.0, abs(v1))
    for x, y in zip(dA1, dB2):
        assert np.allclose(x, y, rtol=0, atol=1e-13)


def test_central_differences_of_the_ttm_loss():
    """<W, TTM(A, B)> by the oracle's TTM product with every singular value
    kept (chi_out = chi_A chi_B, eps = 0): central differences with h = 1e-6
    along random directions match the gradient."""
    rng = np.random.default_rng(5)
    W = I.random_tt(5, 2, 4, 50)
    A = I.random_tt(5, 2, 2, 51)
    B = I.random_tt(5, 2, 2, 52)

    def loss(A_, B_):
        res = O.ttm(A_, B_, 4, 0.0, chi_mid=0)
        return O.inner(W, res.cores)

    _, dA, dB = O.inner3_grad(W, A, B)
    h = 1e-6
    for trial in range(3):
        EA = [rng.standard_normal(a.shape) for a in A]
        EB = [rng.standard_normal(b.shape) for b in B]
        plus = loss([a + h * e for a, e in zip(A, EA)], [b + h * e for b, e in zip(B, EB)])
        minus = loss([a - h * e for a, e in zip(A, EA)], [b - h * e for b, e in zip(B, EB)])
        fd = (plus - minus) / (2 * h)
        an = sum(np.sum(g * e) for g, e in zip(dA, EA)) + sum(np.sum(g * e) for g, e in zip(dB, EB))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (trial, fd, an)
