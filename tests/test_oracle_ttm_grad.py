"""Pins of the oracle's reverse mode through the TTM product (no GPU).

oracle.ttm_vjp differentiates the truncated product C = TTM(A, B) step by
step.  Its pins do not use its own arithmetic: central differences of the
forward product (oracle.ttm, ranks held fixed) along random directions, the
gradient of the exact <W, A*B> (oracle.inner3_grad) where nothing is
truncated, and central differences of each primitive adjoint.
"""
import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

H = 1e-6


def _loss(W, A, B, chi, eps, forced=None, **kw):
    res = O.ttm(A, B, chi, eps, forced_ranks=forced, **kw)
    ones = [np.ones((1, c.shape[1], 1)) for c in res.cores]
    return O.inner3(W, res.cores, ones), res


def _cbar(W, cores):
    ones = [np.ones((1, c.shape[1], 1)) for c in cores]
    return O.inner3_grad(W, cores, ones)[1]


@pytest.mark.parametrize("n,d,chi_a,chi_b,chi,chi_w", [(4, 2, 3, 2, 3, 2), (6, 3, 4, 3, 5, 3), (5, 2, 4, 4, 3, 3)])
def test_vjp_matches_central_differences_truncated(n, d, chi_a, chi_b, chi, chi_w):
    """<W, TTM(A, B)> with every swap and the final sweep truncating: the
    reverse-mode gradient against central differences (h = 1e-6, ranks held
    at the unperturbed product's) along random directions."""
    A, B, W = I.random_tt(n, d, chi_a, 1), I.random_tt(n, d, chi_b, 2), I.random_tt(n, d, chi_w, 3)
    L0, res = _loss(W, A, B, chi, 1e-14)
    assert res.error_bound > 1e-4          # truncation drops weight
    C, Ab, Bb = O.ttm_vjp(A, B, chi, 1e-14, _cbar(W, res.cores))
    assert O.rel_frob(C, res.cores) == 0.0
    rng = np.random.default_rng(n * 10 + d)
    for _ in range(3):
        EA = [rng.standard_normal(a.shape) for a in A]
        EB = [rng.standard_normal(b.shape) for b in B]
        lp, _ = _loss(W, [a + H * e for a, e in zip(A, EA)], [b + H * e for b, e in zip(B, EB)], chi, 1e-14,
                      forced=res.ranks)
        lm, _ = _loss(W, [a - H * e for a, e in zip(A, EA)], [b - H * e for b, e in zip(B, EB)], chi, 1e-14,
                      forced=res.ranks)
        fd = (lp - lm) / (2 * H)
        an = sum(float(np.sum(x * y)) for x, y in zip(Ab + Bb, EA + EB))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3 * abs(L0)), (fd, an)


def test_vjp_equals_exact_gradient_without_truncation():
    """Where nothing is truncated TTM(A, B) = A * B, so the reverse mode must
    give the gradient of the exact <W, A*B> (three-train environments)."""
    A, B, W = I.random_tt(4, 2, 3, 1), I.random_tt(4, 2, 2, 2), I.random_tt(4, 2, 2, 3)
    _, res = _loss(W, A, B, 64, 1e-20, chi_mid=0)
    assert res.error_bound < 1e-12
    _, Ab, Bb = O.ttm_vjp(A, B, 64, 1e-20, _cbar(W, res.cores), chi_mid=0)
    _, gA, gB = O.inner3_grad(W, A, B)
    for x, y in zip(Ab + Bb, gA + gB):
        assert np.abs(x - y).max() <= 1e-9 * np.abs(y).max()


def test_vjp_gradient_differs_from_exact_when_truncating():
    """The reason for the reverse mode: with truncation the gradient of
    <W, TTM(A, B)> is not that of <W, A*B>."""
    A, B, W = I.random_tt(6, 3, 4, 1), I.random_tt(6, 3, 3, 2), I.random_tt(6, 3, 3, 3)
    _, res = _loss(W, A, B, 5, 1e-14)
    _, Ab, _ = O.ttm_vjp(A, B, 5, 1e-14, _cbar(W, res.cores))
    _, gA, _ = O.inner3_grad(W, A, B)
    num = np.sqrt(sum(np.sum((x - y) ** 2) for x, y in zip(Ab, gA)))
    den = np.sqrt(sum(np.sum(y ** 2) for y in gA))
    assert num / den > 1e-3


@pytest.mark.parametrize("m,n", [(7, 4), (4, 4), (3, 6)])
def test_qr_vjp_central_differences(m, n):
    rng = np.random.default_rng(m * 10 + n)
    M = rng.standard_normal((m, n))
    Qb = rng.standard_normal((m, min(m, n)))
    Rb = rng.standard_normal((min(m, n), n))

    def L(M):
        Q, R = np.linalg.qr(M, mode="reduced")
        return np.sum(Q * Qb) + np.sum(R * Rb)

    Q, R = np.linalg.qr(M, mode="reduced")
    g = O.qr_vjp(M, Q, R, Qb, Rb)
    for _ in range(3):
        E = rng.standard_normal(M.shape)
        fd = (L(M + H * E) - L(M - H * E)) / (2 * H)
        assert abs(fd - np.sum(g * E)) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("m,n,r", [(8, 6, 3), (6, 8, 3), (10, 10, 4)])
def test_trunc_svd_vjp_central_differences(m, n, r):
    """Outputs Z = M V_r and V_r^T, through a loss of their product (the
    projection of M on its leading right singular subspace, which does not
    depend on the singular vectors' signs or on rotations among them)."""
    rng = np.random.default_rng(m * 100 + n * 10 + r)
    M = rng.standard_normal((m, n))
    Y = rng.standard_normal((m, n))

    def L(M):
        _, _, vt = np.linalg.svd(M, full_matrices=False)
        Vr = vt[:r].T
        return np.sum(Y * (M @ Vr @ Vr.T))

    _, s, vt = np.linalg.svd(M, full_matrices=False)
    Vr = vt[:r].T
    g = O.trunc_svd_vjp(M, vt, s, r, Y @ Vr, (M @ Vr).T @ Y)
    for _ in range(3):
        E = rng.standard_normal(M.shape)
        fd = (L(M + H * E) - L(M - H * E)) / (2 * H)
        assert abs(fd - np.sum(g * E)) <= 1e-7 * max(1.0, abs(fd))
