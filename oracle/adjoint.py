"""Gradient of the loss <W, A*B> with respect to the cores of A and B
(test infrastructure; FP64, NumPy).

The paper has no gradients; this is the plain definition the GPU adjoint is
checked against.  L(A, B) = <W, A*B> = sum_x W(x) A(x) B(x) for three trains
with the same physical dimensions (the product of Sec. II, then the inner
product with a fixed train W).  L is linear in every core of A and of B, so
its gradient with respect to core k of A is the contraction of everything
except that core: the left environment of the sites before k, cores k of W
and B, and the right environment of the sites after k.  It is also the
gradient of <W, TTM(A, B)> wherever the truncations of Sec. II.B drop
nothing, since there the algorithm's result is A*B itself.

Environments (bond indices w, a, b of W, A, B at a cut):
  left  E_0 = 1,  E_{k+1}[w',a',b'] = sum E_k[w,a,b] W_k[w,s,w'] A_k[a,s,a'] B_k[b,s,b']
  right F_N = 1,  F_k[w,a,b]     = sum W_k[w,s,w'] A_k[a,s,a'] B_k[b,s,b'] F_{k+1}[w',a',b']
"""
from __future__ import annotations

import numpy as np


def left_envs(W, A, B):
    """E_0 .. E_N (E_k has shape [rw_k, ra_k, rb_k]); the sum over the
    physical index s is a loop, each term three tensordots."""
    envs = [np.ones((1, 1, 1))]
    for w, a, b in zip(W, A, B):
        E = envs[-1]
        nxt = np.zeros((w.shape[2], a.shape[2], b.shape[2]))
        for s in range(w.shape[1]):
            t = np.tensordot(E, w[:, s, :], axes=(0, 0))      # [a, b, w']
            t = np.tensordot(t, a[:, s, :], axes=(0, 0))      # [b, w', a']
            nxt += np.tensordot(t, b[:, s, :], axes=(0, 0))   # [w', a', b']
        envs.append(nxt)
    return envs


def right_envs(W, A, B):
    """F_0 .. F_N (F_k has shape [rw_k, ra_k, rb_k])."""
    n = len(A)
    envs = [None] * (n + 1)
    envs[n] = np.ones((1, 1, 1))
    for k in range(n - 1, -1, -1):
        w, a, b, F = W[k], A[k], B[k], envs[k + 1]
        cur = np.zeros((w.shape[0], a.shape[0], b.shape[0]))
        for s in range(w.shape[1]):
            t = np.tensordot(w[:, s, :], F, axes=(1, 0))      # [w, a', b']
            t = np.tensordot(t, a[:, s, :], axes=(1, 1))      # [w, b', a]
            cur += np.tensordot(t, b[:, s, :], axes=(1, 1))   # [w, a, b]
        envs[k] = cur
    return envs


def inner3_grad(W, A, B):
    """(L, dL/dA cores, dL/dB cores) for L = <W, A*B>."""
    assert len(W) == len(A) == len(B)
    E = left_envs(W, A, B)
    F = right_envs(W, A, B)
    dA, dB = [], []
    for k in range(len(A)):
        w, a, b, El, Fr = W[k], A[k], B[k], E[k], F[k + 1]
        ga = np.zeros(a.shape)
        gb = np.zeros(b.shape)
        for s in range(w.shape[1]):
            t = np.tensordot(El, w[:, s, :], axes=(0, 0))                      # [a, b, w']
            ua = np.tensordot(t, b[:, s, :], axes=(1, 0))                      # [a, w', b']
            ga[:, s, :] = np.tensordot(ua, Fr, axes=([1, 2], [0, 2]))          # [a, a']
            ub = np.tensordot(t, a[:, s, :], axes=(0, 0))                      # [b, w', a']
            gb[:, s, :] = np.tensordot(ub, Fr, axes=([1, 2], [0, 1]))          # [b, b']
        dA.append(ga)
        dB.append(gb)
    return float(E[-1][0, 0, 0]), dA, dB
