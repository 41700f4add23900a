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
    """E_0 .. E_N (E_k has shape [rw_k, ra_k, rb_k])."""
    envs = [np.ones((1, 1, 1))]
    for w, a, b in zip(W, A, B):
        envs.append(np.einsum("wab,wsx,asy,bsz->xyz", envs[-1], w, a, b, optimize=True))
    return envs


def right_envs(W, A, B):
    """F_0 .. F_N (F_k has shape [rw_k, ra_k, rb_k])."""
    n = len(A)
    envs = [None] * (n + 1)
    envs[n] = np.ones((1, 1, 1))
    for k in range(n - 1, -1, -1):
        envs[k] = np.einsum("wsx,asy,bsz,xyz->wab", W[k], A[k], B[k], envs[k + 1], optimize=True)
    return envs


def inner3_grad(W, A, B):
    """(L, dL/dA cores, dL/dB cores) for L = <W, A*B>."""
    assert len(W) == len(A) == len(B)
    E = left_envs(W, A, B)
    F = right_envs(W, A, B)
    dA, dB = [], []
    for k in range(len(A)):
        dA.append(np.einsum("wab,wsx,bsz,xyz->asy", E[k], W[k], B[k], F[k + 1], optimize=True))
        dB.append(np.einsum("wab,wsx,asy,xyz->bsz", E[k], W[k], A[k], F[k + 1], optimize=True))
    return float(E[-1][0, 0, 0]), dA, dB
