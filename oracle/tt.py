"""TT basics for the oracle (test infrastructure; FP64, NumPy/LAPACK).

A tensor train is a list of float64 arrays, core i of shape
[r_{i-1}, d_i, r_i] with r_0 = r_N = 1: for each physical value the core is
the r_{i-1} x r_i carriage matrix of Eq. (TT).  The tensor's entry is the
product of the selected carriages, and its dense form uses C order with site 1
as the slowest index.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def bonds_of(cores):
    return [int(cores[0].shape[0])] + [int(c.shape[2]) for c in cores]


def dense(cores):
    """Decompress a TT: multiply the carriages for every index (Eq. TT)."""
    out = cores[0].reshape(cores[0].shape[1], cores[0].shape[2])
    for core in cores[1:]:
        out = out @ core.reshape(core.shape[0], -1)
        out = out.reshape(-1, core.shape[2])
    return out.reshape([c.shape[1] for c in cores])


def brute_force(A, B):
    """Reference product A*B elementwise, on the dense tensors (Sec. II)."""
    return dense(A) * dense(B)


def inner(X, Y):
    """<X, Y> = sum over all indices of X*Y, by transfer matrices."""
    env = np.ones((1, 1))
    for x, y in zip(X, Y):
        # env[a', b'] = sum_{a,b,s} env[a,b] x[a,s,a'] y[b,s,b']
        t = np.tensordot(env, x, axes=(0, 0))          # [b, s, a']
        env = np.tensordot(t, y, axes=([0, 1], [0, 1]))  # [a', b']
    return float(env[0, 0])


def inner3(W, A, B):
    """sum over all indices of W*A*B, by a three-TT environment sweep."""
    env = np.ones((1, 1, 1))
    for w, a, b in zip(W, A, B):
        t = np.tensordot(env, w, axes=(0, 0))            # [a, b, s, w']
        t = np.einsum("absw,asx->bswx", t, a)            # [b, s, w', a']
        env = np.einsum("bswx,bsy->wxy", t, b)           # [w', a', b']
    return float(env[0, 0, 0])


def svd(mat):
    """Thin SVD with singular values in descending order (LAPACK gesdd,
    falling back to gesvd if gesdd does not converge)."""
    try:
        return sla.svd(mat, full_matrices=False, lapack_driver="gesdd", check_finite=True)
    except np.linalg.LinAlgError:
        return sla.svd(mat, full_matrices=False, lapack_driver="gesvd", check_finite=True)


def rank_rule(s, eps, cap):
    """Number of singular values kept, and the discarded weight.

    Eq. (eps): the discarded set S holds the smallest singular values and is
    the largest set with sum_S lambda^2 / sum_all lambda^2 < eps.  Reading:
    r_eps = min{k >= 1 : tail_k < eps * total or tail_k == 0}, where
    tail_k = sum_{i > k} lambda_i^2 is accumulated from the smallest value
    upward in FP64 and total = tail_0.  Then r = min(r_eps, cap) for cap > 0.
    Returns (r, tail_r).
    """
    s = np.asarray(s, dtype=np.float64)
    n = s.shape[0]
    tails = [0.0] * (n + 1)
    acc = 0.0
    for k in range(n - 1, -1, -1):
        acc = acc + float(s[k]) * float(s[k])
        tails[k] = acc
    total = tails[0]
    r = n
    for k in range(1, n + 1):
        if tails[k] <= 0.0 or tails[k] < eps * total:
            r = k
            break
    r = max(r, 1)
    if cap is not None and cap > 0:
        r = min(r, int(cap))
    return r, tails[r]


def left_orthogonalize(cores):
    """QR sweep i = 1..N-1: core i <- Q, core i+1 <- R core i+1.

    The bond may shrink to min(r_{i-1} d_i, r_i) (reduced QR).  Returns new
    cores; the norm of the tensor ends up in the last core.
    """
    cores = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    for i in range(len(cores) - 1):
        rl, d, rr = cores[i].shape
        q, r = np.linalg.qr(cores[i].reshape(rl * d, rr), mode="reduced")
        k = q.shape[1]
        cores[i] = q.reshape(rl, d, k)
        cores[i + 1] = np.tensordot(r, cores[i + 1], axes=(1, 0))
    return cores


def right_orthogonalize(cores):
    """Mirror sweep i = N..2 by QR of the transposed unfolding (an LQ)."""
    cores = [np.array(c, dtype=np.float64, copy=True) for c in cores]
    for i in range(len(cores) - 1, 0, -1):
        rl, d, rr = cores[i].shape
        q, r = np.linalg.qr(cores[i].reshape(rl, d * rr).T, mode="reduced")
        k = q.shape[1]
        cores[i] = q.T.reshape(k, d, rr)
        cores[i - 1] = np.tensordot(cores[i - 1], r.T, axes=(2, 0))
    return cores


def is_left_orthonormal(core, tol=1e-12):
    rl, d, rr = core.shape
    m = core.reshape(rl * d, rr)
    return np.abs(m.T @ m - np.eye(rr)).max() <= tol


def is_right_orthonormal(core, tol=1e-12):
    rl, d, rr = core.shape
    m = core.reshape(rl, d * rr)
    return np.abs(m @ m.T - np.eye(rl)).max() <= tol


def tt_round(cores, chi, eps):
    """TT rounding: left QR sweep, then a right-to-left truncated SVD sweep
    applying the rule of Eq. (eps) with cap ``chi`` at every bond."""
    cores = left_orthogonalize(cores)
    for i in range(len(cores) - 1, 0, -1):
        rl, d, rr = cores[i].shape
        u, s, vt = svd(cores[i].reshape(rl, d * rr))
        r, _ = rank_rule(s, eps, chi)
        cores[i] = vt[:r].reshape(r, d, rr)
        cores[i - 1] = np.tensordot(cores[i - 1], u[:, :r] * s[:r], axes=(2, 0))
    return cores


def tt_norm(cores):
    """Frobenius norm from a left QR sweep (norm of the final centre)."""
    c = left_orthogonalize(cores)
    return float(np.linalg.norm(c[-1]))


def tt_sub(C, R):
    """The TT of C - R: first core [C_1 | -R_1], interior cores
    block-diagonal, last core [C_N ; R_N] (bond dimensions add)."""
    n = len(C)
    if n == 1:
        return [C[0] - R[0]]
    out = []
    for i, (c, r) in enumerate(zip(C, R)):
        cl, d, cr = c.shape
        rl, _, rr = r.shape
        if i == 0:
            core = np.concatenate([c, -r], axis=2)
        elif i == n - 1:
            core = np.concatenate([c, r], axis=0)
        else:
            core = np.zeros((cl + rl, d, cr + rr))
            core[:cl, :, :cr] = c
            core[cl:, :, cr:] = r
        out.append(core)
    return out


def rel_frob(C, R, dense_limit=1 << 24):
    """Gauge-free relative Frobenius error ||C - R|| / ||R||.

    ``R`` may be a TT (list of cores) or a dense array.  Dense when the grid
    has at most ``dense_limit`` points, else through the difference TT.
    """
    if isinstance(R, np.ndarray):
        dc = dense(C)
        return float(np.linalg.norm((dc - R).ravel()) / np.linalg.norm(R.ravel()))
    size = 1
    for c in C:
        size *= c.shape[1]
    if size <= dense_limit:
        dc, dr = dense(C), dense(R)
        return float(np.linalg.norm((dc - dr).ravel()) / np.linalg.norm(dr.ravel()))
    return tt_norm(tt_sub(C, R)) / tt_norm(R)
