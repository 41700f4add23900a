"""Reverse mode of the TTM product through its truncated swaps (oracle;
test infrastructure; FP64, NumPy/LAPACK).

The paper has no gradients.  ``ttm_vjp`` differentiates the map
(A, B) -> C = TTM(A, B) of ``oracle.ttm`` (Sec. II.B) as it is computed:
the QR sweeps that canonicalise the inputs, the reversal of the second
train (Eq. (tensor)), the contractions (Eq. (contract)), the QR gauge moves,
the swaps (merge with leg exchange, truncated SVD under Eq. (eps), Fig. 1C)
and the final rounding sweep.  The ranks the truncations choose are piecewise
constant in the inputs and are held at the forward pass's values.  Given the
cotangent Cbar of the output cores (e.g. dL/dC for L = <W, C>), it returns
the cotangents of the input cores.

Steps and their adjoints (each written out below):
* contraction Pi[a, e, b] = sum_c K[a, e, c] X[c, e, b]: one product per e;
* QR of an unfolding M = Q R with R pushed into the next core: the reverse
  mode of the QR factorisation (Q^T dQ is antisymmetric and dR R^{-1} upper
  triangular), M_bar = [Q_bar + Q sym_l(R R_bar^T - Q_bar^T Q)] R^{-T} for a
  tall M, where sym_l keeps the lower triangle and mirrors it to the upper;
  a wide M = [X | Y] is handled through its leading square block;
* truncated SVD of an unfolding Theta with outputs Z = Theta V_r and V_r^T:
  V_r spans the leading eigenvectors of G = Theta^T Theta, whose first-order
  change along dG is sum_{j != i} v_j (v_j^T dG v_i) / (l_i - l_j)
  (l = sigma^2).  Rotations within the kept set change the bond's gauge only
  and leave the product unchanged, so only kept-dropped pairs (i kept, j
  dropped or in the null space, l_j = 0) contribute:
  G_bar = V_perp [F o (V_perp^T V_r_bar)] V_r^T with F_ji = 1 / (l_i - l_j),
  and Theta_bar = Z_bar V_r^T + Theta (G_bar + G_bar^T).  The gradient
  exists where the kept and dropped values are separated (l_r > l_{r+1}).
Only the default gauge (singular values into the moving carriage) is
differentiated.
"""
from __future__ import annotations

import numpy as np

from .tt import rank_rule, svd


def qr_vjp(M, Q, R, Qbar, Rbar):
    """Cotangent of M = Q R (reduced QR) from those of Q and R."""
    m, n = M.shape
    if m >= n:
        X = R @ Rbar.T - Qbar.T @ Q
        X = np.tril(X) + np.tril(X, -1).T
        # (Qbar + Q X) R^{-T}, by a triangular solve with R
        return np.linalg.solve(R, (Qbar + Q @ X).T).T
    # wide: M = [X | Y] with X the leading m x m block, R = [U | V]
    Xm, Y = M[:, :m], M[:, m:]
    Ybar = Q @ Rbar[:, m:]
    Xbar = qr_vjp(Xm, Q, R[:, :m], Qbar + Y @ Rbar[:, m:].T, Rbar[:, :m])
    return np.concatenate([Xbar, Ybar], axis=1)


def trunc_svd_vjp(mat, vt_full, s, r, Zbar, Vtbar):
    """Cotangent of ``mat`` (m x n) for the outputs Z = mat V_r (m x r) and
    V_r^T (r x n) of its truncated SVD.  ``vt_full`` holds the k = min(m, n)
    right singular vectors as rows (thin SVD), ``s`` the k values."""
    m, n = mat.shape
    k = vt_full.shape[0]
    V = vt_full.T                                   # n x k
    Vr = V[:, :r]
    lam = np.asarray(s, dtype=np.float64) ** 2
    Vrbar = mat.T @ Zbar + Vtbar.T                  # total cotangent of V_r (n x r)
    matbar = Zbar @ Vr.T
    # dropped values r..k-1
    Vp = V[:, r:]
    F = 1.0 / (lam[None, :r] - lam[r:, None])       # (k - r) x r, F[j, i] = 1 / (l_i - l_j)
    Gbar = Vp @ (F * (Vp.T @ Vrbar)) @ Vr.T
    # the null space of mat (n > k): l_j = 0, projector I - V V^T
    if n > k:
        Nbar = Vrbar - V @ (V.T @ Vrbar)
        Gbar = Gbar + (Nbar / lam[None, :r]) @ Vr.T
    matbar = matbar + mat @ (Gbar + Gbar.T)
    return matbar


def _merge(P, X):
    dl, dp, dm = P.shape
    _, dx, dr = X.shape
    theta = np.tensordot(P, X, axes=(2, 0))          # [a, e, w, b]
    return theta.transpose(0, 2, 1, 3).reshape(dl * dx, dp * dr)


def _merge_vjp(P, X, matbar):
    """Cotangents of P[a, e, c] and X[c, w, b] from that of the leg-exchanged
    unfolding Theta[(a, w), (e, b)] = sum_c P[a, e, c] X[c, w, b]."""
    dl, dp, dm = P.shape
    _, dx, dr = X.shape
    tb = matbar.reshape(dl, dx, dp, dr).transpose(0, 2, 1, 3)   # [a, e, w, b]
    Pbar = np.tensordot(tb, X, axes=([2, 3], [1, 2]))           # [a, e, c]
    Xbar = np.tensordot(P, tb, axes=([0, 1], [0, 1]))           # [c, w, b]
    return Pbar, Xbar


def _contract(K, X):
    dl, d, _ = K.shape
    out = np.empty((dl, d, X.shape[2]))
    for e in range(d):
        out[:, e, :] = K[:, e, :] @ X[:, e, :]
    return out


def _contract_vjp(K, X, Pibar):
    Kbar = np.empty_like(K)
    Xbar = np.empty_like(X)
    for e in range(K.shape[1]):
        Kbar[:, e, :] = Pibar[:, e, :] @ X[:, e, :].T
        Xbar[:, e, :] = K[:, e, :].T @ Pibar[:, e, :]
    return Kbar, Xbar


def ttm_vjp(A, B, chi_out, eps, Cbar, chi_mid=None, final_round=True, forced_ranks=None):
    """(C, A_bar, B_bar): the product C = TTM(A, B) (the schedule of
    ``oracle.ttm`` with the default gauge) and the cotangents of A's and B's
    cores for the cotangent ``Cbar`` of C's cores.  ``forced_ranks`` fixes the
    ranks (swaps, then the final sweep), e.g. for finite differences."""
    n = len(A)
    if chi_mid is None:
        chi_mid = chi_out
    forced = list(forced_ranks) if forced_ranks is not None else None
    tape = []

    def take_forced():
        return forced.pop(0) if forced is not None else None

    def qr_move(cores, p, label):
        rl, d, rr = cores[p].shape
        M = cores[p].reshape(rl * d, rr)
        Q, R = np.linalg.qr(M, mode="reduced")
        nxt = cores[p + 1]
        tape.append((label, p, M, Q, R, nxt))
        cores[p] = Q.reshape(rl, d, Q.shape[1])
        cores[p + 1] = np.tensordot(R, nxt, axes=(1, 0))

    # ---- forward pass, recording what the reverse pass needs
    A = [np.array(c, dtype=np.float64, copy=True) for c in A]
    B = [np.array(c, dtype=np.float64, copy=True) for c in B]
    for i in range(n - 1):
        qr_move(A, i, "qrA")
    for i in range(n - 1):
        qr_move(B, i, "qrB")
    Bt = [np.ascontiguousarray(b.transpose(2, 1, 0)) for b in B]      # Eq. (tensor)
    tape.append(("reverse",))
    Pi = [None] * n
    tape.append(("contract", n - 1, A[n - 1], Bt[n - 1]))
    Pi[n - 1] = _contract(A[n - 1], Bt[n - 1])
    for j in range(n - 2, -1, -1):
        for p in range(j + 1, n - 1):
            qr_move(Pi, p, "qrPi")
        X = Bt[j]
        for p in range(n - 1, j, -1):
            mat = _merge(Pi[p], X)
            u, s, vt = svd(mat)
            f = take_forced()
            r = rank_rule(s, eps, chi_mid)[0] if f is None else int(f)
            tape.append(("swap", p, j, Pi[p], X, mat, vt, s, r))
            dl, dp, _ = Pi[p].shape
            _, dx, dr = X.shape
            X = (u[:, :r] * s[:r]).reshape(dl, dx, r)
            Pi[p] = vt[:r].reshape(r, dp, dr)
        tape.append(("contract", j, A[j], X))
        Pi[j] = _contract(A[j], X)
    if final_round:
        for i in range(n - 1):
            rl, d, rr = Pi[i].shape
            M = Pi[i].reshape(rl * d, rr)
            u, s, vt = svd(M)
            f = take_forced()
            r = rank_rule(s, eps, chi_out)[0] if f is None else int(f)
            nxt = Pi[i + 1]
            Zt = s[:r, None] * vt[:r]                  # S_r V_r^T, pushed into the next core
            tape.append(("round", i, M, u, s, r, Zt, nxt, (rl, d, rr)))
            Pi[i] = u[:, :r].reshape(rl, d, r)
            Pi[i + 1] = np.tensordot(Zt, nxt, axes=(1, 0))
    C = Pi

    # ---- reverse pass
    Pib = [np.array(c, dtype=np.float64, copy=True) for c in Cbar]
    Ab = [None] * n
    Bb = [None] * n
    Btb = [None] * n
    Xb = None
    for entry in reversed(tape):
        kind = entry[0]
        if kind == "round":
            _, i, M, u, s, r, Zt, nxt, (rl, d, rr) = entry
            nb = Pib[i + 1]
            Ztb = np.tensordot(nb, nxt, axes=([1, 2], [1, 2]))     # r x rr
            Pib[i + 1] = np.tensordot(Zt, nb, axes=(0, 0))
            # Pi[i] = U_r and Zt^T = M^T U_r are the outputs of the truncated
            # SVD of M^T, whose right singular vectors are M's left ones
            Ub = Pib[i].reshape(rl * d, r)
            Mtb = trunc_svd_vjp(M.T, u.T, s, r, Ztb.T, Ub.T)
            Pib[i] = Mtb.T.reshape(rl, d, rr)
        elif kind == "contract":
            _, j, K, Xc = entry
            Kb, Xcb = _contract_vjp(K, Xc, Pib[j])
            Ab[j] = Kb
            Pib[j] = None
            if j == n - 1:
                Btb[n - 1] = Xcb
            else:
                Xb = Xcb
        elif kind == "swap":
            _, p, j, P, Xs, mat, vt, s, r = entry
            dl, dp, _ = P.shape
            _, dx, dr = Xs.shape
            matbar = trunc_svd_vjp(mat, vt, s, r, Xb.reshape(dl * dx, r), Pib[p].reshape(r, dp * dr))
            Pib[p], Xb = _merge_vjp(P, Xs, matbar)
            if p == n - 1:                              # the chain's first swap took B~_j
                Btb[j] = Xb
        elif kind == "reverse":
            for i in range(n):
                Bb[i] = np.ascontiguousarray(Btb[i].transpose(2, 1, 0))
        else:   # QR moves: qrA, qrB, qrPi
            _, p, M, Q, R, nxt = entry
            cb = {"qrA": Ab, "qrB": Bb, "qrPi": Pib}[kind]
            rl_d, rr = M.shape
            nb = cb[p + 1]
            Rb = np.tensordot(nb, nxt, axes=([1, 2], [1, 2]))
            nxtb = np.tensordot(R, nb, axes=(0, 0))
            Qb = cb[p].reshape(Q.shape)
            Mb = qr_vjp(M, Q, R, Qb, Rb)
            cb[p] = Mb.reshape(cb[p].shape[0], cb[p].shape[1], rr)
            cb[p + 1] = nxtb
    return C, Ab, Bb
