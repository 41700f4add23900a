"""TTM, step by step, as Sec. II.B describes it (oracle; test infrastructure).

Notation follows the paper: the first factor phi has carriages K (here ``A``),
the second factor psi has carriages M (here ``B``), the product Omega has
carriages Pi.  The chain of Eq. (tensor) is [A_1 ... A_N, B_N ... B_1] with
psi's carriages in reverse order; reversing a carriage list transposes each
carriage, so B~_i[b, w, a] = B_i[a, w, b].

Readings where the paper is silent or ambiguous (kept identical in the GPU
library):
* Both inputs are first brought to left-orthonormal form by a QR sweep in their
  own orientation; after reversal B's carriages are right-orthonormal, so the
  chain is in mixed-canonical gauge around the middle bond.
* Each swap absorbs the singular values into the carriage that keeps moving
  left (the one of psi), so the gauge centre always lies inside the next swap
  pair.  The truncated result is the same whichever carriage of the pair holds
  the centre.
* After a contraction the centre sits at the new Pi_j; QR moves carry it back
  to the right end of the Pi block before the next run of swaps.
* ``chi_mid`` caps every swap's rank (0: uncapped); ``final_round`` runs one
  left-to-right truncated-SVD sweep over the product with cap ``chi_out``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .tt import left_orthogonalize, rank_rule, svd


def contract(a_core, x_core):
    """Eq. (contract): Pi[m, eta, n] = sum_c K^eta[m, c] M^eta[c, n].

    The COPY tensor keeps only sigma = omega = eta, so this is one matrix
    product per physical value.
    """
    dl, d, dm = a_core.shape
    dm2, d2, dr = x_core.shape
    assert dm == dm2 and d == d2
    out = np.empty((dl, d, dr))
    for eta in range(d):
        out[:, eta, :] = a_core[:, eta, :] @ x_core[:, eta, :]
    return out


def _merge_and_split(p_core, x_core, eps, cap, forced):
    """The common part of a Swap (Fig. 1C, Eq. (eps)): the pair (p_core,
    x_core) = (P[a, eta, c], X[c, w, b]) is contracted over its shared bond,
    the physical legs are exchanged, the result is unfolded as rows (a, w)
    and columns (eta, b), and its SVD is truncated by the rule of Eq. (eps)
    (or at a forced rank).  Returns (u, s, vt, r, discarded weight)."""
    dl, dp, dm = p_core.shape
    dm2, dx, dr = x_core.shape
    assert dm == dm2
    theta = np.tensordot(p_core, x_core, axes=(2, 0))          # [a, eta, w, b]
    mat = theta.transpose(0, 2, 1, 3).reshape(dl * dx, dp * dr)  # (a, w) x (eta, b)
    u, s, vt = svd(mat)
    if forced is None:
        r, disc = rank_rule(s, eps, cap)
    else:
        r = int(forced)
        assert 1 <= r <= s.shape[0]
        disc = float(np.sum(s[r:][::-1] ** 2)) if r < s.shape[0] else 0.0
    return u, s, vt, r, disc


def swap(p_core, x_core, eps, cap, forced=None):
    """The Swap of Fig. 1C and Eq. (eps), the singular values kept in the
    carriage that moves on: X' = U_r S_r (moves left, carries the centre),
    P' = V_r^T.  Returns (X', P', r, discarded weight, singular values)."""
    dl, dp, _ = p_core.shape
    _, dx, dr = x_core.shape
    u, s, vt, r, disc = _merge_and_split(p_core, x_core, eps, cap, forced)
    x_new = (u[:, :r] * s[:r]).reshape(dl, dx, r)
    p_new = vt[:r].reshape(r, dp, dr)
    return x_new, p_new, r, disc, s


def swap_centre_right(p_core, x_core, eps, cap, forced=None):
    """The Swap with the gauge centre where the mixed-canonical paragraph of
    Sec. II.B puts it: on the right carriage of the pair, the singular values
    absorbed to the right (X' = U_r, P' = S_r V_r^T).  The next swap pairs X'
    with the carriage to its left, so the centre is first moved into X' by
    an LQ factorisation P' = L Q (X' <- X' L, P' <- Q).
    Returns (X', P', r, discarded weight, singular values, R) with R the
    triangular factor of the QR of P'^T (L = R^T)."""
    dl, dp, _ = p_core.shape
    _, dx, dr = x_core.shape
    u, s, vt, r, disc = _merge_and_split(p_core, x_core, eps, cap, forced)
    x_new = u[:, :r]                       # U_r, orthonormal columns
    p_new = s[:r, None] * vt[:r]           # S_r V_r^T holds the centre
    # LQ of P': the QR of its transpose, P'^T = Q R, so P' = R^T Q^T
    q, rf = np.linalg.qr(p_new.T, mode="reduced")
    x_new = x_new @ rf.T
    p_new = q.T
    return x_new.reshape(dl, dx, r), p_new.reshape(r, dp, dr), r, disc, s, rf


def _svd_flops(m, n, r):
    if m < n:
        m, n = n, m
    return 4.0 * m * n * n - (4.0 / 3.0) * n ** 3 + 4.0 * (m + n) * n * r


def _qr_flops(m, n):
    if m >= n:
        return 4.0 * m * n * n - (4.0 / 3.0) * n ** 3
    return 2.0 * n * m * m + (2.0 / 3.0) * m ** 3


def model_flops(ops):
    """Algorithmic flop count of a recorded operation list.

    contract: 2 d Dl Dm Dr; merge: 2 (Dl dx) Dm (dp Dr); SVD of m x n keeping
    r: 4 m n^2 - 4/3 n^3 + 4 (m + n) n r (m >= n); QR of m x n:
    4 m n^2 - 4/3 n^3 (m >= n); the R (or S V^T) product into the next core:
    2 k n (d Dnext).
    """
    total = 0.0
    for op in ops:
        kind = op[0]
        if kind == "contract":
            _, dl, d, dm, dr = op
            total += 2.0 * d * dl * dm * dr
        elif kind == "merge":
            _, dl, dp, dm, dx, dr = op
            total += 2.0 * dl * dx * dm * dp * dr
        elif kind == "svd":
            _, m, n, r = op
            total += _svd_flops(m, n, r)
        elif kind == "qr":
            _, m, n = op
            total += _qr_flops(m, n)
        elif kind == "gemm":
            _, m, k, n = op
            total += 2.0 * m * k * n
    return total


@dataclass
class TTMResult:
    cores: list
    ranks: list = field(default_factory=list)       # one per truncating SVD, in order
    discards: list = field(default_factory=list)    # discarded weight per SVD
    max_bond: int = 0
    n_contract: int = 0
    n_swap: int = 0
    n_qr: int = 0
    n_svd: int = 0
    ops: list = field(default_factory=list)

    @property
    def error_bound(self):
        """sum_k delta_k: each truncation at a centre changes the chain by
        delta_k in norm, later steps are isometries or projections."""
        return float(sum(np.sqrt(max(d, 0.0)) for d in self.discards))

    @property
    def flops(self):
        return model_flops(self.ops)


def _qr_move_right(cores, p, res):
    """Move the centre from cores[p] to cores[p+1] by a QR of cores[p]."""
    rl, d, rr = cores[p].shape
    q, r = np.linalg.qr(cores[p].reshape(rl * d, rr), mode="reduced")
    k = q.shape[1]
    nxt = cores[p + 1]
    res.ops.append(("qr", rl * d, rr))
    res.ops.append(("gemm", k, rr, nxt.shape[1] * nxt.shape[2]))
    res.n_qr += 1
    cores[p] = q.reshape(rl, d, k)
    cores[p + 1] = np.tensordot(r, nxt, axes=(1, 0))


def ttm(A, B, chi_out, eps, chi_mid=None, final_round=True, forced_ranks=None,
        canonicalize=True, move_factor="second", gauge="moving"):
    """The TTM product of two TTs, C = A * B elementwise.

    ``chi_mid``: rank cap of every swap (None: same as chi_out; 0: uncapped).
    ``forced_ranks``: optional list of ranks that replaces the rule of Eq.
    (eps) for each truncating SVD in order (swaps, then the final sweep).
    ``move_factor``: "second" (psi, as in Sec. II.B) or "smaller" (the
    train with the smaller largest bond is reversed and moved; ties: the
    second).  ``gauge``: "moving" (singular values into the carriage that
    moves on) or "right" (into the right carriage of the pair, as Sec. II.B
    states, followed by an LQ move of the centre, see swap_centre_right).
    """
    assert move_factor in ("second", "smaller") and gauge in ("moving", "right")
    if move_factor == "smaller":
        if max(c.shape[0] for c in A) < max(c.shape[0] for c in B):
            A, B = B, A
    n = len(A)
    assert len(B) == n and n >= 1
    for a, b in zip(A, B):
        assert a.shape[1] == b.shape[1], "physical dimensions differ"
    assert A[0].shape[0] == 1 and A[-1].shape[2] == 1
    assert B[0].shape[0] == 1 and B[-1].shape[2] == 1
    if chi_mid is None:
        chi_mid = chi_out
    forced = list(forced_ranks) if forced_ranks is not None else None
    res = TTMResult(cores=[])
    max_bond = max(max(c.shape[0] for c in A), max(c.shape[0] for c in B))

    def take_forced():
        if forced is None:
            return None
        return forced.pop(0)

    # Inputs to left-orthonormal form, each in its own orientation.
    if canonicalize:
        for tt in (A, B):
            # each QR acts on the core as the sweep has left it: its left bond
            # is the rank k of the previous QR
            rl = tt[0].shape[0]
            for i in range(n - 1):
                _, d, rr = tt[i].shape
                k = min(rl * d, rr)
                res.ops.append(("qr", rl * d, rr))
                res.ops.append(("gemm", k, rr, tt[i + 1].shape[1] * tt[i + 1].shape[2]))
                res.n_qr += 1
                rl = k
        A = left_orthogonalize(A)
        B = left_orthogonalize(B)
    else:
        A = [np.array(c, dtype=np.float64) for c in A]
        B = [np.array(c, dtype=np.float64) for c in B]

    # Eq. (tensor): psi enters reversed, each carriage transposed.
    Bt = [np.ascontiguousarray(b.transpose(2, 1, 0)) for b in B]

    Pi = [None] * n
    # Sites N are adjacent through the middle bond of size one.
    Pi[n - 1] = contract(A[n - 1], Bt[n - 1])
    res.ops.append(("contract", A[n - 1].shape[0], A[n - 1].shape[1], 1, Bt[n - 1].shape[2]))
    res.n_contract += 1
    max_bond = max(max_bond, Pi[n - 1].shape[0], Pi[n - 1].shape[2])

    for j in range(n - 2, -1, -1):
        # Centre sits at Pi[j+1]; carry it to the right end of the block.
        for p in range(j + 1, n - 1):
            _qr_move_right(Pi, p, res)
        x = Bt[j]
        for p in range(n - 1, j, -1):
            dl, dp, dm = Pi[p].shape
            _, dx, dr = x.shape
            res.ops.append(("merge", dl, dp, dm, dx, dr))
            if gauge == "moving":
                x, Pi[p], r, disc, _ = swap(Pi[p], x, eps, chi_mid, take_forced())
                res.ops.append(("svd", dl * dx, dp * dr, r))
            else:
                x, Pi[p], r, disc, _, _ = swap_centre_right(Pi[p], x, eps, chi_mid, take_forced())
                res.ops.append(("svd", dl * dx, dp * dr, r))
                res.ops.append(("qr", dp * dr, r))
                res.ops.append(("gemm", dl * dx, r, r))
                res.n_qr += 1
            res.ranks.append(r)
            res.discards.append(disc)
            res.n_swap += 1
            res.n_svd += 1
            max_bond = max(max_bond, r)
        res.ops.append(("contract", A[j].shape[0], A[j].shape[1], A[j].shape[2], x.shape[2]))
        Pi[j] = contract(A[j], x)
        res.n_contract += 1
        max_bond = max(max_bond, Pi[j].shape[0], Pi[j].shape[2])

    if final_round:
        # Left-to-right truncated sweep; the centre starts at Pi[0] and every
        # core to its right is right-orthonormal after the last run of swaps.
        for i in range(n - 1):
            rl, d, rr = Pi[i].shape
            u, s, vt = svd(Pi[i].reshape(rl * d, rr))
            f = take_forced()
            if f is None:
                r, disc = rank_rule(s, eps, chi_out)
            else:
                r = int(f)
                disc = float(np.sum(s[r:][::-1] ** 2)) if r < s.shape[0] else 0.0
            res.ops.append(("svd", rl * d, rr, r))
            nxt = Pi[i + 1]
            res.ops.append(("gemm", r, rr, nxt.shape[1] * nxt.shape[2]))
            res.ranks.append(r)
            res.discards.append(disc)
            res.n_svd += 1
            Pi[i] = u[:, :r].reshape(rl, d, r)
            Pi[i + 1] = np.tensordot(s[:r, None] * vt[:r], nxt, axes=(1, 0))
    res.cores = Pi
    res.max_bond = int(max_bond)
    return res
