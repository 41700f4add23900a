"""The conventional product of Sec. II.A (oracle; test infrastructure).

Two forms:
* ``conventional_exact``: the Kronecker carriages of Eq. (carriageXi),
  Pi^s = K^s (x) M^s with bond chi*chi', followed by TT rounding.  Exact
  (before rounding) by construction; feasible only for small bonds.
* ``conventional_variational``: the single-site variational fit of Omega to
  Phi psi (the MPO form of Eq. (PhiMPO) applied to psi), never forming the
  Kronecker cores.  The paper gives only its name and cost; the reading used
  here: seeded initial guess, left-to-right then right-to-left sweeps, stop
  when the norm of the centre changes by at most tol relative between two
  full sweeps, or after max_sweeps.
"""
from __future__ import annotations

import numpy as np

from .tt import right_orthogonalize, tt_round
from ttm_inputs import structural_bonds

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _splitmix64(x):
    # SplitMix64 finaliser (Steele, Lea, Flood 2014).
    z = x & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64_uniform(seed, count, start=0):
    """Counter-based SplitMix64: output k is mix(seed + (k+1) * gamma),
    mapped to [-1, 1) as 2 * (z >> 11) * 2^-53 - 1."""
    out = np.empty(count)
    for k in range(count):
        z = _splitmix64((seed + (start + k + 1) * _GAMMA) & _MASK)
        out[k] = 2.0 * ((z >> 11) * (1.0 / 9007199254740992.0)) - 1.0
    return out


def initial_guess(phys, chi_out, seed):
    """Initial product guess: structural bonds capped at chi_out, entries from
    the counter-based generator, one counter across all cores in C order."""
    bonds = structural_bonds(phys, chi_out)
    cores = []
    start = 0
    for i, d in enumerate(phys):
        shape = (bonds[i], d, bonds[i + 1])
        cnt = shape[0] * shape[1] * shape[2]
        cores.append(splitmix64_uniform(seed, cnt, start).reshape(shape))
        start += cnt
    return cores


def kron_cores(A, B):
    """Eq. (carriageXi): Pi^s_{(m m')(n n')} = K^s_{mn} M^s_{m'n'}."""
    out = []
    for a, b in zip(A, B):
        al, d, ar = a.shape
        bl, _, br = b.shape
        core = np.empty((al * bl, d, ar * br))
        for s in range(d):
            core[:, s, :] = np.kron(a[:, s, :], b[:, s, :])
        out.append(core)
    return out


def conventional_exact(A, B, chi_out, eps):
    return tt_round(kron_cores(A, B), chi_out, eps)


def _local(L, a, b, R):
    """Optimal single-site core: sum L[c,a,b] A[a,s,a'] B[b,s,b'] R[c',a',b'],
    contracted in the chi^4 order (L B), then A over the shared s, then R."""
    t1 = np.tensordot(L, b, axes=(2, 0))                   # [c, a, s, b']
    t2 = np.einsum("casy,asx->csxy", t1, a)                # [c, s, a', b']
    return np.tensordot(t2, R, axes=([2, 3], [1, 2])), t2  # [c, s, c']


def _left_env(q, t2):
    # L'[c', a', b'] = sum_{c,s} q[c,s,c'] t2[c,s,a',b']
    return np.tensordot(q, t2, axes=([0, 1], [0, 1]))


def _right_env(c, a, b, R):
    u1 = np.tensordot(c, R, axes=(2, 0))                   # [c, s, a', b']
    u2 = np.einsum("asx,csxy->csay", a, u1)                # [c, s, a, b']
    return np.einsum("bsy,csay->cab", b, u2)               # [c, a, b]


def conventional_variational(A, B, chi_out, tol=1e-12, max_sweeps=10, seed=12345,
                             init=None):
    """Single-site variational fit of C ~ A*B with bonds capped at chi_out.

    Returns (cores, sweeps_run, norm_history).
    """
    n = len(A)
    phys = [c.shape[1] for c in A]
    C = initial_guess(phys, chi_out, seed) if init is None else [np.array(c) for c in init]
    C = right_orthogonalize(C)
    one = np.ones((1, 1, 1))
    R = [None] * (n + 1)
    R[n] = one
    for i in range(n - 1, 0, -1):
        R[i] = _right_env(C[i], A[i], B[i], R[i + 1])
    L = [None] * (n + 1)
    L[0] = one
    hist = []
    prev = None
    sweeps = 0
    for sweep in range(max_sweeps):
        sweeps += 1
        for i in range(n):
            c, t2 = _local(L[i], A[i], B[i], R[i + 1])
            if i < n - 1:
                rl, d, rr = c.shape
                q, r = np.linalg.qr(c.reshape(rl * d, rr), mode="reduced")
                k = q.shape[1]
                C[i] = q.reshape(rl, d, k)
                L[i + 1] = _left_env(C[i], t2)
            else:
                C[i] = c
        for i in range(n - 1, -1, -1):
            c, _ = _local(L[i], A[i], B[i], R[i + 1])
            if i > 0:
                rl, d, rr = c.shape
                q, r = np.linalg.qr(c.reshape(rl, d * rr).T, mode="reduced")
                k = q.shape[1]
                C[i] = q.T.reshape(k, d, rr)
                R[i] = _right_env(C[i], A[i], B[i], R[i + 1])
            else:
                C[i] = c
        nrm = float(np.linalg.norm(C[0]))
        hist.append(nrm)
        if prev is not None and abs(nrm - prev) <= tol * nrm:
            break
        prev = nrm
    return C, sweeps, hist
