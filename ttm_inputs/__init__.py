"""Seeded synthetic inputs for TT multiplication.

This module generates the tensor trains that both the CPU oracle and the GPU
library multiply.  It holds no step of the multiplication itself: it builds
cores (random, closed-form, or compressed from a synthetic field) and nothing
else.

Core layout everywhere: a tensor train is a list of NumPy float64 arrays,
core ``i`` of shape ``[r_{i-1}, d_i, r_i]`` with ``r_0 = r_N = 1``
(the carriage of Eq. (TT): one ``r_{i-1} x r_i`` matrix per physical value).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "structural_bonds",
    "random_tt",
    "ones_tt",
    "exp_qtt",
    "sin_qtt",
    "cos_qtt",
    "poly1_qtt",
    "square_qtt",
    "const_qtt",
    "turbulence_component",
    "qtt_encode_3d",
    "tt_svd",
    "turbulence_qtt",
    "turbulence_qtt_device",
    "turbulence_qtt_binary_device",
    "advective_qtts_device",
    "ADVECTIVE_CHIS",
    "app_a_toy_tt",
]


def structural_bonds(phys, chi):
    """Bond caps r_i = min(prod_{k<=i} d_k, prod_{k>i} d_k, chi), r_0 = r_N = 1.

    This is Eq. (bond) generalised from d = 2 to per-site physical
    dimensions d_k.  ``chi <= 0`` means no cap.
    """
    n = len(phys)
    cap = 1 << 62
    bonds = [1] * (n + 1)
    for i in range(1, n):
        left = 1
        for k in range(i):
            left = min(left * int(phys[k]), cap)
        right = 1
        for k in range(i, n):
            right = min(right * int(phys[k]), cap)
        b = min(left, right)
        if chi and chi > 0:
            b = min(b, int(chi))
        bonds[i] = b
    return bonds


def random_tt(n_sites, d, chi, seed, scale=None):
    """Random TT with structural bonds capped at ``chi``.

    Entries are i.i.d. N(0,1) times ``scale`` (default 1/sqrt(2*chi)), drawn
    from NumPy's PCG64 stream ``seed`` core by core, left to right, in C order.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    phys = [d] * n_sites if np.isscalar(d) else list(d)
    bonds = structural_bonds(phys, chi)
    if scale is None:
        scale = 1.0 / np.sqrt(2.0 * chi)
    cores = []
    for i in range(n_sites):
        shape = (bonds[i], phys[i], bonds[i + 1])
        cores.append(rng.standard_normal(shape) * scale)
    return cores


def ones_tt(n_sites, d):
    """The all-ones tensor as a TT: every bond 1, every entry 1."""
    phys = [d] * n_sites if np.isscalar(d) else list(d)
    return [np.ones((1, p, 1)) for p in phys]


def _grid_weights(n_sites, dx):
    # x = a + dx * sum_i sigma_i 2^{i-1}: site 1 carries the finest bit
    # (the one-dimensional quantics encoding of the benchmark section).
    return [dx * float(2 ** i) for i in range(n_sites)]


def const_qtt(n_sites, value):
    cores = [np.ones((1, 2, 1)) for _ in range(n_sites)]
    cores[0] = cores[0] * value
    return cores


def exp_qtt(n_sites, c, a=0.0, dx=None):
    """QTT of exp(c x) on the 2^N grid x = a + dx * sum sigma_i 2^{i-1}; rank 1."""
    if dx is None:
        dx = 1.0 / (2 ** n_sites - 1)
    w = _grid_weights(n_sites, dx)
    cores = []
    for i in range(n_sites):
        core = np.empty((1, 2, 1))
        core[0, 0, 0] = 1.0
        core[0, 1, 0] = np.exp(c * w[i])
        cores.append(core)
    cores[0] = cores[0] * np.exp(c * a)
    return cores


def _trig_qtt(n_sites, c, a, dx, want_sin):
    if dx is None:
        dx = 1.0 / (2 ** n_sites - 1)
    w = _grid_weights(n_sites, dx)
    # state after site i: (cos phi_i, sin phi_i), phi_i = c*(a + partial sum)
    cores = []
    for i in range(n_sites):
        if i == 0:
            core = np.empty((1, 2, 2))
            for s in range(2):
                ph = c * (a + w[0] * s)
                core[0, s, :] = (np.cos(ph), np.sin(ph))
        else:
            core = np.empty((2, 2, 2))
            for s in range(2):
                th = c * w[i] * s
                ct, st = np.cos(th), np.sin(th)
                core[:, s, :] = [[ct, st], [-st, ct]]
        cores.append(core)
    last = cores[-1]
    col = 1 if want_sin else 0
    cores[-1] = last[:, :, col:col + 1].copy()
    return cores


def sin_qtt(n_sites, c, a=0.0, dx=None):
    """QTT of sin(c x); rank 2."""
    return _trig_qtt(n_sites, c, a, dx, True)


def cos_qtt(n_sites, c, a=0.0, dx=None):
    """QTT of cos(c x); rank 2."""
    return _trig_qtt(n_sites, c, a, dx, False)


def poly1_qtt(n_sites, a=0.0, dx=None):
    """QTT of x itself; rank 2 (state: 1, partial sum)."""
    if dx is None:
        dx = 1.0 / (2 ** n_sites - 1)
    w = _grid_weights(n_sites, dx)
    cores = []
    for i in range(n_sites):
        core = np.zeros((2, 2, 2))
        for s in range(2):
            t = w[i] * s
            core[:, s, :] = [[1.0, t], [0.0, 1.0]]
        cores.append(core)
    cores[0] = cores[0][0:1] + 0.0
    cores[0][0, :, 1] += a
    cores[-1] = cores[-1][:, :, 1:2].copy()
    return cores


def square_qtt(n_sites, a=0.0, dx=None):
    """QTT of x^2; rank 3 (state: 1, s, s^2)."""
    if dx is None:
        dx = 1.0 / (2 ** n_sites - 1)
    w = _grid_weights(n_sites, dx)
    cores = []
    for i in range(n_sites):
        core = np.zeros((3, 2, 3))
        for s in range(2):
            t = w[i] * s
            core[:, s, :] = [[1.0, t, t * t], [0.0, 1.0, 2.0 * t], [0.0, 0.0, 1.0]]
        cores.append(core)
    first = np.zeros((1, 2, 3))
    for s in range(2):
        t = a + w[0] * s
        first[0, s, :] = (1.0, t, t * t)
    cores[0] = first
    cores[-1] = cores[-1][:, :, 2:3].copy()
    return cores


def turbulence_component(n, seed, kprime=None):
    """One component of a 3D random-phase synthetic turbulence field on n^3.

    Follows the artificial turbulence recipe of App. B lifted to three
    dimensions: amplitude |u(k)| = c k^{-11/6} sigma(k) (the 3D analogue of the
    2D k^{-2} law, giving E(k) ~ k^{-5/3}), sigmoid cut-off
    sigma(k) = 1/(1+exp(beta (k - k'))) with beta = 2/k', random phases with
    theta(-k) = -theta(k) (taken from the FFT of real white noise, which has
    that symmetry), division by sqrt(2), a real inverse DFT, and modes with
    k = 0 or |k| > n/2 set to zero.  The grid is periodic with integer wave
    numbers; c is fixed by normalising the field to unit RMS.
    """
    if kprime is None:
        kprime = n / 8.0
    beta = 2.0 / kprime
    rng = np.random.Generator(np.random.PCG64(seed))
    noise = rng.standard_normal((n, n, n))
    phase = np.angle(np.fft.rfftn(noise))
    del noise
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kr = np.fft.rfftfreq(n, 1.0 / n)
    k = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2)
    with np.errstate(divide="ignore", over="ignore"):
        amp = np.where(k > 1e-16, k ** (-11.0 / 6.0), 0.0) / (1.0 + np.exp(beta * (k - kprime)))
    amp[k > n / 2.0] = 0.0
    uk = amp * np.exp(1j * phase) / np.sqrt(2.0)
    del amp, phase, k
    u = np.fft.irfftn(uk, s=(n, n, n), axes=(0, 1, 2))
    u /= np.sqrt(np.mean(u * u))
    return u


def qtt_encode_3d(field):
    """Reshape an n^3 field (n = 2^L) to the interleaved-bit order.

    Site s = 1..L carries bit s (most significant first) of x, y and z, with
    physical index eta_s = 4 x_s + 2 y_s + z_s.  Returns a dense array of
    shape (8,)*L in that site order.
    """
    n = field.shape[0]
    L = int(round(np.log2(n)))
    assert 2 ** L == n and field.shape == (n, n, n)
    t = field.reshape((2,) * (3 * L))
    order = []
    for s in range(L):
        order += [s, L + s, 2 * L + s]
    return t.transpose(order).reshape((8,) * L)


def tt_svd(dense, chi):
    """Left-to-right TT-SVD of a dense tensor, keeping at most ``chi`` values
    per bond (``chi <= 0``: no cap) and dropping exact zeros only."""
    shape = dense.shape
    n = len(shape)
    cores = []
    rest = dense.reshape(1, -1)
    r_left = 1
    for i in range(n - 1):
        mat = rest.reshape(r_left * shape[i], -1)
        u, s, vt = np.linalg.svd(mat, full_matrices=False)
        r = int(np.count_nonzero(s > 0))
        r = max(r, 1)
        if chi and chi > 0:
            r = min(r, chi)
        cores.append(u[:, :r].reshape(r_left, shape[i], r))
        rest = s[:r, None] * vt[:r]
        r_left = r
    cores.append(rest.reshape(r_left, shape[-1], 1))
    return cores


def turbulence_qtt(n, seed, chi, kprime=None):
    """QTT (N = log2 n sites, d = 8) of one synthetic turbulence component."""
    u = turbulence_component(n, seed, kprime)
    t = qtt_encode_3d(u)
    del u
    return tt_svd(t, chi)


def _spectrum_device(n, seed, kprime, device):
    """Random-phase spectrum of one component (the recipe of
    ``turbulence_component``, on ``device`` with torch's generator) and the
    rfft wave-number axes.  Returns (uk, k1, kr)."""
    import torch

    if kprime is None:
        kprime = n / 8.0
    beta = 2.0 / kprime
    f64 = torch.float64
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    noise = torch.randn((n, n, n), generator=g, dtype=f64, device=device)
    phase = torch.angle(torch.fft.rfftn(noise))
    del noise
    k1 = torch.fft.fftfreq(n, 1.0 / n, dtype=f64, device=device)
    kr = torch.fft.rfftfreq(n, 1.0 / n, dtype=f64, device=device)
    k = torch.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2)
    amp = torch.where(k > 1e-16, k.clamp_min(1e-16) ** (-11.0 / 6.0), torch.zeros_like(k))
    amp = amp / (1.0 + torch.exp(torch.clamp(beta * (k - kprime), max=700.0)))
    amp[k > n / 2.0] = 0.0
    del k
    uk = torch.polar(amp / np.sqrt(2.0), phase)
    return uk, k1, kr


def _interleave_device(u):
    """An n^3 device field in the interleaved-bit order of ``qtt_encode_3d``,
    flattened, in two passes (torch views hold at most 16 dimensions): high
    halves of the three coordinates, then low halves."""
    n = u.shape[0]
    L = int(round(np.log2(n)))
    h, lo = L // 2, L - L // 2

    def interleave(nb):
        return [a * nb + b for b in range(nb) for a in range(3)]

    t = u.reshape(2 ** h, 2 ** lo, 2 ** h, 2 ** lo, 2 ** h, 2 ** lo).permute(0, 2, 4, 1, 3, 5).contiguous()
    t = t.reshape((2,) * (3 * h) + (2 ** (3 * lo),)).permute(interleave(h) + [3 * h]).contiguous()
    t = t.reshape((2 ** (3 * h),) + (2,) * (3 * lo)).permute([0] + [1 + i for i in interleave(lo)])
    return t.contiguous().reshape(-1)


def _tt_compress_device(field, L, chi, d=8):
    """Left-to-right TT-SVD (L sites of dimension d) of a flattened
    interleaved field with at most ``chi`` values per bond, via the leading
    eigenvectors of each unfolding's Gram matrix on its smaller side."""
    import torch

    cores = []
    rest = field.reshape(1, -1)
    r_left = 1
    for i in range(L - 1):
        mat = rest.reshape(r_left * d, -1)
        m, ncol = mat.shape
        r = min(m, ncol, chi) if chi and chi > 0 else min(m, ncol)
        if m <= ncol:
            _, evec = torch.linalg.eigh(mat @ mat.T)
            U = evec[:, -r:].flip(1).contiguous()
            cores.append(U.reshape(r_left, d, r).cpu().numpy())
            rest = U.T @ mat
        else:
            _, evec = torch.linalg.eigh(mat.T @ mat)
            V = evec[:, -r:].flip(1).contiguous()
            US = mat @ V
            s = torch.linalg.norm(US, dim=0)
            U = US / torch.where(s > 0, s, torch.ones_like(s))
            cores.append(U.reshape(r_left, d, r).cpu().numpy())
            rest = s[:, None] * V.T
        r_left = r
    cores.append(rest.reshape(r_left, d, 1).cpu().numpy())
    return cores


def turbulence_qtt_device(n, seed, chis, device, kprime=None):
    """QTTs of one synthetic turbulence component for grids too large for
    the host path (1024^3: 8 GiB per field), one per bond cap in ``chis``.

    The recipe of ``turbulence_component`` / ``turbulence_qtt`` run with
    torch on ``device``: the same amplitudes and cut-off, phases from the FFT
    of seeded real white noise (torch's generator on the device, so not the
    host path's draws), unit RMS, the interleaved-bit order of
    ``qtt_encode_3d``.  The left-to-right TT-SVD takes the leading
    eigenvectors of each unfolding's Gram matrix (smaller side) instead of an
    SVD; for an input that only has to be a TT of this field's structure at
    bond cap chi, the squared conditioning of the Gram matrix is harmless.
    Returns {chi: list of float64 numpy cores [r, 8, r']}.
    """
    import torch

    uk, _, _ = _spectrum_device(n, seed, kprime, device)
    u = torch.fft.irfftn(uk, s=(n, n, n))
    del uk
    u /= torch.sqrt(torch.mean(u * u))
    field = _interleave_device(u)
    del u
    L = int(round(np.log2(n)))
    return {chi: _tt_compress_device(field, L, chi) for chi in chis}


def turbulence_qtt_binary_device(n, seed, chi, device, kprime=None):
    """The field of ``turbulence_qtt_device`` (same seed, same draws) as a
    binary QTT: each d = 8 site (bits x_s, y_s, z_s) split into three sites
    of dimension 2, 3 log2(n) sites in all, compressed at bond cap chi.  The
    flattened interleaved order is the same, so only the TT-SVD differs."""
    import torch

    uk, _, _ = _spectrum_device(n, seed, kprime, device)
    u = torch.fft.irfftn(uk, s=(n, n, n))
    del uk
    u /= torch.sqrt(torch.mean(u * u))
    field = _interleave_device(u)
    del u
    L = int(round(np.log2(n)))
    return _tt_compress_device(field, 3 * L, chi, d=2)


ADVECTIVE_CHIS = (512, 128, 64, 256, 32, 128, 64, 256, 32)


def advective_qtts_device(n, seed, chis=ADVECTIVE_CHIS, device="cuda", kprime=None):
    """Operands of the nine products u_j * d_j u_i (i, j in {x, y, z}; the
    sum over j is the advection term (u . grad) u_i of the momentum equation)
    for a synthetic turbulence velocity field on an n^3 grid.

    Component c in (x, y, z) is the field of ``turbulence_qtt_device`` drawn
    with seed ``seed + c``, scaled to unit RMS; its derivative along axis j
    is spectral, the inverse transform of i k_j u_c(k) with the same scale
    (the Nyquist plane of axis j set to zero so the result is real and the
    derivative exact for the band-limited field).  Product p = 3 i + j is
    compressed at bond cap ``chis[p]`` (both operands).  Returns a list of
    nine (A cores, B cores, chi): A = QTT of u_j, B = QTT of d_j u_i.
    """
    import torch

    L = int(round(np.log2(n)))
    cache = {}

    def compressed(key, chi, make):
        if (key, chi) not in cache:
            field = make()
            cache[(key, chi)] = _tt_compress_device(field, L, chi)
            del field
        return cache[(key, chi)]

    spectra = []
    scales = []
    for c in range(3):
        uk, k1, kr = _spectrum_device(n, seed + c, kprime, device)
        u = torch.fft.irfftn(uk, s=(n, n, n))
        scales.append(float(torch.sqrt(torch.mean(u * u))))
        del u
        spectra.append(uk)
    kz = kr.clone()
    kxy = k1.clone()
    kxy[n // 2] = 0.0
    if n % 2 == 0:
        kz[-1] = 0.0
    axes = [kxy[:, None, None], kxy[None, :, None], kz[None, None, :]]

    def velocity(c):
        def make():
            u = torch.fft.irfftn(spectra[c], s=(n, n, n)) / scales[c]
            return _interleave_device(u)
        return make

    def derivative(c, j):
        def make():
            du = torch.fft.irfftn(spectra[c] * (1j * axes[j]), s=(n, n, n)) / scales[c]
            return _interleave_device(du)
        return make

    out = []
    for i in range(3):
        for j in range(3):
            chi = int(chis[3 * i + j])
            A = compressed(("u", j), chi, velocity(j))
            B = compressed(("du", i, j), chi, derivative(i, j))
            out.append((A, B, chi))
    return out


def app_a_toy_tt(n_sites, d_rest=2, chi=4, seed=0):
    """The toy TT of App. A: the first two carriages are

        M^{s2=0} = (M^{s1=0})^T = 2^{-1/4} (1, 0),
        (M^{s2=1})^T = M^{s1=1} = 2^{-1/4} (0, 1),

    so bits 1 and 2 are maximally correlated with each other and with nothing
    else (the bond between carriages 2 and 3 is 1); carriages 3..N are random.
    """
    assert n_sites > 2
    rng = np.random.Generator(np.random.PCG64(seed))
    c = 2.0 ** -0.25
    m1 = np.zeros((1, 2, 2))
    m1[0, 0, :] = (c, 0.0)
    m1[0, 1, :] = (0.0, c)
    m2 = np.zeros((2, 2, 1))
    m2[:, 0, 0] = (c, 0.0)
    m2[:, 1, 0] = (0.0, c)
    phys = [2, 2] + [d_rest] * (n_sites - 2)
    rest_bonds = structural_bonds(phys[2:], chi)
    cores = [m1, m2]
    for i in range(n_sites - 2):
        cores.append(rng.standard_normal((rest_bonds[i], phys[2 + i], rest_bonds[i + 1])))
    return cores
