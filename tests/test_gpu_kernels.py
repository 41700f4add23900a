"""Kernel-level GPU parity: each building block against NumPy on random operands."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _env():
    import torch
    import paper_2410_19747_amd as T
    assert torch.cuda.is_available()
    return torch, T.lib()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("M,N,K,batch", [(1, 1, 1, 1), (16, 16, 4, 1), (70, 45, 33, 3), (130, 129, 200, 2)])
def test_gemm_rowmajor_batched(M, N, K, batch):
    torch, L = _env()
    _say("gemm %d %d %d %d" % (M, N, K, batch))
    rng = np.random.default_rng(M * 1000 + N)
    A = rng.standard_normal((batch, M, K))
    B = rng.standard_normal((batch, K, N))
    dA, dB = _dev(torch, A), _dev(torch, B)
    dC = torch.zeros(batch * M * N, dtype=torch.float64, device="cuda")
    rc = L.ttm_test_gemm(M, N, K, batch, _ptr(dA), K, 1, M * K, _ptr(dB), N, 1, K * N, _ptr(dC), M * N,
                         1, 1, N, 0, 1, 0, None)
    assert rc == 0
    C = dC.cpu().numpy().reshape(batch, M, N)
    assert np.allclose(C, A @ B, rtol=1e-13, atol=1e-13)


# Error of a reduced-precision product against the exact one, relative to
# |A| |B| (entrywise), for operands rounded to FP32 (unit roundoff 2^-24), to
# BF16 (2^-8) and split into three BF16 terms (about 2^-24), with FP32
# accumulation.  The bounds are a few unit roundoffs times sqrt(K).
PREC_BOUND = {1: 4e-7, 2: 2e-2, 3: 4e-7}


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 16), (70, 45, 33), (130, 129, 200)])
def test_gemm_reduced_precision(prec, M, N, K):
    """FP32, BF16 and 3 x BF16 operands with FP32 accumulation on the matrix
    cores (also checks the operand and accumulator lane layouts: a wrong one
    gives errors of order one)."""
    torch, L = _env()
    _say("gemm prec %d: %d %d %d" % (prec, M, N, K))
    rng = np.random.default_rng(M * 7 + N * 3 + K + prec)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    dA, dB = _dev(torch, A), _dev(torch, B)
    dC = torch.zeros(M * N, dtype=torch.float64, device="cuda")
    rc = L.ttm_test_gemm_prec(prec, M, N, K, _ptr(dA), K, 1, _ptr(dB), N, 1, _ptr(dC), N, None)
    assert rc == 0
    C = dC.cpu().numpy().reshape(M, N)
    scale = np.abs(A) @ np.abs(B)
    err = np.abs(C - A @ B) / scale
    assert err.max() <= PREC_BOUND[prec] * np.sqrt(K), err.max()
    if prec == 2:
        # BF16 really rounds: far above the FP32 level
        assert K < 8 or err.max() > 1e-5


def test_gemm_strided_operands_and_split_output():
    """Merge of a swap pair: theta[(a,e),(w,b)] stored as Theta[(a,w),(e,b)] column-major."""
    torch, L = _env()
    _say("gemm merge layout")
    rng = np.random.default_rng(5)
    Dl, dp, Dm, dx, Dr = 7, 3, 9, 4, 5
    P = rng.standard_normal((Dl, dp, Dm))
    X = rng.standard_normal((Dm, dx, Dr))
    m, n = Dl * dx, dp * Dr
    dP, dX = _dev(torch, P), _dev(torch, X)
    dW = torch.zeros(m * n, dtype=torch.float64, device="cuda")
    rc = L.ttm_test_gemm(Dl * dp, dx * Dr, Dm, 1, _ptr(dP), Dm, 1, 0, _ptr(dX), dx * Dr, 1, 0, _ptr(dW), 0,
                         dp, Dr, dx, m * Dr, 1, m, None)
    assert rc == 0
    theta = np.einsum("aec,cwb->aewb", P, X)
    Theta = theta.transpose(0, 2, 1, 3).reshape(m, n)
    W = dW.cpu().numpy().reshape(n, m).T      # column-major
    assert np.allclose(W, Theta, rtol=1e-13, atol=1e-13)
    # transposed (wide) layout
    dW.zero_()
    rc = L.ttm_test_gemm(Dl * dp, dx * Dr, Dm, 1, _ptr(dP), Dm, 1, 0, _ptr(dX), dx * Dr, 1, 0, _ptr(dW), 0,
                         dp, Dr, n * dx, Dr, n, 1, None)
    assert rc == 0
    Wt = dW.cpu().numpy().reshape(m, n)        # Theta^T column-major == Theta row-major
    assert np.allclose(Wt, Theta, rtol=1e-13, atol=1e-13)
    # transposed operand (a_cs != 1)
    At = rng.standard_normal((20, 30))
    dAt = _dev(torch, At)
    dB = _dev(torch, rng.standard_normal((20, 11)))
    dC = torch.zeros(30 * 11, dtype=torch.float64, device="cuda")
    rc = L.ttm_test_gemm(30, 11, 20, 1, _ptr(dAt), 1, 30, 0, _ptr(dB), 11, 1, 0, _ptr(dC), 0, 1, 1, 11, 0, 1, 0, None)
    assert rc == 0
    assert np.allclose(dC.cpu().numpy().reshape(30, 11), At.T @ dB.cpu().numpy(), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 3), (37, 11), (11, 37), (300, 64), (1024, 128), (1100, 100),
                                 (1500, 40), (2048, 48), (2500, 40), (5000, 33), (8192, 40)])
def test_qr(m, n):
    """Householder QR with explicit Q.  Panels of more than 2048 rows run on
    ceil(rows / 1024) workgroups with a grid barrier per column (2500: three,
    the last one partly filled; 5000: five, with a one-column last panel;
    8192: eight)."""
    torch, L = _env()
    _say("qr %d %d" % (m, n))
    rng = np.random.default_rng(m * 7 + n)
    M = rng.standard_normal((m, n))
    k = min(m, n)
    dM = _dev(torch, M)
    dQ = torch.zeros(m * k, dtype=torch.float64, device="cuda")
    dR = torch.zeros(k * n, dtype=torch.float64, device="cuda")
    dS = torch.zeros(int(L.ttm_test_qr_scratch(m, n)), dtype=torch.float64, device="cuda")
    assert L.ttm_test_qr(_ptr(dM), m, n, _ptr(dQ), _ptr(dR), _ptr(dS), None) == 0
    Q = dQ.cpu().numpy().reshape(m, k)
    R = dR.cpu().numpy().reshape(k, n)
    assert np.abs(Q.T @ Q - np.eye(k)).max() < 1e-13
    assert np.allclose(Q @ R, M, rtol=1e-12, atol=1e-12)
    assert np.allclose(np.tril(R, -1), 0.0)


def _svd(torch, L, M, eps=0.0, cap=0, forced=0, left_pow=1, right_pow=0, block_width=0):
    m, n = M.shape
    k = min(m, n)
    dM = _dev(torch, M)
    dl = torch.zeros(m * k, dtype=torch.float64, device="cuda")
    dr = torch.zeros(k * n, dtype=torch.float64, device="cuda")
    ds = torch.zeros(k, dtype=torch.float64, device="cuda")
    nbytes = int(L.ttm_test_svd_ws_bytes_bw(m, n, block_width))
    assert nbytes > 0
    ws = torch.zeros(nbytes // 8 + 1, dtype=torch.float64, device="cuda")
    rank = ctypes.c_int(0)
    sweeps = ctypes.c_int(0)
    rc = L.ttm_test_svd_bw(_ptr(dM), m, n, eps, cap, forced, left_pow, right_pow, _ptr(dl), _ptr(dr), _ptr(ds),
                           ctypes.byref(rank), ctypes.byref(sweeps), block_width, _ptr(ws), ws.numel() * 8,
                           None)
    assert rc == 0, rc
    r = rank.value
    return (dl.cpu().numpy()[: m * r].reshape(m, r), dr.cpu().numpy()[: r * n].reshape(r, n),
            ds.cpu().numpy(), r, sweeps.value)


@pytest.mark.parametrize("m,n", [(1, 1), (5, 1), (1, 5), (2, 2), (3, 3), (9, 3), (50, 30), (30, 50), (200, 200),
                                 (300, 290), (700, 520), (257, 1100), (300, 8192), (2100, 1500), (1500, 2100)])
def test_svd_full_rank(m, n):
    torch, L = _env()
    _say("svd %d %d" % (m, n))
    rng = np.random.default_rng(m * 31 + n)
    M = rng.standard_normal((m, n))
    left, right, s, r, sw = _svd(torch, L, M)
    ref = np.linalg.svd(M, compute_uv=False)
    assert r == min(m, n)
    assert np.allclose(s, ref, rtol=1e-12, atol=1e-14 * ref[0])
    assert np.allclose(left @ right, M, rtol=1e-12, atol=1e-12 * ref[0])
    assert np.abs(right @ right.T - np.eye(r)).max() < 1e-12   # V^T rows orthonormal
    _say("  sweeps %d" % sw)


def test_svd_power_law_truncated():
    torch, L = _env()
    _say("svd power law 256x192")
    rng = np.random.default_rng(9)
    m, n = 256, 192
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.arange(1, n + 1, dtype=float) ** -2.0
    M = (U * s) @ V.T
    left, right, sv, r, sw = _svd(torch, L, M, eps=1e-10, cap=0)
    ref = np.linalg.svd(M, compute_uv=False)
    assert np.allclose(sv, ref, rtol=1e-10, atol=1e-15)
    # rank rule on the reference values
    import oracle as O
    rr, _ = O.rank_rule(ref, 1e-10, 0)
    assert r == rr
    u, s2, vt = np.linalg.svd(M)
    best = (u[:, :r] * s2[:r]) @ vt[:r]
    assert np.linalg.norm(left @ right - best) <= 1e-12 * np.linalg.norm(M)
    # cap and forced
    _, _, _, r2, _ = _svd(torch, L, M, eps=1e-10, cap=17)
    assert r2 == 17
    _, _, _, r3, _ = _svd(torch, L, M, eps=1e-10, forced=5)
    assert r3 == 5


def test_svd_swap_size_2048_power_law():
    """An SVD at the largest swap size of chi = 256 (2048 x 2048; 16-column
    blocks, so 32-column pairs with the XOR pairing) against LAPACK: singular
    values, the rank rule with a cap, and the truncated factorisation against
    the best rank-r approximation."""
    torch, L = _env()
    _say("svd power law 2048x2048")
    rng = np.random.default_rng(21)
    n = 2048
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = (1.0 + np.arange(n)) ** -1.5
    M = (U * s) @ V.T
    ref = np.linalg.svd(M, compute_uv=False)
    left, right, sv, r, sw = _svd(torch, L, M, eps=1e-14, cap=256)
    assert r == 256
    assert np.allclose(sv, ref, rtol=1e-11, atol=1e-14 * ref[0])
    best = (U[:, :r] * s[:r]) @ V[:, :r].T
    assert np.linalg.norm(left @ right - best) <= 1e-11 * np.linalg.norm(M)
    assert np.abs(right @ right.T - np.eye(r)).max() < 1e-12
    _say("  sweeps %d" % sw)


@pytest.mark.parametrize("n,cap", [(1024, 128), (2048, 256), (4096, 512)])
def test_svd_64_column_pairs_power_law(n, cap):
    """The 64-column-pair Jacobi path (32-column blocks, 1024-thread solve
    with the rotation in LDS, circle pairing, three launches per round),
    which every 8192-row swap matrix of the chi = 1024 product takes, forced
    on power-law matrices small enough for LAPACK: singular values, the rank
    rule with a cap, the best rank-r approximation, orthonormal factors, and
    the same results within the parity bar as the 32-column-pair path.  At
    4096 each Gram workgroup sums two row chunks (as at 8192, where it sums
    eight)."""
    torch, L = _env()
    _say("svd 64-column pairs, power law %dx%d" % (n, n))
    rng = np.random.default_rng(n + 5)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = (1.0 + np.arange(n)) ** -1.5
    M = (U * s) @ V.T
    ref = np.linalg.svd(M, compute_uv=False)
    left, right, sv, r, sw = _svd(torch, L, M, eps=1e-14, cap=cap, block_width=32)
    assert r == cap
    assert np.allclose(sv, ref, rtol=1e-11, atol=1e-14 * ref[0])
    best = (U[:, :r] * s[:r]) @ V[:, :r].T
    assert np.linalg.norm(left @ right - best) <= 1e-11 * np.linalg.norm(M)
    assert np.abs(right @ right.T - np.eye(r)).max() < 1e-12
    _say("  sweeps %d" % sw)
    # the other orientation (left factor orthonormal) and the rank rule alone
    left2, right2, sv2, r2, _ = _svd(torch, L, M, eps=1e-6, cap=0, left_pow=0, right_pow=1, block_width=32)
    import oracle as O
    rr, _ = O.rank_rule(ref, 1e-6, 0)
    assert r2 == rr
    best2 = (U[:, :r2] * s[:r2]) @ V[:, :r2].T
    assert np.linalg.norm(left2 @ right2 - best2) <= 1e-11 * np.linalg.norm(M)
    assert np.abs(left2.T @ left2 - np.eye(r2)).max() < 1e-12
    # the automatic choice (32-column pairs) agrees within the parity bar
    left3, right3, _, r3, _ = _svd(torch, L, M, eps=1e-14, cap=cap)
    assert r3 == r
    assert np.linalg.norm(left3 @ right3 - left @ right) <= 1e-12 * np.linalg.norm(M)


def test_svd_gram_over_several_row_chunks():
    """32-column pairs with circle pairing at 2900 columns (not a power of
    two): 23 row chunks of 128, summed two at a time by the Gram workgroups,
    the last one alone.  Against LAPACK."""
    torch, L = _env()
    n, cap = 2900, 300
    _say("svd 32-column pairs, circle pairing, power law %dx%d" % (n, n))
    rng = np.random.default_rng(29)
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = (1.0 + np.arange(n)) ** -1.5
    M = (U * s) @ V.T
    ref = np.linalg.svd(M, compute_uv=False)
    left, right, sv, r, sw = _svd(torch, L, M, eps=1e-14, cap=cap)
    assert r == cap
    assert np.allclose(sv, ref, rtol=1e-11, atol=1e-14 * ref[0])
    best = (U[:, :r] * s[:r]) @ V[:, :r].T
    assert np.linalg.norm(left @ right - best) <= 1e-11 * np.linalg.norm(M)
    assert np.abs(right @ right.T - np.eye(r)).max() < 1e-12
    _say("  sweeps %d" % sw)


@pytest.mark.parametrize("m,n", [(1100, 1024), (1024, 1100), (700, 520)])
def test_svd_64_column_pairs_random(m, n):
    """Forced 64-column pairs on dense random matrices (full rank, odd block
    counts padded with zero columns) against LAPACK."""
    torch, L = _env()
    _say("svd 64-column pairs, random %dx%d" % (m, n))
    rng = np.random.default_rng(m * 7 + n)
    M = rng.standard_normal((m, n))
    left, right, s, r, sw = _svd(torch, L, M, block_width=32)
    ref = np.linalg.svd(M, compute_uv=False)
    assert r == min(m, n)
    assert np.allclose(s, ref, rtol=1e-12, atol=1e-14 * ref[0])
    assert np.allclose(left @ right, M, rtol=1e-12, atol=1e-12 * ref[0])
    assert np.abs(right @ right.T - np.eye(r)).max() < 1e-12
    _say("  sweeps %d" % sw)


def test_svd_rank_deficient_and_zero():
    torch, L = _env()
    _say("svd rank deficient")
    rng = np.random.default_rng(3)
    M = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 25))
    left, right, s, r, _ = _svd(torch, L, M, eps=1e-24)
    assert r == 3
    assert np.allclose(left @ right, M, atol=1e-12)
    Z = np.zeros((6, 4))
    left, right, s, r, _ = _svd(torch, L, Z, eps=1e-12)
    assert r == 1 and np.all(s == 0.0)


@pytest.mark.parametrize("m,n", [(300, 200), (1500, 1100), (2500, 600)])
def test_qr_block_pivoting(m, n):
    """launch_qr_inplace with block column pivoting (register, register + LDS
    and memory panels): S P = Q R, so R^T R equals the Gram matrix of the
    permuted columns, and the first pivot is the column of largest norm."""
    torch, L = _env()
    _say("qr pivoted %d %d" % (m, n))
    rng = np.random.default_rng(m + 3 * n)
    M = rng.standard_normal((m, n)) * np.exp(rng.uniform(-6, 6, n))[None, :]
    dS = torch.tensor(M.T.copy().reshape(-1), dtype=torch.float64, device="cuda")  # column-major
    perm = torch.arange(n, dtype=torch.int32, device="cuda")
    scratch = torch.zeros(int(L.ttm_test_qr_pivoted_scratch(m, n)), dtype=torch.float64, device="cuda")
    assert L.ttm_test_qr_pivoted(_ptr(dS), m, n, _ptr(perm), _ptr(scratch), None) == 0
    S = dS.cpu().numpy().reshape(n, m).T
    P = perm.cpu().numpy()
    assert sorted(P.tolist()) == list(range(n))
    k = min(m, n)
    R = np.triu(S[:k, :])
    MP = M[:, P]
    G = MP.T @ MP
    assert np.abs(R.T @ R - G).max() <= 1e-12 * np.abs(G).max()
    norms = np.linalg.norm(M, axis=0)
    assert abs(abs(R[0, 0]) - norms.max()) <= 1e-12 * norms.max()


def test_mfma_f64_rate_probe():
    """The FP64 matrix-core probe runs, writes finite sums, and reports a
    rate of the order of the published peak."""
    torch, L = _env()
    _say("mfma f64 rate probe")
    out = torch.empty(512 * 256, dtype=torch.float64, device="cuda")
    sec, fl = ctypes.c_double(0.0), ctypes.c_double(0.0)
    assert L.ttm_test_mfma_f64_rate(512, 2000, _ptr(out), ctypes.byref(sec), ctypes.byref(fl), None) == 0
    assert bool(torch.isfinite(out).all())
    assert fl.value == 512 * 4 * 2000 * 8 * 2048.0
    rate = fl.value / sec.value / 1e12
    _say("  %.1f TFLOP/s" % rate)
    assert 5.0 < rate < 200.0


@pytest.mark.parametrize("p,l,cond", [(1024, 256, 1e3), (700, 130, 1e6), (2048, 512, 1e4), (64, 64, 10.0)])
def test_cholqr2_orthonormalises(p, l, cond):
    """CholeskyQR2 (the orthonormalisation of the randomized swap SVD):
    blocked Cholesky of Y^T Y on 64 x 64 diagonal blocks, blocked triangular
    solve; ragged last block (l = 130), square case.  Q^T Q = I to rounding,
    span(Q) = span(Y), and no breakdown up to cond(Y) = 1e6."""
    torch, L = _env()
    _say("cholqr2 %dx%d cond %.0e" % (p, l, cond))
    rng = np.random.default_rng(p + l)
    U, _ = np.linalg.qr(rng.standard_normal((p, l)))
    V, _ = np.linalg.qr(rng.standard_normal((l, l)))
    Y = (U * np.geomspace(1.0, 1.0 / cond, l)) @ V.T
    dY = _dev(torch, Y.T)  # column-major p x l
    ws = torch.empty(L.ttm_test_cholqr2_ws_bytes(p, l) // 8 + 1, dtype=torch.float64, device="cuda")
    bd = ctypes.c_int(-1)
    rc = L.ttm_test_cholqr2(_ptr(dY), p, l, ctypes.byref(bd), _ptr(ws), ws.numel() * 8, None)
    assert rc == 0 and bd.value == 0
    Q = dY.cpu().numpy().T
    assert np.abs(Q.T @ Q - np.eye(l)).max() < 1e-13
    # Y lies in span(Q): the residual of its projection is at rounding level
    assert np.linalg.norm(Y - Q @ (Q.T @ Y)) <= 1e-13 * np.linalg.norm(Y)


def test_cholqr2_reports_breakdown():
    """A rank-deficient Y (two equal columns) raises the breakdown flag
    instead of returning a non-orthonormal Q."""
    torch, L = _env()
    _say("cholqr2 rank deficient")
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((512, 128))
    Y[:, 77] = Y[:, 5]
    dY = _dev(torch, Y.T)
    ws = torch.empty(L.ttm_test_cholqr2_ws_bytes(512, 128) // 8 + 1, dtype=torch.float64, device="cuda")
    bd = ctypes.c_int(-1)
    rc = L.ttm_test_cholqr2(_ptr(dY), 512, 128, ctypes.byref(bd), _ptr(ws), ws.numel() * 8, None)
    assert rc == 0 and bd.value == 1
    assert np.isfinite(dY.cpu().numpy()).all()
