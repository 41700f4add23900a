"""GPU parity of the adjoint: ttm_inner_grad against the oracle's gradient of
<W, A*B>, and the autograd loss <W, TTM(A, B)> against central differences
of the GPU loss itself, through the C ABI."""
import sys

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _host(packed):
    return [c.detach().cpu().numpy() for c in packed.cores()]


def _rel_cores(xs, ys):
    """Relative Frobenius distance of two lists of cores, core by core (the
    cores of a gradient are not a train, so no gauge freedom applies)."""
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(xs, ys))
    return np.sqrt(num / sum(float(np.sum(y ** 2)) for y in ys))


def _rel(xs, ys):
    num = np.sqrt(sum(np.sum((x - y) ** 2) for x, y in zip(xs, ys)))
    den = np.sqrt(sum(np.sum(y ** 2) for y in ys))
    return num / den


CASES = [
    # (n, d, chi_W, chi_A, chi_B, seed)
    (1, 5, 1, 1, 1, 1),
    (2, 3, 2, 3, 3, 2),
    (4, [2, 3, 2, 3], 3, 2, 2, 3),
    (6, 2, 5, 4, 3, 4),
    (8, 8, 16, 24, 20, 5),
    (10, [2, 8, 3, 8, 2, 8, 3, 8, 2, 8], 7, 33, 17, 6),
]


@pytest.mark.parametrize("case", CASES, ids=[str(c[:5]) for c in CASES])
def test_gpu_inner_grad_vs_oracle(case):
    import paper_2410_19747_amd as T
    _torch()
    n, d, cw, ca, cb, seed = case
    _say("case: inner_grad n=%d d=%s chis W=%d A=%d B=%d" % (n, d, cw, ca, cb))
    W = I.random_tt(n, d, cw, 100 + seed)
    A = I.random_tt(n, d, ca, 200 + seed)
    B = I.random_tt(n, d, cb, 300 + seed)
    v, dA, dB = T.inner_grad(W, A, B)
    vo, dAo, dBo = O.inner3_grad(W, A, B)
    assert abs(v - vo) <= TOL * max(abs(vo), 1e-300)
    assert _rel(_host(dA), dAo) <= TOL
    assert _rel(_host(dB), dBo) <= TOL
    v2, none_a, none_b = T.inner_grad(W, A, B, grads=False)
    assert none_a is None and none_b is None
    assert abs(v2 - vo) <= TOL * abs(vo)


def test_gpu_inner_grad_turbulence_1024_chi128():
    """Loss <W, A*B> with A, B the 1024^3 turbulence QTTs at chi = 128 (10
    sites, d = 8) and W a random train at chi = 32: gradients against the
    oracle; FP32 contractions at the mixed-precision bound."""
    import paper_2410_19747_amd as T
    torch = _torch()
    _say("case: inner_grad 1024^3 turbulence chi=128, W chi=32")
    qa = I.turbulence_qtt_device(1024, 101, [128], torch.device("cuda", 0))[128]
    qb = I.turbulence_qtt_device(1024, 102, [128], torch.device("cuda", 0))[128]
    torch.cuda.empty_cache()
    W = I.random_tt(10, 8, 32, 77)
    v, dA, dB = T.inner_grad(W, qa, qb)
    vo, dAo, dBo = O.inner3_grad(W, qa, qb)
    _say("  value %.6e oracle %.6e" % (v, vo))
    assert abs(v - vo) <= TOL * abs(vo)
    ea, eb = _rel(_host(dA), dAo), _rel(_host(dB), dBo)
    _say("  rel err dA %.2e dB %.2e" % (ea, eb))
    assert ea <= TOL and eb <= TOL
    v32, dA32, dB32 = T.inner_grad(W, qa, qb, contract_precision="f32")
    e32 = max(_rel(_host(dA32), dAo), _rel(_host(dB32), dBo))
    _say("  FP32 contractions: rel err %.2e" % e32)
    assert e32 <= 1e-6


def test_gpu_autograd_loss_matches_finite_differences():
    """loss = <W, TTM(A, B)> on the GPU with nothing truncated (chi_out =
    chi_A chi_B, eps = 0, so only singular values at the rounding-noise level
    are dropped): backward against the oracle gradient and against central
    differences (h = 1e-6) of the GPU loss along random directions."""
    import paper_2410_19747_amd as T
    torch = _torch()
    _say("case: autograd loss vs central differences")
    n, d = 6, 3
    W = I.random_tt(n, d, 4, 11)
    A = I.random_tt(n, d, 3, 12)
    B = I.random_tt(n, d, 2, 13)
    Ap, Bp = T.pack(A), T.pack(B)
    Ap.data.requires_grad_(True)
    Bp.data.requires_grad_(True)
    loss = T.ttm_inner_loss(W, Ap, Bp, 6, 0.0, chi_mid=0)
    loss.backward()
    vo, dAo, dBo = O.inner3_grad(W, A, B)
    # the forward product is exact to rounding: |<W, C - A*B>| <= ||W|| ||C - A*B||
    scale = np.linalg.norm(O.dense(W)) * np.linalg.norm(O.brute_force(A, B))
    assert abs(float(loss.detach()) - vo) <= 1e-13 * scale
    gA = T.PackedTT(Ap.data.grad.detach().clone(), Ap.phys, Ap.bonds, Ap.offsets)
    gB = T.PackedTT(Bp.data.grad.detach().clone(), Bp.phys, Bp.bonds, Bp.offsets)
    assert _rel(_host(gA), dAo) <= TOL and _rel(_host(gB), dBo) <= TOL
    rng = np.random.default_rng(3)
    h = 1e-6
    for trial in range(3):
        ea = torch.tensor(rng.standard_normal(Ap.data.numel()), device=Ap.data.device)
        eb = torch.tensor(rng.standard_normal(Bp.data.numel()), device=Bp.data.device)

        def loss_at(sign):
            a = T.PackedTT((Ap.data.detach() + sign * h * ea).contiguous(), Ap.phys, Ap.bonds, Ap.offsets)
            b = T.PackedTT((Bp.data.detach() + sign * h * eb).contiguous(), Bp.phys, Bp.bonds, Bp.offsets)
            return float(T.ttm_inner_loss(W, a, b, 6, 0.0, chi_mid=0))

        fd = (loss_at(1.0) - loss_at(-1.0)) / (2 * h)
        an = float((Ap.data.grad * ea).sum() + (Bp.data.grad * eb).sum())
        _say("  direction %d: fd %.10e analytic %.10e" % (trial, fd, an))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


def test_gpu_autograd_loss_truncated_product():
    """Where the TTM product truncates, <W, TTM(A, B)> is not <W, A*B>: the
    forward value is the truncated product's, and backward differentiates
    the truncated product (the reverse mode through its swaps), matching the
    oracle's reverse mode, not the gradient of <W, A*B>."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: autograd loss on a truncating product")
    W = I.random_tt(10, 2, 4, 21)
    A, B = I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)
    Ap, Bp = T.pack(A), T.pack(B)
    Ap.data.requires_grad_(True)
    Bp.data.requires_grad_(True)
    loss = T.ttm_inner_loss(W, Ap, Bp, 8, 1e-14)
    o = O.ttm(A, B, 8, 1e-14)
    ones = [np.ones((1, 2, 1))] * 10
    vo = O.inner3(W, o.cores, ones)
    assert abs(float(loss.detach()) - vo) <= 1e-12 * max(1.0, abs(vo))
    loss.backward()
    _, oA, oB = O.ttm_vjp(A, B, 8, 1e-14, O.inner3_grad(W, o.cores, ones)[1])
    gA = [x.detach().cpu().numpy() for x in T.PackedTT(Ap.data.grad, Ap.phys, Ap.bonds, Ap.offsets).cores()]
    gB = [x.detach().cpu().numpy() for x in T.PackedTT(Bp.data.grad, Bp.phys, Bp.bonds, Bp.offsets).cores()]
    assert _rel_cores(gA, oA) <= 1e-9 and _rel_cores(gB, oB) <= 1e-9
    # and it is not the gradient of the exact product's loss
    _, eA, _ = O.inner3_grad(W, A, B)
    assert _rel_cores(gA, eA) > 1e-6


def test_gpu_inner_grad_error_codes():
    import paper_2410_19747_amd as T
    _torch()
    _say("case: inner_grad error codes")
    W = I.random_tt(4, 2, 2, 1)
    A = I.random_tt(4, 3, 2, 2)
    with pytest.raises(T.TTMError) as ei:
        T.inner_grad(W, A, A)
    assert ei.value.code == T.TTM_ESHAPE
    bad = I.random_tt(4, 2, 2, 3)
    bad[1] = bad[1].copy()
    bad[1][0, 0, 0] = np.inf
    with pytest.raises(T.TTMError) as ei:
        T.inner_grad(W, bad, W)
    assert ei.value.code == T.TTM_ENONFINITE


def test_gpu_inner_grad_wide_w_and_fp32():
    """W with larger bonds than A and B, mixed physical dimensions; FP32
    contractions at the mixed-precision bound."""
    import paper_2410_19747_amd as T
    _torch()
    _say("case: inner_grad wide W, FP32")
    d = [4, 2, 5, 3, 4, 2, 3]
    W = I.random_tt(7, d, 40, 31)
    A = I.random_tt(7, d, 6, 32)
    B = I.random_tt(7, d, 9, 33)
    vo, dAo, dBo = O.inner3_grad(W, A, B)
    v, dA, dB = T.inner_grad(W, A, B)
    assert abs(v - vo) <= TOL * abs(vo)
    assert _rel(_host(dA), dAo) <= TOL and _rel(_host(dB), dBo) <= TOL
    v32, dA32, dB32 = T.inner_grad(W, A, B, contract_precision="f32")
    assert _rel(_host(dA32), dAo) <= 1e-6 and _rel(_host(dB32), dBo) <= 1e-6


@pytest.mark.parametrize("n", [1, 2, 7, 10])
def test_gpu_inner_grad_checkpointed_environments_bitwise(n):
    """Right environments kept only at checkpoints and recomputed segment by
    segment give bitwise the value and gradients of the stored form, for
    every stride (including strides that do not divide N)."""
    import paper_2410_19747_amd as T
    torch = _torch()
    _say("case: checkpointed environments, N=%d" % n)
    d = [2, 3, 2, 4, 2, 3, 2, 2, 3, 2][:n]

    def train(chi, seed):
        r = np.random.default_rng(seed)
        b = [1] + [int(min(chi, x)) for x in r.integers(2, chi + 1, n - 1)] + [1]
        return [r.standard_normal((b[i], d[i], b[i + 1])) for i in range(n)]

    W, A, B = train(4, 1 + n), train(7, 2 + n), train(6, 3 + n)
    v1, a1, b1 = T.inner_grad(W, A, B, env_stride=1)
    for stride in (0, 2, 3, 4, n + 5):
        v, a, b = T.inner_grad(W, A, B, env_stride=stride)
        assert v == v1, stride
        assert torch.equal(a.data, a1.data) and torch.equal(b.data, b1.data), stride
