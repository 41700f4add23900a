"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: brute force
on tiny grids, closed forms, the App. A toy model, exactness regimes,
invariants and error bounds.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import ttm_inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _r10():
    return I.random_tt(10, 2, 8, 1), I.random_tt(10, 2, 8, 2)


# ---------------------------------------------------------------- bond rule
def test_bond_rule_golden():
    g = json.load(open(os.path.join(GOLD, "bond_rule.json")))
    for case in g["cases"]:
        b = I.structural_bonds([case["d"]] * case["N"], case["chi"])
        if "bonds" in case:
            assert b == case["bonds"]
        else:
            assert max(b) == case["max_bond"]


# ---------------------------------------------------------------- rank rule
def test_rank_rule_strict_inequality():
    s = np.array([1.0, 0.5])              # s^2 = 1, 0.25; total 1.25
    assert O.rank_rule(s, 0.2, 0)[0] == 2     # 0.25 < 0.2*1.25 is false
    assert O.rank_rule(s, 0.21, 0)[0] == 1
    r, disc = O.rank_rule(s, 0.21, 0)
    assert disc == 0.25


def test_rank_rule_tail_and_caps():
    s = np.array([1.0, 1e-7, 1e-8])
    assert O.rank_rule(s, 1e-14, 0)[0] == 2   # tail_1 = 1.01e-14 is not < 1e-14
    assert O.rank_rule(s, 1.02e-14, 0)[0] == 1
    assert O.rank_rule(s, 1e-14, 1)[0] == 1   # cap
    # eps = 0 keeps every value whose square is > 0 in FP64
    assert O.rank_rule(np.array([1.0, 1e-100, 0.0]), 0.0, 0)[0] == 2
    assert O.rank_rule(np.array([1.0, 1e-200, 0.0]), 0.0, 0)[0] == 1  # square underflows
    assert O.rank_rule(np.zeros(4), 1e-12, 0)[0] == 1


def test_rank_rule_discard_count():
    s = np.array([1.0] + [1e-9] * 50)        # each tail value squares to 1e-18
    r, disc = O.rank_rule(s, 1e-16, 0)
    # 1e-16 * total ~ 1e-16 allows discarding 99 values of 1e-18: all 50 go.
    assert r == 1 and np.isclose(disc, 50e-18, rtol=1e-12)
    r, disc = O.rank_rule(s, 2.05e-17, 0)
    # 2.05e-17 * total admits a tail < 2.05e-17, i.e. at most 20 values.
    assert r == 31 and np.isclose(disc, 20e-18, rtol=1e-12)


# ---------------------------------------------------------------- brute force
def test_dense_matches_carriage_products():
    A = I.random_tt(4, 2, 4, 7)
    D = O.dense(A)
    for idx in np.ndindex(*D.shape):
        m = np.eye(1)
        for i, s in enumerate(idx):
            m = m @ A[i][:, s, :]
        assert np.isclose(D[idx], m[0, 0], rtol=1e-13, atol=1e-15)


def test_ttm_exact_vs_brute_force_config1():
    A, B = _r10()
    ref = O.brute_force(A, B)
    res = O.ttm(A, B, 64, 1e-28, chi_mid=0)
    assert O.rel_frob(res.cores, ref) <= 1e-12
    assert res.n_contract == 10 and res.n_swap == 45


def test_conventional_exact_vs_brute_force():
    A, B = _r10()
    ref = O.brute_force(A, B)
    assert O.rel_frob(O.conventional_exact(A, B, 64, 1e-28), ref) <= 1e-12


def test_kron_cores_exact_without_rounding():
    A, B = I.random_tt(5, 3, 4, 11), I.random_tt(5, 3, 4, 12)
    K = O.kron_cores(A, B)
    assert np.allclose(O.dense(K), O.brute_force(A, B), rtol=1e-13, atol=1e-15)


def test_variational_exact_when_chi_large():
    A, B = _r10()
    ref = O.brute_force(A, B)
    C, sweeps, _ = O.conventional_variational(A, B, 64, 1e-13, max_sweeps=6)
    assert O.rel_frob(C, ref) <= 1e-12


def test_ttm_mixed_dims_brute_force():
    phys = [3, 2, 4, 2, 3]
    A, B = I.random_tt(5, phys, 100, 21), I.random_tt(5, phys, 100, 22)
    ref = O.brute_force(A, B)
    res = O.ttm(A, B, 10 ** 6, 0.0, chi_mid=0)
    assert O.rel_frob(res.cores, ref) <= 1e-12


def test_ttm_single_site():
    A, B = I.random_tt(1, 5, 4, 1), I.random_tt(1, 5, 4, 2)
    res = O.ttm(A, B, 4, 1e-28)
    assert O.rel_frob(res.cores, O.brute_force(A, B)) <= 1e-14
    assert res.n_swap == 0 and res.n_contract == 1


# ---------------------------------------------------------------- identity, commutativity
def test_identity_with_all_ones():
    # The moving factor is the all-ones TT: its middle-block ranks are 1, so
    # every intermediate bond stays <= chi_A and any chi_mid >= chi_A is exact.
    A = I.random_tt(6, 8, 64, 5)
    one = I.ones_tt(6, 8)
    for cm in (64, 0):
        res = O.ttm(A, one, 64, 1e-28, chi_mid=cm)
        assert O.rel_frob(res.cores, A) <= 1e-12
        assert res.max_bond <= 64
    # With A moving, intermediates can need chi_A^2: exact only uncapped.
    A = I.random_tt(5, 4, 16, 6)
    one = I.ones_tt(5, 4)
    res = O.ttm(one, A, 16, 1e-28, chi_mid=0)
    assert O.rel_frob(res.cores, A) <= 1e-12


def test_commutativity_exact():
    A, B = _r10()
    c1 = O.ttm(A, B, 64, 1e-28, chi_mid=0).cores
    c2 = O.ttm(B, A, 64, 1e-28, chi_mid=0).cores
    assert O.rel_frob(c1, c2) <= 1e-12


def test_commutativity_truncated_within_bounds():
    A, B = _r10()
    r1 = O.ttm(A, B, 8, 1e-10)
    r2 = O.ttm(B, A, 8, 1e-10)
    nrm = O.tt_norm(r1.cores)
    diff = O.rel_frob(r1.cores, r2.cores) * O.tt_norm(r2.cores)
    assert diff <= r1.error_bound + r2.error_bound + 1e-12 * nrm


# ---------------------------------------------------------------- closed forms, N = 40
@pytest.mark.parametrize("case", ["exp", "sin2", "x2"])
def test_closed_forms_long_chain(case):
    n = 40
    if case == "exp":
        A, B = I.exp_qtt(n, 0.7), I.exp_qtt(n, -1.9)
        ref = I.exp_qtt(n, 0.7 - 1.9)
        bonds_expected = 1
    elif case == "sin2":
        A = B = I.sin_qtt(n, 3.0)
        # sin^2 = (1 - cos 2x)/2 : a rank-1 constant plus a rank-2 cosine
        c = I.cos_qtt(n, 6.0)
        c[0] = c[0] * -0.5
        ref = O.tt_sub(I.const_qtt(n, 0.5), [(-1.0 if i == 0 else 1.0) * x for i, x in enumerate(c)])
        bonds_expected = 3
    else:
        A = B = I.poly1_qtt(n, a=-0.3)
        ref = I.square_qtt(n, a=-0.3)
        bonds_expected = 3
    # fine-scale cuts carry singular values near dx ~ 1e-12 (weight ~1e-24):
    # keep them; rounding noise (weight ~1e-32) still goes.
    res = O.ttm(A, B, 16, 1e-28)
    assert O.rel_frob(res.cores, ref) <= 1e-12
    assert max(O.bonds_of(res.cores)) == bonds_expected


# ---------------------------------------------------------------- App. A toy model
def _entropy(lam):
    p = lam ** 2 / np.sum(lam ** 2)
    p = p[p > 0]
    return float(-np.sum(p * np.log2(p)))


def test_app_a_golden_first_carriages():
    g = json.load(open(os.path.join(GOLD, "app_a_toy.json")))
    T = I.app_a_toy_tt(5, seed=3)
    m = T[0].reshape(2, 2) @ T[1].reshape(2, 2)   # [sigma1, sigma2]
    assert np.allclose(m, np.array(g["two_bit_matrix"]), atol=1e-15)
    assert np.allclose(np.linalg.svd(m, compute_uv=False), g["two_bit_singular_values"], atol=1e-15)


def test_app_a_swap_spectrum_doubles():
    """Moving bit 2 to the end with the oracle's swap: every swap's spectrum is
    (1/sqrt2, 1/sqrt2) (x) lambda_init and the entropy grows by one bit."""
    n = 7
    T = I.app_a_toy_tt(n, d_rest=2, chi=4, seed=9)
    T = [c / (np.linalg.norm(O.dense(T)) ** (1.0 / n)) for c in T]
    D0 = O.dense(T)
    # centre to position 2 (0-based 1): right-orthogonalise, move once.
    cores = O.right_orthogonalize(T)
    q, r = np.linalg.qr(cores[0].reshape(-1, cores[0].shape[2]))
    cores[0] = q.reshape(1, 2, -1)
    cores[1] = np.tensordot(r, cores[1], axes=(1, 0))
    for k in range(1, n - 1):
        # bit 2 sits at position k; swap it with position k+1.
        x_new, p_new, rank, disc, s = O.swap(cores[k], cores[k + 1], 0.0, 0)
        cores[k], cores[k + 1] = x_new, p_new
        # bipartition after the swap: left = {s1, s3..s_{k+2}}, right = {s2, ...}
        left = D0.reshape(4, -1)  # placeholder shape guard
        m = D0.reshape([2] * n)
        lam_init = np.linalg.svd(m.reshape(2 ** (k + 2), -1), compute_uv=False)
        lam_init = lam_init[lam_init > 1e-14 * lam_init[0]]
        pred = np.sort(np.kron([2 ** -0.5, 2 ** -0.5], lam_init))[::-1]
        got = s[s > 1e-14 * s[0]]
        assert got.shape == pred.shape
        assert np.allclose(got, pred, rtol=1e-12, atol=1e-14)
        assert abs(_entropy(got) - (_entropy(lam_init) + 1.0)) <= 1e-10
        # centre to the next pair
        q, r = np.linalg.qr(cores[k].reshape(-1, cores[k].shape[2]))
        cores[k] = q.reshape(cores[k].shape[0], cores[k].shape[1], -1)
        cores[k + 1] = np.tensordot(r, cores[k + 1], axes=(1, 0))
    # the state is the original with bit 2 moved to the end
    perm = [0] + list(range(2, n)) + [1]
    assert np.allclose(O.dense(cores), D0.transpose(perm), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- invariants and bounds
def test_invariants_inner_products():
    A, B = _r10()
    res = O.ttm(A, B, 8, 1e-12)
    one = I.ones_tt(10, 2)
    err_abs = O.rel_frob(res.cores, O.brute_force(A, B)) * np.linalg.norm(O.brute_force(A, B))
    # <C, 1> = <A, B> up to ||1|| * ||C - A*B||
    assert abs(O.inner(res.cores, one) - O.inner(A, B)) <= np.sqrt(2 ** 10) * err_abs + 1e-15
    W = I.random_tt(10, 2, 4, 99)
    wn = np.linalg.norm(O.dense(W))
    assert abs(O.inner(W, res.cores) - O.inner3(W, A, B)) <= wn * err_abs * (1 + 1e-9) + 1e-15
    exact = O.ttm(A, B, 64, 1e-28, chi_mid=0)
    assert np.isclose(O.inner(W, exact.cores), O.inner3(W, A, B), rtol=1e-11)


def test_inner3_brute_force():
    W, A, B = I.random_tt(6, 2, 4, 1), I.random_tt(6, 2, 4, 2), I.random_tt(6, 2, 4, 3)
    assert np.isclose(O.inner3(W, A, B), np.sum(O.dense(W) * O.dense(A) * O.dense(B)), rtol=1e-12)


def test_counts_and_orthonormal_output():
    A, B = I.random_tt(8, 2, 8, 3), I.random_tt(8, 2, 8, 4)
    res = O.ttm(A, B, 12, 1e-12)
    assert res.n_contract == 8 and res.n_swap == 8 * 7 // 2
    for c in res.cores[:-1]:
        assert O.is_left_orthonormal(c, 1e-12)


def test_truncated_error_between_bounds():
    A, B = _r10()
    ref = O.brute_force(A, B)
    res = O.ttm(A, B, 8, 1e-14)
    err = O.rel_frob(res.cores, ref) * np.linalg.norm(ref)
    assert err <= res.error_bound * (1 + 1e-10) + 1e-15
    # Eckart-Young: any TT with bond <= 8 at cut k is at least this far away
    for k in range(1, 10):
        s = np.linalg.svd(ref.reshape(2 ** k, -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[8:] ** 2)) * (1 - 1e-10)


def test_truncated_error_between_bounds_uncapped_swaps():
    """chi_mid = 0 (reading R5): the swaps keep every value the rule of Eq.
    (eps) keeps, and only the final sweep (reading R6) caps the bonds."""
    A, B = _r10()
    ref = O.brute_force(A, B)
    res = O.ttm(A, B, 8, 1e-14, chi_mid=0)
    assert max(O.bonds_of(res.cores)) <= 8
    assert max(res.ranks[:45]) > 8
    err = O.rel_frob(res.cores, ref) * np.linalg.norm(ref)
    assert err <= res.error_bound * (1 + 1e-10) + 1e-15
    for k in range(1, 10):
        s = np.linalg.svd(ref.reshape(2 ** k, -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[8:] ** 2)) * (1 - 1e-10)


def _regauge(T, rng, spread=1.5):
    """The same tensor with G_k G_k^-1 inserted at every inner bond; each G_k
    is a random rotation times a scaling over 2*spread decades, times a
    rotation."""
    T = [np.array(c, copy=True) for c in T]
    for k in range(len(T) - 1):
        r = T[k].shape[2]
        q1, _ = np.linalg.qr(rng.standard_normal((r, r)))
        q2, _ = np.linalg.qr(rng.standard_normal((r, r)))
        g = q1 @ np.diag(np.logspace(-spread, spread, r)) @ q2
        T[k] = np.tensordot(T[k], g, axes=(2, 0))
        T[k + 1] = np.tensordot(np.linalg.inv(g), T[k + 1], axes=(1, 0))
    return T


def test_gauge_invariance_of_the_product():
    """The product depends on the tensors A and B, not on the gauge of their
    carriages: the inputs are brought to canonical form before the swaps
    (Sec. II.B, the gauge requirement), so a far-from-orthogonal change of
    gauge at every bond leaves the ranks and the truncated result unchanged
    up to rounding."""
    A, B = _r10()
    rng = np.random.default_rng(77)
    Ag, Bg = _regauge(A, rng), _regauge(B, rng)
    assert O.rel_frob(Ag, O.dense(A)) <= 1e-10 and O.rel_frob(Bg, O.dense(B)) <= 1e-10
    r1 = O.ttm(A, B, 8, 1e-14)
    r2 = O.ttm(Ag, Bg, 8, 1e-14)
    assert r2.ranks == r1.ranks
    assert O.rel_frob(r2.cores, r1.cores) <= 1e-9


def test_forced_ranks_reproduce_schedule():
    A, B = _r10()
    r1 = O.ttm(A, B, 8, 1e-10)
    r2 = O.ttm(A, B, 8, 0.5, forced_ranks=r1.ranks)
    assert r2.ranks == r1.ranks
    assert O.rel_frob(r2.cores, r1.cores) <= 1e-13
    # the weight a forced rank discards is the tail of Eq. (eps) at that rank
    assert np.allclose(r2.discards, r1.discards, rtol=1e-10, atol=0.0)


def test_tt_sub_and_rel_frob_modes():
    A, B = I.random_tt(6, 2, 4, 1), I.random_tt(6, 2, 4, 2)
    d = O.dense(O.tt_sub(A, B))
    assert np.allclose(d, O.dense(A) - O.dense(B), atol=1e-14)
    r_dense = O.rel_frob(A, B)
    r_tt = O.rel_frob(A, B, dense_limit=1)
    assert np.isclose(r_dense, r_tt, rtol=1e-12)


def test_tt_norm_and_orthogonalize():
    A = I.random_tt(7, 3, 9, 4)
    n0 = np.linalg.norm(O.dense(A))
    assert np.isclose(O.tt_norm(A), n0, rtol=1e-13)
    L = O.left_orthogonalize(A)
    R = O.right_orthogonalize(A)
    for c in L[:-1]:
        assert O.is_left_orthonormal(c)
    for c in R[1:]:
        assert O.is_right_orthonormal(c)
    assert O.rel_frob(L, A) <= 1e-13 and O.rel_frob(R, A) <= 1e-13


# ---------------------------------------------------------------- conventional variational
def test_variational_truncated_quality():
    A, B = _r10()
    ref = O.brute_force(A, B)
    C, sweeps, hist = O.conventional_variational(A, B, 8, 1e-13, max_sweeps=10)
    err = O.rel_frob(C, ref)
    svd_err = O.rel_frob(O.conventional_exact(A, B, 8, 0.0), ref)
    assert err <= svd_err * 1.05
    assert max(O.bonds_of(C)) <= 8
    for k in range(1, 10):
        s = np.linalg.svd(ref.reshape(2 ** k, -1), compute_uv=False)
        assert err * np.linalg.norm(ref) >= np.sqrt(np.sum(s[8:] ** 2)) * (1 - 1e-10)


def test_splitmix64_published_outputs():
    C = O.conventional
    outs = [C._splitmix64((0 + k * C._GAMMA) & C._MASK) for k in (1, 2, 3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = O.splitmix64_uniform(7, 1000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.1


# ---------------------------------------------------------------- turbulence inputs
def test_turbulence_generator_properties():
    u = I.turbulence_component(16, 201)
    assert u.shape == (16, 16, 16)
    assert np.isclose(np.sqrt(np.mean(u * u)), 1.0)
    uk = np.fft.fftn(u)
    assert abs(uk[0, 0, 0]) < 1e-9                     # k = 0 removed
    T = I.turbulence_qtt(16, 201, 0)
    assert O.bonds_of(T) == [1, 8, 64, 8, 1]
    assert np.allclose(O.dense(T), I.qtt_encode_3d(u), atol=1e-12)


def test_ttm_turbulence_t16_exact():
    A = I.turbulence_qtt(16, 201, 0)
    B = I.turbulence_qtt(16, 202, 0)
    ref = O.brute_force(A, B)
    res = O.ttm(A, B, 64, 1e-28, chi_mid=0)
    assert O.rel_frob(res.cores, ref) <= 1e-12


def test_device_turbulence_generator_on_host():
    """The device-side turbulence generator (run here with torch on the CPU):
    unit RMS, the interleaved bit order of qtt_encode_3d, and an exact TT at
    the structural bonds (a 16^3 field has bonds 8, 64, 8)."""
    torch = pytest.importorskip("torch")
    out = I.turbulence_qtt_device(16, 5, [64, 8], torch.device("cpu"))
    exact = O.dense(out[64])
    assert [c.shape for c in out[64]] == [(1, 8, 8), (8, 8, 64), (64, 8, 8), (8, 8, 1)]
    assert abs(np.sqrt(np.mean(exact ** 2)) - 1.0) < 1e-12
    # the chi = 8 train is the leading part of the same field
    assert O.rel_frob(out[8], exact) < 0.2
    # decoding the interleaved order gives a field whose spectrum has no k = 0 mode and
    # nothing beyond the cut-off |k| > n/2
    n = 16
    t = exact.reshape((2,) * 12)
    order = [0] * 12
    for s in range(4):
        for a in range(3):
            order[a * 4 + s] = 3 * s + a
    u = t.transpose(order).reshape(n, n, n)
    uk = np.fft.fftn(u)
    assert abs(uk[0, 0, 0]) < 1e-9 * np.abs(uk).max()
    k = np.fft.fftfreq(n, 1.0 / n)
    kk = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    assert np.abs(uk[kk > n / 2]).max() < 1e-9 * np.abs(uk).max()


# ---------------------------------------------------------------- flop model
def _frac(s):
    from fractions import Fraction
    return Fraction(s)


def _fixture_trains(sch):
    rng = np.random.default_rng(sch["seed"])
    d = sch["d"]

    def train(b):
        return [rng.standard_normal((b[i], d, b[i + 1])) for i in range(len(b) - 1)]

    return train(sch["A_bonds"]), train(sch["B_bonds"])


def test_model_flops_per_operation_golden():
    """model_flops against the per-operation formulas evaluated by hand in
    tests/golden/model_flops.json (both sides of the QR and SVD branches)."""
    g = json.load(open(os.path.join(GOLD, "model_flops.json")))
    for case in g["ops"]:
        op = tuple(case["op"])
        assert np.isclose(O.model_flops([op]), float(_frac(case["flops"])), rtol=1e-14, atol=0), op


def test_model_flops_schedule_golden():
    """The operation list the oracle records for a fixed three-site schedule
    (every bond written out in the fixture) and its flop total."""
    g = json.load(open(os.path.join(GOLD, "model_flops.json")))
    for sch in g["schedules"]:
        A, B = _fixture_trains(sch)
        res = O.ttm(A, B, sch["chi_out"], sch["eps"])
        want = [tuple(op) for op, _ in sch["ops"]]
        assert [tuple(int(x) if not isinstance(x, str) else x for x in op) for op in res.ops] == want
        assert res.ranks == sch["ranks"]
        assert sum(_frac(f) for _, f in sch["ops"]) == _frac(sch["total"])
        assert np.isclose(res.flops, float(_frac(sch["total"])), rtol=1e-14, atol=0)
        assert res.n_contract == 3 and res.n_swap == 3


# ---------------------------------------------------------------- schedule variants
def test_centre_right_gauge_exact_and_within_bounds():
    """The swap with the singular values on the right carriage and an LQ move
    of the centre (the gauge as Sec. II.B states it) gives the exact product
    where nothing is truncated, and in the truncated regime a result between
    the Eckart-Young bound and its own sum of discarded norms, with the
    ranks and the tensor of the default (mirrored) gauge: any position of the
    centre inside the pair gives the same truncation."""
    A, B = _r10()
    ref = O.brute_force(A, B)
    ex = O.ttm(A, B, 64, 1e-28, chi_mid=0, gauge="right")
    assert O.rel_frob(ex.cores, ref) <= 1e-12
    assert ex.n_qr == 2 * 9 + 36 + 45            # canonicalisation, gauge moves, one LQ per swap
    res = O.ttm(A, B, 8, 1e-14, gauge="right")
    err = O.rel_frob(res.cores, ref) * np.linalg.norm(ref)
    assert err <= res.error_bound * (1 + 1e-10) + 1e-15
    for k in range(1, 10):
        s = np.linalg.svd(ref.reshape(2 ** k, -1), compute_uv=False)
        assert err >= np.sqrt(np.sum(s[8:] ** 2)) * (1 - 1e-10)
    mirrored = O.ttm(A, B, 8, 1e-14)
    assert res.ranks == mirrored.ranks
    assert O.rel_frob(res.cores, mirrored.cores) <= 1e-12


def test_centre_right_swap_factors():
    """One swap in the stated gauge: the moved carriage comes out with
    orthonormal columns before the LQ move, the LQ factor L = R^T is lower
    triangular, and after the move the right carriage has orthonormal rows
    while the pair's product is the truncated unfolding."""
    rng = np.random.default_rng(5)
    P = rng.standard_normal((3, 2, 4))
    X = rng.standard_normal((4, 2, 5))
    x, p, r, disc, s, rf = O.swap_centre_right(P, X, 1e-14, 0)
    assert np.allclose(np.tril(rf.T), rf.T)
    pm = p.reshape(r, -1)
    assert np.abs(pm @ pm.T - np.eye(r)).max() < 1e-13
    theta = np.tensordot(P, X, axes=(2, 0)).transpose(0, 2, 1, 3).reshape(6, 10)
    assert np.allclose(x.reshape(6, r) @ pm, theta, atol=1e-13)
    # the L factor holds the singular values: |diag(L)| = s_r up to ordering of the QR
    assert np.isclose(np.linalg.norm(rf), np.linalg.norm(s[:r]), rtol=1e-13)


def test_move_smaller_factor():
    """Moving the train with the smaller bonds (A * B = B * A) gives the same
    exact product.  The bond a swap creates splits the moving train at two
    cuts and the fixed one at one, so exact intermediate bonds are at most
    chi_fixed chi_moving^2 (reading of the moving factor): with a chi-16 and
    a chi-2 train on 16 binary sites, moving the narrow one keeps every
    swap rank within 16 * 2 * 2 = 64, moving the wide one exceeds it."""
    wide = I.random_tt(16, 2, 16, 61)
    narrow = I.random_tt(16, 2, 2, 62)
    ref = O.brute_force(narrow, wide)
    moves_wide = O.ttm(narrow, wide, 4096, 1e-28, chi_mid=0)
    moves_narrow = O.ttm(narrow, wide, 4096, 1e-28, chi_mid=0, move_factor="smaller")
    assert O.rel_frob(moves_wide.cores, ref) <= 1e-12 and O.rel_frob(moves_narrow.cores, ref) <= 1e-12
    assert max(moves_narrow.ranks[:120]) <= 16 * 2 * 2
    assert max(moves_wide.ranks[:120]) > 16 * 2 * 2
    same = O.ttm(wide, narrow, 4096, 1e-28, chi_mid=0, move_factor="smaller")  # already in place
    assert same.ranks == moves_narrow.ranks
